// Adjoint of the fixed-grid two-layer step (reverse mode, hand-written), for
// states in which both layers are wet everywhere, plus the gauge misfit and the
// map from (eta1_0, B) to the initial state and their adjoints.
//
// The step is  Q+ = Y(X(G(Q), B), B):  G fills the wall ghost cells, X and Y are
// the x- and y-sweeps.  A sweep updates cell k of a line by
//   out_k = q_k - nu ((A+dQ_k - F_k) + (A-dQ_{k+1} + F_{k+1}))
// where edge k lies between cells k-1 and k and F is the limited correction
// flux.  Its adjoint is computed per edge: the lane of edge e solves it once,
// gathers the adjoint of its own waves from its fluctuations, its correction
// flux and the correction fluxes of its neighbours whose limiter looks at it
// (their waves and limiter terms come from the neighbouring lanes), and pushes
// it back through the edge solve onto its two cells; each cell then sums the
// contributions of its two edges with its own output adjoint, in the same
// kernel.  A fold pass maps ghost cells back through the walls.
#include "mlswe_kernels.hpp"
#include "mlswe_wave.hpp"

namespace mlswe {

namespace {

__device__ __forceinline__ long long aidx(const AdjView& V, int line, int k) {
  return V.base + (long long)line * V.lstride + (long long)k * V.kstride;
}

__device__ __forceinline__ long long lidx(const AdjView& V, int line, int k) {
  return V.lbase + (long long)line * V.llstride + (long long)k * V.lkstride;
}

// Cell seen along the line (normal / transverse momenta by orientation).
__device__ __forceinline__ CellX adj_cell(const AdjView& V, int line, int k) {
  const long long id = aidx(V, line, k);
  const double* q = V.q;
  const long long pl = V.plane;
  const int fm1 = V.orient ? 2 : 1, ft1 = V.orient ? 1 : 2;
  const int fm2 = V.orient ? 5 : 4, ft2 = V.orient ? 4 : 5;
  return load_cell(V.P, q[id], q[fm1 * pl + id], q[ft1 * pl + id], q[3 * pl + id], q[fm2 * pl + id],
                   q[ft2 * pl + id], V.B[id]);
}

// Adjoint of the outputs of cell k in line-local order (h1 m1 t1 h2 m2 t2); zero
// outside the updated cells 0..n-1.
__device__ __forceinline__ void adj_lam(const AdjView& V, int line, int k, double l[6]) {
  if (k < 0 || k >= V.n) {
#pragma unroll
    for (int c = 0; c < 6; ++c) l[c] = 0.0;
    return;
  }
  const long long id = lidx(V, line, k);
  const long long pl = V.lplane;
  const int fm1 = V.orient ? 2 : 1, ft1 = V.orient ? 1 : 2;
  const int fm2 = V.orient ? 5 : 4, ft2 = V.orient ? 4 : 5;
  l[0] = V.lam[id]; l[1] = V.lam[fm1 * pl + id]; l[2] = V.lam[ft1 * pl + id];
  l[3] = V.lam[3 * pl + id]; l[4] = V.lam[fm2 * pl + id]; l[5] = V.lam[ft2 * pl + id];
}

// Limiter quantities of wave p of an edge: whether its correction is active, K =
// sign(s)/2 (1 - nu |s|), phi(theta) and phi'(theta) along the branch taken.
struct LimP {
  bool on;
  double K, phi, dphi, th, dd, sg;
};

__device__ __forceinline__ LimP lim_of(const EdgeW& W, int p, double dd, double dot_left, double dot_right,
                                       double nu) {
  LimP L;
  L.on = false; L.K = 0.0; L.phi = 0.0; L.dphi = 0.0; L.th = 0.0; L.dd = dd; L.sg = 0.0;
  const double sv = W.s[p];
  if (slot_mode(W, p) != 0 || sv == 0.0 || dd == 0.0) return L;
  L.on = true;
  const double dn = sv > 0.0 ? dot_left : dot_right;
  const double th = dn / dd;
  L.th = th;
  const double a = 0.5 * (1.0 + th);
  const double b = 2.0 * th;
  double m1, d1;
  if (a < 2.0) { m1 = a; d1 = 0.5; } else { m1 = 2.0; d1 = 0.0; }
  double m, dm;
  if (m1 < b) { m = m1; dm = d1; } else { m = b; dm = 2.0; }
  if (0.0 > m) { L.phi = 0.0; L.dphi = 0.0; } else { L.phi = m; L.dphi = dm; }
  L.sg = sv > 0.0 ? 0.5 : -0.5;
  const double as = sv < 0.0 ? 0.0 - sv : sv;
  L.K = L.sg * (1.0 - nu * as);
  return L;
}

// Full components of wave p.
__device__ __forceinline__ void wvec(const EdgeW& W, int p, double z[6]) {
#pragma unroll
  for (int c = 0; c < 6; ++c) z[c] = wcomp(W, p, c);
}

// Adjoint of one CellX (all fields) accumulated into q-bar (h1 m1 t1 h2 m2 t2 B).
struct CellBar {
  double h1, m1, t1, h2, m2, t2, B, u1, w1, u2, w2, s1, s2, e1, e2;
};

__device__ __forceinline__ void zero_cb(CellBar& b) {
  b.h1 = b.m1 = b.t1 = b.h2 = b.m2 = b.t2 = b.B = 0.0;
  b.u1 = b.w1 = b.u2 = b.w2 = b.s1 = b.s2 = b.e1 = b.e2 = 0.0;
}

__device__ __forceinline__ void cell_reverse(const CellX& c, const CellBar& b, double out[7]) {
  double h1 = b.h1, h2 = b.h2, Bb = b.B;
  double e2 = b.e2 + b.e1;
  h1 += b.e1;
  Bb += e2;
  h2 += e2;
  // layer 1: u = m / h, w = t / h, s = sqrt(h)
  const double i1 = 1.0 / c.h1;
  double m1 = b.u1 * i1, t1 = b.w1 * i1;
  double inv1b = b.u1 * c.m1 + b.w1 * c.t1;
  h1 += -inv1b * i1 * i1 + b.s1 / (2.0 * c.s1);
  const double i2 = 1.0 / c.h2;
  double m2 = b.u2 * i2, t2 = b.w2 * i2;
  double inv2b = b.u2 * c.m2 + b.w2 * c.t2;
  h2 += -inv2b * i2 * i2 + b.s2 / (2.0 * c.s2);
  out[0] = h1; out[1] = m1 + b.m1; out[2] = t1 + b.t1;
  out[3] = h2; out[4] = m2 + b.m2; out[5] = t2 + b.t2; out[6] = Bb;
}

// Solves M^T y = r (4 x 4) by elimination with partial pivoting.  Rows are
// exchanged by compare-and-swap against the pivot row with fixed indices (the
// largest entry of the column ends up in the pivot row), so the matrix stays in
// registers.
__device__ __forceinline__ void solve4T(const double R[4][4], const double r[4], double y[4]) {
  double a[4][5];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j) a[i][j] = R[j][i];
    a[i][4] = r[i];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
#pragma unroll
    for (int i = k + 1; i < 4; ++i) {
      const bool sw = fabs(a[i][k]) > fabs(a[k][k]);
#pragma unroll
      for (int j = 0; j < 5; ++j) {
        const double t = a[k][j];
        a[k][j] = sw ? a[i][j] : t;
        a[i][j] = sw ? t : a[i][j];
      }
    }
    const double ik = 1.0 / a[k][k];
#pragma unroll
    for (int i = k + 1; i < 4; ++i) {
      const double f = a[i][k] * ik;
#pragma unroll
      for (int j = k; j < 5; ++j) a[i][j] -= f * a[k][j];
    }
  }
#pragma unroll
  for (int i = 3; i >= 0; --i) {
    double s = a[i][4];
#pragma unroll
    for (int j = i + 1; j < 4; ++j) s -= a[i][j] * y[j];
    y[i] = s / a[i][i];
  }
}

// Reverse of the coupled (all wet) edge solve: given the adjoint of the factored
// waves (Abar, Cbar, sbar[6], v1bar, v2bar, z4bar, z5bar), accumulates the
// adjoints of the two cells' fields.
__device__ __forceinline__ void riemann_reverse(const PhysParams& P, const CellX& L, const CellX& R,
                                                const double Ab[4], const double Cb[4], const double sb_in[6],
                                                double v1b, double v2b, double z4b, double z5b, CellBar& Lb,
                                                CellBar& Rb) {
  // ---- forward recomputation (same expressions as the solve)
  const double hb1 = 0.5 * (L.h1 + R.h1);
  const double hb2 = 0.5 * (L.h2 + R.h2);
  const double d1 = 1.0 / (L.s1 + R.s1);
  const double nu1 = FMA(L.s1, L.u1, R.s1 * R.u1), nw1 = FMA(L.s1, L.w1, R.s1 * R.w1);
  const double ub1 = nu1 * d1, wb1 = nw1 * d1;
  const double d2 = 1.0 / (L.s2 + R.s2);
  const double nu2 = FMA(L.s2, L.u2, R.s2 * R.u2), nw2 = FMA(L.s2, L.w2, R.s2 * R.w2);
  const double ub2 = nu2 * d2, wb2 = nw2 * d2;
  const double del1 = R.m1 - L.m1;
  const double del2 = FMA(P.g * hb1, R.e1 - L.e1, FMA(R.m1, R.u1, -(L.m1 * L.u1)));
  const double del3 = R.m2 - L.m2;
  const double J4 = FMA(P.r, R.h1 - L.h1, R.e2 - L.e2);
  const double del4 = FMA(P.g * hb2, J4, FMA(R.m2, R.u2, -(L.m2 * L.u2)));
  const double H = hb1 + hb2;
  const double iH = 1.0 / H;
  const double ce = __builtin_sqrt(P.g * H);
  const double du = ub1 - ub2;
  double kap = FMA(-((du * du) * iH), P.inv_gp, 1.0);
  bool clamped = false;
  if (kap < P.kmin) { kap = P.kmin; clamped = true; }
  const double ci = __builtin_sqrt((((P.gp * hb1) * hb2) * iH) * kap);
  const double U = FMA(hb1, ub1, hb2 * ub2) * iH;
  const double Uc = FMA(hb1, ub2, hb2 * ub1) * iH;
  double s[4] = {U - ce, Uc - ci, Uc + ci, U + ce};
  const double gh1 = P.g * hb1;
  const double igh = 1.0 / gh1;
  double a[4], al[4];
#pragma unroll
  for (int p = 0; p < 4; ++p) { a[p] = s[p] - ub1; al[p] = FMA(a[p], a[p], -gh1) * igh; }
  double Rm[4][4];
#pragma unroll
  for (int p = 0; p < 4; ++p) { Rm[0][p] = 1.0; Rm[1][p] = s[p]; Rm[2][p] = al[p]; Rm[3][p] = al[p] * s[p]; }
  // beta from the forward solve, recomputed through the same elimination
  double be[4];
  {
    double m11 = s[1] - s[0], m12 = s[2] - s[0], m13 = s[3] - s[0];
    double m21 = al[1] - al[0], m22 = al[2] - al[0], m23 = al[3] - al[0];
    double q0 = al[0] * s[0];
    double m31 = FMA(al[1], s[1], -q0), m32 = FMA(al[2], s[2], -q0), m33 = FMA(al[3], s[3], -q0);
    double b0 = del1, b1 = FMA(-s[0], del1, del2), b2 = FMA(-al[0], del1, del3), b3 = FMA(-q0, del1, del4);
    double ip1 = 1.0 / m11;
    double f2 = m21 * ip1, f3 = m31 * ip1;
    m22 = FMA(-f2, m12, m22); m23 = FMA(-f2, m13, m23); b2 = FMA(-f2, b1, b2);
    m32 = FMA(-f3, m12, m32); m33 = FMA(-f3, m13, m33); b3 = FMA(-f3, b1, b3);
    double ip2 = 1.0 / m22;
    double f4 = m32 * ip2;
    m33 = FMA(-f4, m23, m33); b3 = FMA(-f4, b2, b3);
    be[3] = b3 / m33;
    be[2] = FMA(-m23, be[3], b2) * ip2;
    be[1] = FMA(-m13, be[3], FMA(-m12, be[2], b1)) * ip1;
    be[0] = ((b0 - be[1]) - be[2]) - be[3];
  }
  // ---- reverse
  double sb[4], alb[4], beb[4];
  double ub1b = sb_in[4], ub2b = sb_in[5];
  double wb1b = v1b - z4b * del1, wb2b = v2b - z5b * del3;  // z4 = dt1 - wb1 del1, z5 likewise
  double dt1b = z4b, dt2b = z5b;
  double del1b = -z4b * wb1, del3b = -z5b * wb2, del2b = 0.0, del4b = 0.0;
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    sb[p] = sb_in[p];
    beb[p] = Ab[p] + Cb[p] * al[p];
    alb[p] = Cb[p] * be[p];
  }
  double y[4];
  solve4T(Rm, beb, y);
  del1b += y[0]; del2b += y[1]; del3b += y[2]; del4b += y[3];
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    sb[p] += -y[1] * be[p] - y[3] * be[p] * al[p];
    alb[p] += -y[2] * be[p] - y[3] * be[p] * s[p];
  }
  double gh1b = 0.0;
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const double ab = alb[p] * 2.0 * a[p] * igh;
    gh1b += alb[p] * (-igh) * (1.0 + al[p]);
    sb[p] += ab;
    ub1b -= ab;
  }
  double hb1b = P.g * gh1b, hb2b = 0.0;
  const double Ub = sb[0] + sb[3], ceb = sb[3] - sb[0];
  const double Ucb = sb[1] + sb[2], cib = sb[2] - sb[1];
  const double Xb = cib / (2.0 * ci);
  double iHb = 0.0;
  hb1b += Xb * P.gp * hb2 * iH * kap;
  hb2b += Xb * P.gp * hb1 * iH * kap;
  iHb += Xb * P.gp * hb1 * hb2 * kap;
  const double kapb = Xb * P.gp * hb1 * hb2 * iH;
  if (!clamped) {
    const double dub = kapb * (-2.0 * du * iH * P.inv_gp);
    iHb += kapb * (-du * du * P.inv_gp);
    ub1b += dub;
    ub2b -= dub;
  }
  double Hb = ceb * P.g / (2.0 * ce);
  hb1b += Ub * ub1 * iH + Ucb * ub2 * iH;
  ub1b += Ub * hb1 * iH + Ucb * hb2 * iH;
  hb2b += Ub * ub2 * iH + Ucb * ub1 * iH;
  ub2b += Ub * hb2 * iH + Ucb * hb1 * iH;
  iHb += Ub * (hb1 * ub1 + hb2 * ub2) + Ucb * (hb1 * ub2 + hb2 * ub1);
  Hb += -iHb * iH * iH;
  hb1b += Hb;
  hb2b += Hb;
  // transverse fluxes
  Rb.t1 += dt1b * R.u1; Rb.u1 += dt1b * R.t1; Lb.t1 -= dt1b * L.u1; Lb.u1 -= dt1b * L.t1;
  Rb.t2 += dt2b * R.u2; Rb.u2 += dt2b * R.t2; Lb.t2 -= dt2b * L.u2; Lb.u2 -= dt2b * L.t2;
  // jumps
  Rb.m1 += del1b; Lb.m1 -= del1b;
  Rb.m1 += del2b * R.u1; Rb.u1 += del2b * R.m1; Lb.m1 -= del2b * L.u1; Lb.u1 -= del2b * L.m1;
  hb1b += del2b * P.g * (R.e1 - L.e1);
  Rb.e1 += del2b * P.g * hb1; Lb.e1 -= del2b * P.g * hb1;
  Rb.m2 += del3b; Lb.m2 -= del3b;
  Rb.m2 += del4b * R.u2; Rb.u2 += del4b * R.m2; Lb.m2 -= del4b * L.u2; Lb.u2 -= del4b * L.m2;
  hb2b += del4b * P.g * J4;
  Rb.e2 += del4b * P.g * hb2; Lb.e2 -= del4b * P.g * hb2;
  Rb.h1 += del4b * P.g * hb2 * P.r; Lb.h1 -= del4b * P.g * hb2 * P.r;
  // Roe averages
  {
    const double nu1b = ub1b * d1, nw1b = wb1b * d1;
    const double d1b = ub1b * nu1 + wb1b * nw1;
    Lb.s1 += nu1b * L.u1 + nw1b * L.w1; Lb.u1 += nu1b * L.s1; Lb.w1 += nw1b * L.s1;
    Rb.s1 += nu1b * R.u1 + nw1b * R.w1; Rb.u1 += nu1b * R.s1; Rb.w1 += nw1b * R.s1;
    Lb.s1 += -d1b * d1 * d1; Rb.s1 += -d1b * d1 * d1;
    const double nu2b = ub2b * d2, nw2b = wb2b * d2;
    const double d2b = ub2b * nu2 + wb2b * nw2;
    Lb.s2 += nu2b * L.u2 + nw2b * L.w2; Lb.u2 += nu2b * L.s2; Lb.w2 += nw2b * L.s2;
    Rb.s2 += nu2b * R.u2 + nw2b * R.w2; Rb.u2 += nu2b * R.s2; Rb.w2 += nw2b * R.s2;
    Lb.s2 += -d2b * d2 * d2; Rb.s2 += -d2b * d2 * d2;
  }
  Lb.h1 += 0.5 * hb1b; Rb.h1 += 0.5 * hb1b;
  Lb.h2 += 0.5 * hb2b; Rb.h2 += 0.5 * hb2b;
}

__device__ __forceinline__ bool all_wet(const CellX& c) { return c.wet1 && c.wet2; }

// Adjoint of an edge's waves in factored form (strengths A, C, speeds s,
// transverse velocities v1, v2, shear jumps z4, z5).  add_zbar adds the
// adjoint X of the six components of wave p, Z = (A, A s, A v1, C, C s, C v2)
// (shear waves: the single component z4 or z5), pulled back to the factors.
struct WaveBar {
  double Ab[4], Cb[4], sb[6], v1b, v2b, z4b, z5b;
};
__device__ __forceinline__ void add_zbar(WaveBar& B, const EdgeW& W, int p, const double X[6]) {
  if (p == 4) { B.z4b += X[2]; return; }
  if (p == 5) { B.z5b += X[5]; return; }
  B.Ab[p] += X[0] + X[1] * W.s[p] + X[2] * W.v1;
  B.Cb[p] += X[3] + X[4] * W.s[p] + X[5] * W.v2;
  B.sb[p] += X[1] * W.A[p] + X[4] * W.C[p];
  B.v1b += X[2] * W.A[p];
  B.v2b += X[5] * W.C[p];
}

}  // namespace

// Edge adjoints, one solve and one limiter evaluation per edge.  A wave takes
// 64 consecutive edges of one line, e = 61 s - 3 + L on lane L of segment s;
// the waves of edges e - 1 and e + 1 come from lanes L - 1 and L + 1 by
// whole-wave rotations.  Lanes 1..62 own their edges (own: in range and not
// an end lane), lanes 0 and 63 lend their waves and limiter terms.  The term by which a neighbour's limiter
// looks at edge e is the neighbour's own coefficient dnu (the adjoint of its
// ratio's numerator) times the neighbour's wave, so each lane evaluates only
// its own limiter and passes dnu on.  Per edge the contributions are: the
// edge's fluctuations and correction flux, the correction fluxes of the
// neighbours whose limiter reads it, and (through its own limiter ratio) the
// upwind neighbour's wave; they are pushed back through the edge solve onto
// its two cells (ol: left cell, orr: right cell, line-local field order).
// Src gives the line's cells and output adjoints by position along the line.
template <class Src>
__device__ __forceinline__ void adj_edge_lane(const Src& src, const PhysParams& P, double nu, int n, int e,
                                              bool exists, int* status, bool own, double ol[7], double orr[7]) {
  const bool hasPrev = e >= 0, hasNext = e <= n;
  EdgeW W;
  int okc;
  {
    CellX Cm1, C0;
    if (exists) {
      Cm1 = src.cell(e - 1);
      C0 = src.cell(e);
    } else {
      Cm1 = load_cell(P, 1.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0);  // a still, flat edge, lent to no owned lane
      C0 = Cm1;
    }
    okc = all_wet(Cm1) && all_wet(C0);
    riemann(P, Cm1, C0, W);
  }
  const int okm = shup_i(okc), okp = shdn_i(okc);
  const bool ok = okc && (!hasPrev || okm) && (!hasNext || okp);
  double dotp[6], dotm[6];
  {
    const EdgeW Wp = shdn_edge(W);
#pragma unroll
    for (int p = 0; p < 6; ++p) dotp[p] = hasNext ? wdot(W, Wp, p) : 0.0;
  }
#pragma unroll
  for (int p = 0; p < 6; ++p) {
    dotm[p] = shup(dotp[p]);
    if (!hasPrev) dotm[p] = 0.0;
  }
  WaveBar Bw;
#pragma unroll
  for (int p = 0; p < 4; ++p) { Bw.Ab[p] = 0.0; Bw.Cb[p] = 0.0; }
#pragma unroll
  for (int p = 0; p < 6; ++p) Bw.sb[p] = 0.0;
  Bw.v1b = 0.0; Bw.v2b = 0.0; Bw.z4b = 0.0; Bw.z5b = 0.0;
  // own fluctuations and correction flux (edges 0..n feed the updates; the
  // end lanes too, their dnu serves the owned lanes beside them)
  double dnu[6];
#pragma unroll
  for (int p = 0; p < 6; ++p) dnu[p] = 0.0;
  if (exists && e >= 0 && e <= n) {
    double l0[6], lm1[6];
    src.lam(e, l0);
    src.lam(e - 1, lm1);
    double Fb[6], amb[6], apb[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      Fb[c] = nu * (l0[c] - lm1[c]);
      amb[c] = -nu * lm1[c];
      apb[c] = -nu * l0[c];
    }
#pragma unroll
    for (int p = 0; p < 6; ++p) {
      const double sv = W.s[p];
      const int md = slot_mode(W, p);
      const double wm = md == 2 ? 0.0 : (sv < 0.0 ? 1.0 : (sv == 0.0 ? 0.5 : 0.0));
      const double wp = md == 1 ? 0.0 : (sv > 0.0 ? 1.0 : (sv == 0.0 ? 0.5 : 0.0));
      double z[6];
      wvec(W, p, z);
      LimP Lm = lim_of(W, p, wdot(W, W, p), dotm[p], dotp[p], nu);
      double coefb = 0.0, X[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        X[c] = wm * amb[c] + wp * apb[c] + Lm.K * Lm.phi * Fb[c];
        coefb += Fb[c] * z[c];
      }
      add_zbar(Bw, W, p, X);
      if (Lm.on) {
        const double sgn = sv > 0.0 ? 1.0 : -1.0;
        Bw.sb[p] += coefb * Lm.phi * Lm.sg * (-nu * sgn);
        const double thb = coefb * Lm.K * Lm.dphi;
        const double ddb = -thb * Lm.th / Lm.dd;
        dnu[p] = thb / Lm.dd;
#pragma unroll
        for (int c = 0; c < 6; ++c) X[c] = 2.0 * ddb * z[c];
        add_zbar(Bw, W, p, X);
      }
    }
  }
  {
    // edge e+1: its right-going waves' limiter reads edge e; edge e's
    // left-going waves' limiter reads edge e+1
    const EdgeW Wp = shdn_edge(W);
#pragma unroll
    for (int p = 0; p < 6; ++p) {
      const double dn = shdn(dnu[p]);
      double X[6], u[6];
      if (hasNext && Wp.s[p] > 0.0 && dn != 0.0) {
        wvec(Wp, p, u);
#pragma unroll
        for (int c = 0; c < 6; ++c) X[c] = dn * u[c];
        add_zbar(Bw, W, p, X);
      }
      if (!(W.s[p] > 0.0) && dnu[p] != 0.0) {
        wvec(Wp, p, u);
#pragma unroll
        for (int c = 0; c < 6; ++c) X[c] = dnu[p] * u[c];
        add_zbar(Bw, W, p, X);
      }
    }
  }
  {
    // edge e-1: its left-going waves' limiter reads edge e; edge e's
    // right-going waves' limiter reads edge e-1
    const EdgeW Wm = shup_edge(W);
#pragma unroll
    for (int p = 0; p < 6; ++p) {
      const double dn = shup(dnu[p]);
      double X[6], u[6];
      if (hasPrev && Wm.s[p] < 0.0 && dn != 0.0) {
        wvec(Wm, p, u);
#pragma unroll
        for (int c = 0; c < 6; ++c) X[c] = dn * u[c];
        add_zbar(Bw, W, p, X);
      }
      if (W.s[p] > 0.0 && dnu[p] != 0.0) {
        wvec(Wm, p, u);
#pragma unroll
        for (int c = 0; c < 6; ++c) X[c] = dnu[p] * u[c];
        add_zbar(Bw, W, p, X);
      }
    }
  }
#pragma unroll
  for (int f = 0; f < 7; ++f) { ol[f] = 0.0; orr[f] = 0.0; }
  if (own && !ok) atomicOr(status, 1);
  if (own && ok) {
    // the two cells again (not held through the limiter passes)
    const CellX Cm1 = src.cell_again(e - 1), C0 = src.cell_again(e);
    CellBar Lb, Rb;
    zero_cb(Lb);
    zero_cb(Rb);
    riemann_reverse(P, Cm1, C0, Bw.Ab, Bw.Cb, Bw.sb, Bw.v1b, Bw.v2b, Bw.z4b, Bw.z5b, Lb, Rb);
    cell_reverse(Cm1, Lb, ol);
    cell_reverse(C0, Rb, orr);
  }
}

// A line's cells and output adjoints straight from the level arrays.
struct LineSrc {
  const AdjView* V;
  int line;
  __device__ CellX cell(int k) const { return adj_cell(*V, line, k); }
  __device__ CellX cell_again(int k) const {
    // an address the compiler cannot match with the first loads
    long long d = 0;
    __asm__ volatile("" : "+v"(d));
    AdjView Vr = *V;
    Vr.base += d;
    return adj_cell(Vr, line, k);
  }
  __device__ void lam(int k, double l[6]) const { adj_lam(*V, line, k, l); }
};

// Cells and output adjoints of one column of a tile staged in LDS: rows k0 ..
// k0 + 64 of TCOLS columns, 13 fields in line-local order (h1 m1 t1 h2 m2 t2
// B, then the six output adjoints; zero outside the updated cells).
constexpr int TCOLS = 4, TPAD = 5, TROWS = 65;
struct TileSrc {
  const double* t;  // [13][TROWS][TPAD]
  int k0, col, n;
  PhysParams P;
  __device__ double at(int f, int k) const { return t[(f * TROWS + (k - k0)) * TPAD + col]; }
  __device__ CellX cell(int k) const {
    return load_cell(P, at(0, k), at(1, k), at(2, k), at(3, k), at(4, k), at(5, k), at(6, k));
  }
  __device__ CellX cell_again(int k) const { return cell(k); }
  __device__ void lam(int k, double l[6]) const {
#pragma unroll
    for (int c = 0; c < 6; ++c) l[c] = at(7 + c, k);
  }
};

// Cell k of a line sums its own output adjoint (cells 0..n-1), what edge k
// gives its right cell and what edge k + 1 gives its left cell: lane L holds
// edge k = e and receives edge k + 1 from lane L + 1.  Lanes 1..61 write cells
// k = 61 s - 2 + L - 1, so the segments' cells tile -2 .. n+1 once.
__device__ __forceinline__ void cell_sums(const double ol[7], const double orr[7], const double l0[6], bool hasR,
                                          bool hasL, double out[7]) {
#pragma unroll
  for (int f = 0; f < 7; ++f) {
    const double fromL = shdn(ol[f]);  // edge k + 1, lane L + 1
    double v = f < 6 ? l0[f] : 0.0;
    if (hasR) v += orr[f];
    if (hasL) v += fromL;
    out[f] = v;
  }
}

// Rows (the x-sweep's lines): one wave per 61 cells of a row, cells read by
// each lane from memory (consecutive lanes, consecutive cells).  Writes the
// adjoint of the wall-filled state (lam_in, level layout) and the row sweep's
// bathymetry adjoint.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_adj_edges_row(AdjView V,
                                                                                                double* lam_in,
                                                                                                double* Bbar) {
  const int lane = (int)(threadIdx.x & 63);
  const long long wv = (long long)blockIdx.x * 4 + (long long)(threadIdx.x >> 6);
  const int n = V.n;
  const int nseg = (n + 4 + 60) / 61;
  if (wv >= (long long)nseg * V.nlines) return;  // whole waves
  const int line = (int)(wv / nseg), seg = (int)(wv % nseg);
  const int e = 61 * seg - 3 + lane;
  const bool exists = e >= -1 && e <= n + 1;
  const bool own = exists && lane >= 1 && lane <= 62;
  const LineSrc src{&V, line};
  double ol[7], orr[7];
  adj_edge_lane(src, V.P, V.nu, n, e, exists, V.status, own, ol, orr);
  double l0[6];
  adj_lam(V, line, e, l0);  // zero outside the updated cells
  double out[7];
  cell_sums(ol, orr, l0, e >= -1, e + 1 <= n + 1, out);
  if (lane < 1 || lane > 61 || e < -2 || e > n + 1) return;
  const long long id = aidx(V, line, e);
  const long long pl = V.plane;
#pragma unroll
  for (int f = 0; f < 6; ++f) lam_in[f * pl + id] = out[f];
  Bbar[id] = out[6];
}

// Field plane of line-local field f (h1 m1 t1 h2 m2 t2) along a column, where
// the normal momenta are hv: planes 0 2 1 3 5 4.
__device__ __forceinline__ int col_plane(int f) { return (f == 1 || f == 4) ? f + 1 : (f == 2 || f == 5) ? f - 1 : f; }

// Columns (the y-sweep's lines): a block takes TCOLS adjacent columns and 61
// cells of each, one wave per column.  The block first copies the tile's cells
// and output adjoints (rows of TCOLS consecutive doubles) into LDS, each wave
// then reads its column there by lane, and the cell sums go back through LDS
// so that the stores, too, run along rows.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_adj_edges_col(AdjView V,
                                                                                                double* lam_in,
                                                                                                double* Bbar) {
  __shared__ double tile[13 * TROWS * TPAD];
  const int lane = (int)(threadIdx.x & 63), w = (int)(threadIdx.x >> 6);
  const int n = V.n;
  const int nseg = (n + 4 + 60) / 61;
  const int ncb = (V.nlines + TCOLS - 1) / TCOLS;
  // blocks reach the eight XCDs in turn: XCD x takes the x-th band of the
  // tiles, so the column groups that share cache lines meet in one L2
  const int per = (int)(gridDim.x >> 3);
  const int g = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  const int cb = g % ncb, seg = g / ncb;
  if (seg >= nseg) return;  // whole blocks
  const int i0 = TCOLS * cb, k0 = 61 * seg - 4;
  const long long pl = V.plane;
  // all of a thread's loads are issued, from clamped in-bounds addresses,
  // before its first LDS write; the values past the data are chosen after
  constexpr int NIN = 13 * TROWS * TCOLS, KIN = (NIN + 255) / 256;
  double vin[KIN];
#pragma unroll
  for (int u = 0; u < KIN; ++u) {
    const int x = (int)threadIdx.x + 256 * u;
    const int f = x < NIN ? x / (TROWS * TCOLS) : 12, r = (x / TCOLS) % TROWS, c = x % TCOLS;
    const int k = k0 + r, i = i0 + c;
    const int ii = i < V.nlines ? i : V.nlines - 1;
    double v;
    if (f < 7) {
      const int kk = k < -2 ? -2 : (k > n + 1 ? n + 1 : k);
      v = (f < 6 ? V.q + col_plane(f) * pl : V.B)[aidx(V, ii, kk)];
    } else {
      const int kk = k < 0 ? 0 : (k > n - 1 ? n - 1 : k);
      v = V.lam[col_plane(f - 7) * V.lplane + lidx(V, ii, kk)];
    }
    // cells exist on rows -2 .. n+1 (outside them a still, flat cell); the
    // output adjoints are zero outside the updated cells 0 .. n-1
    const bool in = f < 7 ? (k >= -2 && k <= n + 1) : (k >= 0 && k < n);
    const double dflt = (f == 0 || f == 3) ? 1.0 : 0.0;
    vin[u] = in ? v : dflt;
  }
#pragma unroll
  for (int u = 0; u < KIN; ++u) {
    const int x = (int)threadIdx.x + 256 * u;
    if (x < NIN) tile[(x / (TROWS * TCOLS) * TROWS + (x / TCOLS) % TROWS) * TPAD + x % TCOLS] = vin[u];
  }
  __syncthreads();
  const int line = i0 + w;
  const int e = 61 * seg - 3 + lane;
  const bool exists = line < V.nlines && e >= -1 && e <= n + 1;
  const bool own = exists && lane >= 1 && lane <= 62;
  const TileSrc src{tile, k0, w, n, V.P};
  double ol[7], orr[7];
  adj_edge_lane(src, V.P, V.nu, n, e, exists, V.status, own, ol, orr);
  double l0[6];
  src.lam(e, l0);
  double out[7];
  cell_sums(ol, orr, l0, e >= -1, e + 1 <= n + 1, out);
  __syncthreads();  // the tile's inputs are read; its space takes the sums
  // cell k = e = k0 + 2 + r (r = lane - 1) at [f][r][w]
  if (lane >= 1 && lane <= 61) {
#pragma unroll
    for (int f = 0; f < 7; ++f) tile[(f * TROWS + lane - 1) * TPAD + w] = out[f];
  }
  __syncthreads();
  constexpr int NOUT = 7 * 61 * TCOLS, KOUT = (NOUT + 255) / 256;
#pragma unroll
  for (int u = 0; u < KOUT; ++u) {
    const int x = (int)threadIdx.x + 256 * u;
    const int f = x / (61 * TCOLS), r = (x / TCOLS) % 61, c = x % TCOLS;
    const int k = k0 + 2 + r, i = i0 + c;
    if (x >= NOUT || i >= V.nlines || k < -2 || k > n + 1) continue;
    const double v = tile[(f * TROWS + r) * TPAD + c];
    if (f < 6) lam_in[col_plane(f) * pl + aidx(V, i, k)] = v;
    else Bbar[aidx(V, i, k)] = v;
  }
}

// Interior cell (i, j) collects the adjoint of itself and of every frame cell
// that mirrors it (normal momenta negated), for the state and the bathymetry.
__global__ __launch_bounds__(256) void k_adj_fold(AdjFold F) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)F.nx * F.ny) return;
  const int i = (int)(t % F.nx), j = (int)(t / F.nx);
  int xs[3], ys[3], nxs = 0, nys = 0;
  xs[nxs++] = i;
  ys[nys++] = j;
  if (i <= 1) xs[nxs++] = -1 - i;
  if (i >= F.nx - 2) xs[nxs++] = 2 * F.nx - 1 - i;
  if (j <= 1) ys[nys++] = -1 - j;
  if (j >= F.ny - 2) ys[nys++] = 2 * F.ny - 1 - j;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  double bacc = 0.0;
  for (int a = 0; a < nxs; ++a)
    for (int b = 0; b < nys; ++b) {
      const int ii = xs[a], jj = ys[b];
      const bool fx = a > 0, fy = b > 0;
      const long long id = (long long)(jj + 2) * F.pitch + (ii + XOFF);
#pragma unroll
      for (int f = 0; f < 6; ++f) {
        double v = F.lam_g[f * F.plane + id];
        if ((fx && (f == 1 || f == 4)) || (fy && (f == 2 || f == 5))) v = 0.0 - v;
        acc[f] += v;
      }
      bacc += F.Bbx[id] + F.Bby[id];
    }
  const long long o = (long long)j * F.nx + i;
  const long long pu = (long long)F.nx * F.ny;
#pragma unroll
  for (int f = 0; f < 6; ++f) F.lam_out[f * pu + o] = acc[f];
  F.Bbar[o] += bacc;
}

// Initial state from the parameters: h2 = eta2_0 - B, h1 = eta1_0 - eta2_0, at
// rest, thin layers dry.  q is [6][ny][nx]; B is the level array.
__global__ __launch_bounds__(256) void k_param_map(ParamMap M) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long pu = (long long)M.nx * M.ny;
  if (t >= pu) return;
  const int i = (int)(t % M.nx), j = (int)(t / M.nx);
  const double B = M.B[(long long)(j + 2) * M.pitch + (i + XOFF)];
  double h2 = M.eta2 - B;
  double h1 = M.eta1[t] - M.eta2;
  if (h2 < M.hdry) h2 = 0.0;
  if (h1 < M.hdry) h1 = 0.0;
  M.q[t] = h1; M.q[pu + t] = 0.0; M.q[2 * pu + t] = 0.0;
  M.q[3 * pu + t] = h2; M.q[4 * pu + t] = 0.0; M.q[5 * pu + t] = 0.0;
}

__global__ __launch_bounds__(256) void k_param_map_adj(ParamMap M, const double* __restrict__ lam0,
                                                       double* eta1_bar, double* B_bar) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long pu = (long long)M.nx * M.ny;
  if (t >= pu) return;
  const int i = (int)(t % M.nx), j = (int)(t / M.nx);
  const double B = M.B[(long long)(j + 2) * M.pitch + (i + XOFF)];
  const double h2 = M.eta2 - B;
  const double h1 = M.eta1[t] - M.eta2;
  eta1_bar[t] = h1 < M.hdry ? 0.0 : lam0[t];
  B_bar[t] += h2 < M.hdry ? 0.0 : 0.0 - lam0[3 * pu + t];
}

// Gauge misfit sum over the gn x gn region at (i0, j0) of (eta1 - target)^2,
// eta1 = (B + h2) + h1, added to *loss (one block, fixed reduction order); with
// lam / B_bar given, adds its gradient 2 (eta1 - target) to the h1, h2 and B
// adjoints.
__global__ __launch_bounds__(256) void k_gauge(Gauge Gd) {
  __shared__ double part[256];
  const int n = Gd.gn * Gd.gn;
  double s = 0.0;
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    const int i = Gd.i0 + k % Gd.gn, j = Gd.j0 + k / Gd.gn;
    const long long id = Gd.qlevel ? (long long)(j + 2) * Gd.pitch + (i + XOFF) : (long long)j * Gd.nx + i;
    const double B = Gd.B[(long long)(j + 2) * Gd.pitch + (i + XOFF)];
    const double eta1 = (B + Gd.q[3 * Gd.qplane + id]) + Gd.q[id];
    const double d = eta1 - Gd.target[k];
    s += d * d;
    if (Gd.lam) {
      const long long o = (long long)j * Gd.nx + i;
      const long long pu = (long long)Gd.nx * Gd.ny;
      Gd.lam[o] += 2.0 * d;
      Gd.lam[3 * pu + o] += 2.0 * d;
      if (Gd.B_bar) Gd.B_bar[o] += 2.0 * d;
    }
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0 && Gd.loss) *Gd.loss += part[0];
}

__global__ void k_set_dt(LevelCtl* ctl, double dt) { ctl->dt = dt; }

}  // namespace mlswe
