// Device-side arithmetic of the two-layer shallow-water step and of the
// multilayer refine operator, for gfx950.
//
// Expression order is fixed and written out term by term so that the result is
// reproducible across launches and tile shapes (compiled without floating-point
// contraction; FP64 division and square root are IEEE correctly rounded).
//
// Paper passages: surfaces eta1 = B + h2 + h1, eta2 = B + h2 and the effective
// bathymetry B-hat = B + h2 (Sec. 2.1, Eqs. 4-9); wet ordering of the layers
// (Sec. 2.1); minmod-limited linear interpolant of the surfaces, bottom layer
// first (Sec. 2.1, Eq. 10 and the paragraph after it).  The solver is not written
// in the paper (Sec. 1 cites it): a layered f-wave solve is used at each edge.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// Two builds of the device arithmetic share this source: the exact one (IEEE
// division and square root, no contraction: reproducible bit for bit) and a
// fast one (MLSWE_FAST: Newton-refined hardware reciprocal and reciprocal
// square root, about one ulp, compiled with contraction), kept apart by an
// inline namespace.
#ifndef MLSWE_NS_VARIANT
#define MLSWE_NS_VARIANT exact
#endif

namespace mlswe {

struct PhysParams {
  double g, r, hdry, kmin, gp, inv_gp;
};

inline namespace MLSWE_NS_VARIANT {

#ifdef MLSWE_FAST
// The hardware seeds overflow for magnitudes below about 2^-1022: reciprocals
// through mrcp are taken only of depths, sums of root depths, speed differences
// and pivots, all of normal size; a quotient whose divisor can be a tiny dot
// product (the limiter's ratio) goes through mdiv, which divides exactly there.
// A square root may be taken of zero (the speed of a dry side in the one-layer
// bound), where the reciprocal-root seed is infinite, so zero passes unchanged.
__device__ __forceinline__ double mrcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}
__device__ __forceinline__ double msqrt(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double s = x * y, h = 0.5 * y;
  const double r = __builtin_fma(-s, h, 0.5);
  s = __builtin_fma(s, r, s);
  h = __builtin_fma(h, r, h);
  const double d = __builtin_fma(-s, s, x);
  const double v = __builtin_fma(d, h, s);
  return x == 0.0 ? x : v;
}
__device__ __forceinline__ double mdiv(double a, double b) {
  if (__builtin_expect(__builtin_fabs(b) < 0x1p-1000, 0)) return a / b;
  return a * mrcp(b);
}
#define MRCP(x) mrcp(x)
#define MDIV(a, b) mdiv(a, b)
#define MSQRT(x) msqrt(x)
#else
// Correctly rounded reciprocal and square root without the operand scaling of
// the general sequences.  The hardware's divide and square-root sequences scale
// operands near the ends of the exponent range and patch zeros, infinities and
// NaNs afterwards; between 2^-767 and 2^1000 that scaling is the identity and
// the patch never applies, so the refinement steps below (two Newton steps on
// the reciprocal seed, then one correction by the exact residual, after
// Markstein; Goldschmidt's coupled iteration for the root, then two residual
// corrections) give the correctly rounded result, bit for bit that of 1/x and
// sqrt(x).  Operands outside that range take the general operation.
__device__ __forceinline__ bool plain_range(double a) { return a >= 0x1p-767 && a <= 0x1p+1000; }
__device__ __forceinline__ double rcp_cr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(e, r, r);
  if (__builtin_expect(!plain_range(__builtin_fabs(x)), 0)) r = 1.0 / x;
  return r;
}
__device__ __forceinline__ double sqrt_cr(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double s = x * y, h = y * 0.5;
  const double r = __builtin_fma(-h, s, 0.5);
  s = __builtin_fma(s, r, s);
  double d = __builtin_fma(-s, s, x);
  h = __builtin_fma(h, r, h);
  s = __builtin_fma(d, h, s);
  d = __builtin_fma(-s, s, x);
  s = __builtin_fma(d, h, s);
  if (__builtin_expect(!plain_range(x), 0)) s = __builtin_sqrt(x);
  return s;
}
#define MRCP(x) rcp_cr(x)
#define MDIV(a, b) ((a) / (b))
#define MSQRT(x) sqrt_cr(x)
#endif

#define FMA(a, b, c) __builtin_fma(a, b, c)

// Per-sweep view of one cell.  m: normal momentum, t: transverse momentum.
struct CellX {
  double h1, m1, t1, h2, m2, t2, B;
  double u1, w1, u2, w2, s1, s2;
  double e1, e2;
  bool wet1, wet2;
};

__device__ __forceinline__ CellX load_cell(const PhysParams& P, double h1, double m1, double t1,
                                           double h2, double m2, double t2, double B) {
  CellX c;
  c.h1 = h1; c.m1 = m1; c.t1 = t1; c.h2 = h2; c.m2 = m2; c.t2 = t2; c.B = B;
  c.wet1 = h1 >= P.hdry;
  c.wet2 = h2 >= P.hdry;
  if (c.wet1) {
    double inv = MRCP(h1);
    c.u1 = m1 * inv; c.w1 = t1 * inv; c.s1 = MSQRT(h1);
  } else {
    c.u1 = 0.0; c.w1 = 0.0; c.s1 = 0.0;
  }
  if (c.wet2) {
    double inv = MRCP(h2);
    c.u2 = m2 * inv; c.w2 = t2 * inv; c.s2 = MSQRT(h2);
  } else {
    c.u2 = 0.0; c.w2 = 0.0; c.s2 = 0.0;
  }
  c.e2 = B + h2;
  c.e1 = c.e2 + h1;
  return c;
}

// Waves of one edge in factored form.  Slot p = 0..3 carries the vector
// (A, A s, A v1, C, C s, C v2) with A, C its layer-1 / layer-2 strengths and
// v1, v2 the edge's transverse velocities; slots 4 and 5 (shear of layers 1 and
// 2) carry a single component z4 (component 2) or z5 (component 5).
// mode: 0 both fluctuations, 1 only into the left cell, 2 only into the right.
struct EdgeW {
  double s[6];
  double A[4], C[4];
  double v1, v2, z4, z5;
  int mode1, mode2;  // mode of the layer-1 slots (0,3,4) and layer-2 slots (1,2,5)
};

__device__ __forceinline__ int slot_mode(const EdgeW& W, int p) {
  return (p == 0 || p == 3 || p == 4) ? W.mode1 : W.mode2;
}

// Component c of wave p (the same products as the factored form defines).
__device__ __forceinline__ double wcomp(const EdgeW& W, int p, int c) {
  if (p == 4) return c == 2 ? W.z4 : 0.0;
  if (p == 5) return c == 5 ? W.z5 : 0.0;
  switch (c) {
    case 0: return W.A[p];
    case 1: return W.A[p] * W.s[p];
    case 2: return W.A[p] * W.v1;
    case 3: return W.C[p];
    case 4: return W.C[p] * W.s[p];
    default: return W.C[p] * W.v2;
  }
}

__device__ __forceinline__ double dmin(double a, double b) { return a < b ? a : b; }
__device__ __forceinline__ double dmax(double a, double b) { return a > b ? a : b; }

// One layer alone over its effective bottom (some layer dry on some side).
// J: jump of the layer's pressure surface across the edge.
__device__ __forceinline__ void layer_alone(const PhysParams& P, int layer, bool wetL, bool wetR,
                                            bool wallIfDryR, bool wallIfDryL, const CellX& L,
                                            const CellX& R, double J, EdgeW& W) {
  if (!wetL && !wetR) return;
  double hL, mL, tL, uL, wL, qL, hR, mR, tR, uR, wR, qR;
  if (layer == 1) {
    hL = L.h1; mL = L.m1; tL = L.t1; uL = L.u1; wL = L.w1; qL = L.s1;
    hR = R.h1; mR = R.m1; tR = R.t1; uR = R.u1; wR = R.w1; qR = R.s1;
  } else {
    hL = L.h2; mL = L.m2; tL = L.t2; uL = L.u2; wL = L.w2; qL = L.s2;
    hR = R.h2; mR = R.m2; tR = R.t2; uR = R.u2; wR = R.w2; qR = R.s2;
  }
  int mode = 0;
  if (wetL && !wetR) {
    double etaL = (layer == 1) ? L.e1 : L.e2;
    double botR = (layer == 1) ? R.e2 : R.B;
    if (wallIfDryR || etaL <= botR) {
      hR = hL; mR = 0.0 - mL; tR = tL; uR = 0.0 - uL; wR = wL; qR = qL;
      J = 0.0;
      mode = 1;
    } else {
      hR = 0.0; mR = 0.0; tR = 0.0; uR = 0.0; wR = 0.0; qR = 0.0;
    }
  } else if (!wetL && wetR) {
    double etaR = (layer == 1) ? R.e1 : R.e2;
    double botL = (layer == 1) ? L.e2 : L.B;
    if (wallIfDryL || etaR <= botL) {
      hL = hR; mL = 0.0 - mR; tL = tR; uL = 0.0 - uR; wL = wR; qL = qR;
      J = 0.0;
      mode = 2;
    } else {
      hL = 0.0; mL = 0.0; tL = 0.0; uL = 0.0; wL = 0.0; qL = 0.0;
    }
  }
  const bool effL = hL > 0.0, effR = hR > 0.0;
  double hb = 0.5 * (hL + hR);
  double d = MRCP(qL + qR);
  double uh = (qL * uL + qR * uR) * d;
  double wh = (qL * wL + qR * wR) * d;
  double dA = mR - mL;
  double dB = (mR * uR - mL * uL) + (P.g * hb) * J;
  double dT = tR * uR - tL * uL;
  double ch = MSQRT(P.g * hb);
  double sa, sb;
  if (effL) sa = dmin(uL - MSQRT(P.g * hL), uh - ch);
  else      sa = uR - 2.0 * MSQRT(P.g * hR);
  if (effR) sb = dmax(uR + MSQRT(P.g * hR), uh + ch);
  else      sb = uL + 2.0 * MSQRT(P.g * hL);
  double isd = MRCP(sb - sa);
  double bA = (sb * dA - dB) * isd;
  double bB = (dB - sa * dA) * isd;
  if (layer == 1) {
    W.s[0] = sa; W.A[0] = bA;
    W.s[3] = sb; W.A[3] = bB;
    W.v1 = wh;
    W.s[4] = uh; W.z4 = dT - wh * dA;
    W.mode1 = mode;
  } else {
    W.s[1] = sa; W.C[1] = bA;
    W.s[2] = sb; W.C[2] = bB;
    W.v2 = wh;
    W.s[5] = uh; W.z5 = dT - wh * dA;
    W.mode2 = mode;
  }
}

// Layered f-wave solve at one edge.  Returns true if the internal-wave factor
// was clamped.
__device__ __forceinline__ bool riemann(const PhysParams& P, const CellX& L, const CellX& R,
                                        EdgeW& W) {
#pragma unroll
  for (int p = 0; p < 6; ++p) W.s[p] = 0.0;
#pragma unroll
  for (int p = 0; p < 4; ++p) { W.A[p] = 0.0; W.C[p] = 0.0; }
  W.v1 = 0.0; W.v2 = 0.0; W.z4 = 0.0; W.z5 = 0.0;
  W.mode1 = 0; W.mode2 = 0;
  bool clamped = false;
  if (L.wet1 && L.wet2 && R.wet1 && R.wet2) {
    double hb1 = 0.5 * (L.h1 + R.h1);
    double hb2 = 0.5 * (L.h2 + R.h2);
    double d1 = MRCP(L.s1 + R.s1);
    double ub1 = FMA(L.s1, L.u1, R.s1 * R.u1) * d1;
    double wb1 = FMA(L.s1, L.w1, R.s1 * R.w1) * d1;
    double d2 = MRCP(L.s2 + R.s2);
    double ub2 = FMA(L.s2, L.u2, R.s2 * R.u2) * d2;
    double wb2 = FMA(L.s2, L.w2, R.s2 * R.w2) * d2;
    double del1 = R.m1 - L.m1;
    double del2 = FMA(P.g * hb1, R.e1 - L.e1, FMA(R.m1, R.u1, -(L.m1 * L.u1)));
    double del3 = R.m2 - L.m2;
    double J2 = FMA(P.r, R.h1 - L.h1, R.e2 - L.e2);
    double del4 = FMA(P.g * hb2, J2, FMA(R.m2, R.u2, -(L.m2 * L.u2)));
    double dt1 = FMA(R.t1, R.u1, -(L.t1 * L.u1));
    double dt2 = FMA(R.t2, R.u2, -(L.t2 * L.u2));
    double H = hb1 + hb2;
    double iH = MRCP(H);
    double U = FMA(hb1, ub1, hb2 * ub2) * iH;
    double Uc = FMA(hb1, ub2, hb2 * ub1) * iH;
    double ce = MSQRT(P.g * H);
    double du = ub1 - ub2;
    double kap = FMA(-((du * du) * iH), P.inv_gp, 1.0);
    if (kap < P.kmin) { kap = P.kmin; clamped = true; }
    double ci = MSQRT((((P.gp * hb1) * hb2) * iH) * kap);
    double s0 = U - ce, s1 = Uc - ci, s2 = Uc + ci, s3 = U + ce;
    double gh1 = P.g * hb1;
    double igh = MRCP(gh1);
    double a;
    a = s0 - ub1; double al0 = FMA(a, a, -gh1) * igh;
    a = s1 - ub1; double al1 = FMA(a, a, -gh1) * igh;
    a = s2 - ub1; double al2 = FMA(a, a, -gh1) * igh;
    a = s3 - ub1; double al3 = FMA(a, a, -gh1) * igh;
    double m11 = s1 - s0, m12 = s2 - s0, m13 = s3 - s0;
    double m21 = al1 - al0, m22 = al2 - al0, m23 = al3 - al0;
    double q0 = al0 * s0;
    double m31 = FMA(al1, s1, -q0), m32 = FMA(al2, s2, -q0), m33 = FMA(al3, s3, -q0);
    double b0 = del1;
    double b1 = FMA(-s0, del1, del2);
    double b2 = FMA(-al0, del1, del3);
    double b3 = FMA(-q0, del1, del4);
    double ip1 = MRCP(m11);
    double f2 = m21 * ip1, f3 = m31 * ip1;
    m22 = FMA(-f2, m12, m22); m23 = FMA(-f2, m13, m23); b2 = FMA(-f2, b1, b2);
    m32 = FMA(-f3, m12, m32); m33 = FMA(-f3, m13, m33); b3 = FMA(-f3, b1, b3);
    double ip2 = MRCP(m22);
    double f4 = m32 * ip2;
    m33 = FMA(-f4, m23, m33); b3 = FMA(-f4, b2, b3);
    double be3 = MDIV(b3, m33);
    double be2 = FMA(-m23, be3, b2) * ip2;
    double be1 = FMA(-m13, be3, FMA(-m12, be2, b1)) * ip1;
    double be0 = ((b0 - be1) - be2) - be3;
    W.s[0] = s0; W.s[1] = s1; W.s[2] = s2; W.s[3] = s3;
    W.A[0] = be0; W.A[1] = be1; W.A[2] = be2; W.A[3] = be3;
    W.C[0] = be0 * al0; W.C[1] = be1 * al1; W.C[2] = be2 * al2; W.C[3] = be3 * al3;
    W.v1 = wb1; W.v2 = wb2;
    W.s[4] = ub1; W.z4 = FMA(-wb1, del1, dt1);
    W.s[5] = ub2; W.z5 = FMA(-wb2, del3, dt2);
    return clamped;
  }
  double J1 = R.e1 - L.e1;
  double J2 = (R.e2 - L.e2) + P.r * (R.h1 - L.h1);
  layer_alone(P, 1, L.wet1, R.wet1, false, false, L, R, J1, W);
  layer_alone(P, 2, L.wet2, R.wet2, !R.wet1, !L.wet1, L, R, J2, W);
  return false;
}

// A-dQ (into the left cell) and A+dQ (into the right); a tie at s = 0 is split.
__device__ __forceinline__ void fluctuations(const EdgeW& W, double am[6], double ap[6]) {
#pragma unroll
  for (int c = 0; c < 6; ++c) { am[c] = 0.0; ap[c] = 0.0; }
#pragma unroll
  for (int p = 0; p < 6; ++p) {
    const double sv = W.s[p];
    const int md = slot_mode(W, p);
    // Weight 1, 1/2 (tie) or 0 of the wave in each fluctuation, applied by a
    // fused multiply-add: with weight 1 it is the plain sum, with 1/2 the
    // product is exact, and a zero weight adds a zero term, which leaves a sum
    // unchanged (the sums start at +0 and in round-to-nearest a result is -0
    // only if both terms are, so none ever holds -0).  The same result as
    // skipping the wave, without a branch.
    const double wl = (md != 2 && sv < 0.0) ? 1.0 : ((md != 2 && sv == 0.0) ? 0.5 : 0.0);
    const double wr = (md != 1 && sv > 0.0) ? 1.0 : ((md != 1 && sv == 0.0) ? 0.5 : 0.0);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      if ((p == 4 && c != 2) || (p == 5 && c != 5)) continue;  // the shear waves' zero components
      const double z = wcomp(W, p, c);
      am[c] = __builtin_fma(wl, z, am[c]);
      ap[c] = __builtin_fma(wr, z, ap[c]);
    }
  }
}

// Dot product over the six components of wave p of two edges.
__device__ __forceinline__ double wdot(const EdgeW& U, const EdgeW& W, int p) {
  if (p == 4) return U.z4 * W.z4;
  if (p == 5) return U.z5 * W.z5;
  double acc = wcomp(U, p, 0) * wcomp(W, p, 0);
#pragma unroll
  for (int c = 1; c < 6; ++c) acc = __builtin_fma(wcomp(U, p, c), wcomp(W, p, c), acc);
  return acc;
}

// The hardware min/max may return either zero for a (-0, +0) pair, where the
// compare-and-select form returns a fixed one.  The sign of a zero limiter
// value is immaterial: it only scales terms added to correction sums that start
// at +0 (which never hold -0), and adding a zero of either sign leaves them
// unchanged.  For finite ratios the two forms agree in every other case.
__device__ __forceinline__ double mc_limiter(double th) {
  double a = 0.5 * (1.0 + th);
  double b = 2.0 * th;
  double m = __builtin_fmin(__builtin_fmin(a, 2.0), b);
  return __builtin_fmax(0.0, m);
}

// Correction-flux coefficient of wave p at an edge from its own self dot
// product dd and its dot products with the edges on either side.
__device__ __forceinline__ double corr_coef(const EdgeW& W, int p, double dd, double dot_left,
                                            double dot_right, double nu) {
  const double sv = W.s[p];
  // evaluated on every lane (a safe divisor where the wave takes no correction)
  // and selected, so the wave needs no branch
  const bool on = slot_mode(W, p) == 0 && sv != 0.0 && dd != 0.0;
  double dn = sv > 0.0 ? dot_left : dot_right;
  double th = MDIV(dn, on ? dd : 1.0);
  double phi = mc_limiter(th);
  double sg = sv > 0.0 ? 0.5 : -0.5;
  // |s| by the sign-clearing operand modifier: it differs from the select
  // form (-s when s < 0, else s) only at s = -0 (where 1 - nu |s| is 1 either
  // way) and in a NaN's sign bit
  double as = __builtin_fabs(sv);
  return on ? (sg * (1.0 - nu * as)) * phi : 0.0;
}

// F[c] = sum_p coef_p Z_p[c] in slot order.
__device__ __forceinline__ void correction_flux(const EdgeW& W, const double coef[6], double F[6]) {
#pragma unroll
  for (int c = 0; c < 6; ++c) F[c] = 0.0;
#pragma unroll
  for (int p = 0; p < 6; ++p) {
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      if ((p == 4 && c != 2) || (p == 5 && c != 5)) continue;
      F[c] = __builtin_fma(coef[p], wcomp(W, p, c), F[c]);
    }
  }
}

struct FixCount {
  int nclip, repair;
  double clip1, clip2;
  int nonfinite;  // a cell left the fix-up with a non-finite value
};

// Dry-state fix-up: clip thin layers (bottom first), restore the wet ordering.
// CHECK: also note a non-finite value in the wave's cells (the x-sweep, which
// every step passes through, carries the check).
template <bool CHECK = false>
__device__ __forceinline__ void fixup(const PhysParams& P, double q[6], bool count, FixCount& K) {
  if (q[3] < P.hdry) {
    if (count && q[3] != 0.0) { K.nclip++; K.clip2 += q[3]; }
    q[3] = 0.0; q[4] = 0.0; q[5] = 0.0;
  }
  if (q[0] < P.hdry) {
    if (count && q[0] != 0.0) { K.nclip++; K.clip1 += q[0]; }
    q[0] = 0.0; q[1] = 0.0; q[2] = 0.0;
  }
  if (q[0] == 0.0 && q[3] > 0.0) {
    if (count) { K.repair++; K.clip2 += q[3]; }
    q[3] = 0.0; q[4] = 0.0; q[5] = 0.0;
  }
  if (CHECK) {
    // NaN or infinity in a depth of some lane of the wave (kept wave-wide).  A
    // non-finite momentum reaches the depths through the fluxes of the next
    // sweep along it (the normal momentum is the depth's flux).
    K.nonfinite |= __builtin_amdgcn_ballot_w64(!__builtin_isfinite(q[0] + q[3])) != 0ull ? 1 : 0;
  }
}

// ------------------------------------------------------------------ refine
__device__ __forceinline__ double minmod(double a, double b) {
  if (a > 0.0 && b > 0.0) return a < b ? a : b;
  if (a < 0.0 && b < 0.0) return a > b ? a : b;
  return 0.0;
}

// Coarse stencil values: [k][0..5] state, [k][6] bathymetry; k = centre, x-, x+,
// y-, y+.  Fills the fine cell (offsets fa, fb) from them, surfaces of the
// bottom layer first, depths through the fine bathymetry and B-hat = B + h2,
// then the wet ordering.  Returns true if a wet-order repair happened.
__device__ __forceinline__ bool refine_from_stencil(const PhysParams& P, const double (*q)[7], bool inx,
                                                    bool iny, double fa, double fb, double Bf,
                                                    double out[6]) {
  bool sxok[3], syok[3];
  double etaf[3];
#pragma unroll
  for (int m = 2; m >= 1; --m) {
    const int hf = (m == 2) ? 3 : 0;
    sxok[m] = inx && (q[1][hf] >= P.hdry) && (q[0][hf] >= P.hdry) && (q[2][hf] >= P.hdry);
    syok[m] = iny && (q[3][hf] >= P.hdry) && (q[0][hf] >= P.hdry) && (q[4][hf] >= P.hdry);
    double ek[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) ek[k] = (m == 2) ? q[k][6] + q[k][3] : (q[k][6] + q[k][3]) + q[k][0];
    double e = ek[0];
    double sx = sxok[m] ? minmod(e - ek[1], ek[2] - e) : 0.0;
    double sy = syok[m] ? minmod(e - ek[3], ek[4] - e) : 0.0;
    etaf[m] = (e + sx * fa) + sy * fb;
  }
  double h2 = (q[0][3] >= P.hdry) ? etaf[2] - Bf : 0.0;
  if (h2 < P.hdry) h2 = 0.0;
  double Bhat = Bf + h2;
  double h1 = (q[0][0] >= P.hdry) ? etaf[1] - Bhat : 0.0;
  if (h1 < P.hdry) h1 = 0.0;
  bool rep = false;
  if (h1 == 0.0 && h2 > 0.0) { h2 = 0.0; rep = true; }
  auto mom = [&](int f, int m) {
    double v = q[0][f];
    double sx = sxok[m] ? minmod(v - q[1][f], q[2][f] - v) : 0.0;
    double sy = syok[m] ? minmod(v - q[3][f], q[4][f] - v) : 0.0;
    return (v + sx * fa) + sy * fb;
  };
  out[0] = h1;
  out[1] = h1 > 0.0 ? mom(1, 1) : 0.0;
  out[2] = h1 > 0.0 ? mom(2, 1) : 0.0;
  out[3] = h2;
  out[4] = h2 > 0.0 ? mom(4, 2) : 0.0;
  out[5] = h2 > 0.0 ? mom(5, 2) : 0.0;
  return rep;
}

}  // inline namespace
}  // namespace mlswe
