// Reference oracle for the two-layer shallow-water hot path -- TEST INFRASTRUCTURE ONLY.
//
// Plain, slow, single-threaded FP64 implementation of what the GPU path computes.
// It shares no code with the HIP library and is called only from the tests, the
// smoke check and the CPU-baseline leg of the benchmark.  Nothing in the product
// path may link against it.
//
// The paper (Schwarzschild & Mandli, "An Implementation of Adaptive Mesh
// Refinement for Shallow Water Equations") fixes the refine operator (Sec. 2.1,
// Eqs. 3-10), the coarsen operator (Sec. 2.2, Eq. 11) and the level/ratio
// structure (Sec. 2, Eqs. 1-2).  It does not write the governing equations or the
// Riemann solver (Sec. 1 only cites the multilayer GeoClaw solver); the readings
// used for those parts are stated where they are applied below (edge solve,
// wet/dry edges, limiter, update grouping, fix-up).
//
// Every scalar routine is templated on the number type T so that the same code
// runs in double (parity) and in a forward-mode dual number (adjoint pin).
#pragma once
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace ora {

// ---------------------------------------------------------------- numbers
struct Dual {
  double v, d;
  Dual() : v(0), d(0) {}
  Dual(double x) : v(x), d(0) {}
  Dual(double x, double dx) : v(x), d(dx) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
  double q = a.v / b.v;
  return Dual(q, (a.d - q * b.d) / b.v);
}
inline Dual sqrt(Dual a) {
  double s = std::sqrt(a.v);
  return Dual(s, a.d / (2.0 * s));
}
inline double val(double x) { return x; }
inline double val(const Dual& x) { return x.v; }
inline double sqrt_(double x) { return std::sqrt(x); }
inline Dual sqrt_(const Dual& x) { return sqrt(x); }
// Fused multiply-add a*b + c with a single rounding (IEEE 754 fusedMultiplyAdd).
inline double fma_(double a, double b, double c) { return std::fma(a, b, c); }
inline Dual fma_(const Dual& a, const Dual& b, const Dual& c) {
  return Dual(std::fma(a.v, b.v, c.v), a.d * b.v + a.v * b.d + c.d);
}
template <class T> inline T absv(const T& x) { return val(x) < 0.0 ? T(0.0) - x : x; }
template <class T> inline T minv(const T& a, const T& b) { return val(a) < val(b) ? a : b; }
template <class T> inline T maxv(const T& a, const T& b) { return val(a) > val(b) ? a : b; }

// ---------------------------------------------------------------- parameters
struct Params {
  double g;       // gravity
  double r;       // density ratio rho1/rho2 (layer 1 on top)
  double hdry;    // dry tolerance
  double kmin;    // floor of the internal-wave hyperbolicity factor
  double gp;      // reduced gravity (1-r) g
  double inv_gp;  // 1 / ((1-r) g)
};
inline Params make_params(double g, double r, double hdry, double kmin) {
  Params P;
  P.g = g; P.r = r; P.hdry = hdry; P.kmin = kmin;
  P.gp = (1.0 - r) * g;
  P.inv_gp = 1.0 / ((1.0 - r) * g);
  return P;
}

struct Counters {
  int64_t hyp = 0;      // internal-wave factor clamped
  int64_t nclip = 0;    // cells whose nonzero depth fell below the dry tolerance
  int64_t repair = 0;   // wet-ordering repairs (top dry over wet bottom)
  double clip1 = 0.0;   // mass removed from layer 1 by clipping
  double clip2 = 0.0;   // mass removed from layer 2 by clipping / repair
};

// Field order of the state: h1, h1u1, h1v1, h2, h2u2, h2v2.
enum { F_H1 = 0, F_HU1 = 1, F_HV1 = 2, F_H2 = 3, F_HU2 = 4, F_HV2 = 5 };

// ---------------------------------------------------------------- per-cell values
// A cell seen from one sweep direction: m = normal momentum, t = transverse.
template <class T> struct CellV {
  T h1, m1, t1, h2, m2, t2, B;
  T u1, w1, u2, w2, s1, s2;  // normal/transverse velocities, sqrt of depths
  T eta1, eta2;              // surfaces: eta2 = B + h2, eta1 = eta2 + h1 (Eqs. 6-7)
  bool wet1, wet2;
};

template <class T>
CellV<T> make_cell(const Params& P, const T* q /*local order h1 m1 t1 h2 m2 t2*/, const T& B) {
  CellV<T> c;
  c.h1 = q[0]; c.m1 = q[1]; c.t1 = q[2];
  c.h2 = q[3]; c.m2 = q[4]; c.t2 = q[5];
  c.B = B;
  c.wet1 = val(c.h1) >= P.hdry;
  c.wet2 = val(c.h2) >= P.hdry;
  if (c.wet1) {
    T inv = T(1.0) / c.h1;
    c.u1 = c.m1 * inv; c.w1 = c.t1 * inv; c.s1 = sqrt_(c.h1);
  } else {
    c.u1 = T(0.0); c.w1 = T(0.0); c.s1 = T(0.0);
  }
  if (c.wet2) {
    T inv = T(1.0) / c.h2;
    c.u2 = c.m2 * inv; c.w2 = c.t2 * inv; c.s2 = sqrt_(c.h2);
  } else {
    c.u2 = T(0.0); c.w2 = T(0.0); c.s2 = T(0.0);
  }
  c.eta2 = c.B + c.h2;
  c.eta1 = c.eta2 + c.h1;
  return c;
}

// ---------------------------------------------------------------- edge solve
// Six wave slots.  Slots 0..3 carry the four layered waves (external-, internal-,
// internal+, external+ when both layers are wet on both sides; layer-1 left/right
// in slots 0/3 and layer-2 left/right in slots 1/2 otherwise), slots 4 and 5 the
// shear waves of the transverse momenta of layers 1 and 2.
// mode: 0 both fluctuations used, 1 only the part entering the left cell,
//       2 only the part entering the right cell (reflecting edge of a dry cell).
template <class T> struct Waves {
  T s[6];
  T Z[6][6];
  int mode[6];
};

template <class T> inline void zero_waves(Waves<T>& W) {
  for (int p = 0; p < 6; ++p) {
    W.s[p] = T(0.0);
    W.mode[p] = 0;
    for (int c = 0; c < 6; ++c) W.Z[p][c] = T(0.0);
  }
}

// One layer treated alone as single-layer shallow water (some layer dry on some
// side).  J is the jump of the layer's pressure surface across the edge:
// eta1 for the top layer, eta2 + r h1 for the bottom layer.
template <class T>
void layer_alone(const Params& P, int layer, bool wetL, bool wetR, bool wallIfDryR,
                 bool wallIfDryL, const CellV<T>& L, const CellV<T>& R, T J, Waves<T>& W) {
  const int sA = (layer == 1) ? 0 : 1;  // left-going slot
  const int sB = (layer == 1) ? 3 : 2;  // right-going slot
  const int sS = (layer == 1) ? 4 : 5;  // shear slot
  const int c0 = (layer == 1) ? 0 : 3;  // first component of this layer
  if (!wetL && !wetR) return;

  T hL, mL, tL, uL, wL, qL, hR, mR, tR, uR, wR, qR;
  if (layer == 1) {
    hL = L.h1; mL = L.m1; tL = L.t1; uL = L.u1; wL = L.w1; qL = L.s1;
    hR = R.h1; mR = R.m1; tR = R.t1; uR = R.u1; wR = R.w1; qR = R.s1;
  } else {
    hL = L.h2; mL = L.m2; tL = L.t2; uL = L.u2; wL = L.w2; qL = L.s2;
    hR = R.h2; mR = R.m2; tR = R.t2; uR = R.u2; wR = R.w2; qR = R.s2;
  }
  int mode = 0;
  if (wetL && !wetR) {
    T etaL = (layer == 1) ? L.eta1 : L.eta2;
    T botR = (layer == 1) ? R.eta2 : R.B;  // geometric bottom of the layer on the dry side
    bool wall = wallIfDryR || val(etaL) <= val(botR);
    if (wall) {  // reflect: mirror of the wet state
      hR = hL; mR = T(0.0) - mL; tR = tL; uR = T(0.0) - uL; wR = wL; qR = qL;
      J = T(0.0);
      mode = 1;
    } else {     // overtopping onto a dry cell
      hR = T(0.0); mR = T(0.0); tR = T(0.0); uR = T(0.0); wR = T(0.0); qR = T(0.0);
    }
  } else if (!wetL && wetR) {
    T etaR = (layer == 1) ? R.eta1 : R.eta2;
    T botL = (layer == 1) ? L.eta2 : L.B;
    bool wall = wallIfDryL || val(etaR) <= val(botL);
    if (wall) {
      hL = hR; mL = T(0.0) - mR; tL = tR; uL = T(0.0) - uR; wL = wR; qL = qR;
      J = T(0.0);
      mode = 2;
    } else {
      hL = T(0.0); mL = T(0.0); tL = T(0.0); uL = T(0.0); wL = T(0.0); qL = T(0.0);
    }
  }
  const bool effL = val(hL) > 0.0, effR = val(hR) > 0.0;
  T hb = T(0.5) * (hL + hR);
  T d = T(1.0) / (qL + qR);
  T uh = (qL * uL + qR * uR) * d;
  T wh = (qL * wL + qR * wR) * d;
  T dA = mR - mL;
  T dB = (mR * uR - mL * uL) + (T(P.g) * hb) * J;
  T dT = tR * uR - tL * uL;
  T ch = sqrt_(T(P.g) * hb);
  T sa, sb;
  if (effL) sa = minv(uL - sqrt_(T(P.g) * hL), uh - ch);
  else      sa = uR - T(2.0) * sqrt_(T(P.g) * hR);
  if (effR) sb = maxv(uR + sqrt_(T(P.g) * hR), uh + ch);
  else      sb = uL + T(2.0) * sqrt_(T(P.g) * hL);
  T isd = T(1.0) / (sb - sa);
  T bA = (sb * dA - dB) * isd;
  T bB = (dB - sa * dA) * isd;
  W.s[sA] = sa; W.mode[sA] = mode;
  W.Z[sA][c0] = bA; W.Z[sA][c0 + 1] = bA * sa; W.Z[sA][c0 + 2] = bA * wh;
  W.s[sB] = sb; W.mode[sB] = mode;
  W.Z[sB][c0] = bB; W.Z[sB][c0 + 1] = bB * sb; W.Z[sB][c0 + 2] = bB * wh;
  W.s[sS] = uh; W.mode[sS] = mode;
  W.Z[sS][c0 + 2] = dT - wh * dA;
}

// Layered f-wave solve at one edge: the flux-minus-source jump split into four
// coupled waves (speeds to first order in 1 - r at Roe averages, eigenvectors
// (1, s, alpha, alpha s)) and two shear waves; wet/dry edges per layer.
template <class T>
void riemann(const Params& P, const CellV<T>& L, const CellV<T>& R, Waves<T>& W, Counters& C,
             bool count) {
  zero_waves(W);
  if (L.wet1 && L.wet2 && R.wet1 && R.wet2) {
    // Roe-type edge averages
    T hb1 = T(0.5) * (L.h1 + R.h1);
    T hb2 = T(0.5) * (L.h2 + R.h2);
    T d1 = T(1.0) / (L.s1 + R.s1);
    T ub1 = fma_(L.s1, L.u1, R.s1 * R.u1) * d1;
    T wb1 = fma_(L.s1, L.w1, R.s1 * R.w1) * d1;
    T d2 = T(1.0) / (L.s2 + R.s2);
    T ub2 = fma_(L.s2, L.u2, R.s2 * R.u2) * d2;
    T wb2 = fma_(L.s2, L.w2, R.s2 * R.w2) * d2;
    // flux-minus-source jumps; the hydrostatic parts are written through the surfaces
    // (products and sums fused where a product meets a sum)
    T del1 = R.m1 - L.m1;
    T del2 = fma_(T(P.g) * hb1, R.eta1 - L.eta1, fma_(R.m1, R.u1, -(L.m1 * L.u1)));
    T del3 = R.m2 - L.m2;
    T J2 = fma_(T(P.r), R.h1 - L.h1, R.eta2 - L.eta2);
    T del4 = fma_(T(P.g) * hb2, J2, fma_(R.m2, R.u2, -(L.m2 * L.u2)));
    T dt1 = fma_(R.t1, R.u1, -(L.t1 * L.u1));
    T dt2 = fma_(R.t2, R.u2, -(L.t2 * L.u2));
    // speeds: external U -+ sqrt(gH), internal Uc -+ sqrt(g' h1 h2 / H * kappa)
    T H = hb1 + hb2;
    T iH = T(1.0) / H;
    T U = fma_(hb1, ub1, hb2 * ub2) * iH;
    T Uc = fma_(hb1, ub2, hb2 * ub1) * iH;
    T ce = sqrt_(T(P.g) * H);
    T du = ub1 - ub2;
    T kap = fma_(-((du * du) * iH), T(P.inv_gp), T(1.0));
    if (val(kap) < P.kmin) {
      kap = T(P.kmin);
      if (count) C.hyp++;
    }
    T ci = sqrt_((((T(P.gp) * hb1) * hb2) * iH) * kap);
    T s[4];
    s[0] = U - ce; s[1] = Uc - ci; s[2] = Uc + ci; s[3] = U + ce;
    // eigenvectors (1, s, alpha, alpha s)
    T gh1 = T(P.g) * hb1;
    T igh = T(1.0) / gh1;
    T al[4];
    for (int p = 0; p < 4; ++p) {
      T a = s[p] - ub1;
      al[p] = fma_(a, a, -gh1) * igh;
    }
    // Gaussian elimination of R beta = delta, no pivoting, fixed order
    T m11 = s[1] - s[0], m12 = s[2] - s[0], m13 = s[3] - s[0];
    T m21 = al[1] - al[0], m22 = al[2] - al[0], m23 = al[3] - al[0];
    T q0 = al[0] * s[0];
    T m31 = fma_(al[1], s[1], -q0), m32 = fma_(al[2], s[2], -q0), m33 = fma_(al[3], s[3], -q0);
    T b0 = del1;
    T b1 = fma_(-s[0], del1, del2);
    T b2 = fma_(-al[0], del1, del3);
    T b3 = fma_(-q0, del1, del4);
    T ip1 = T(1.0) / m11;
    T f2 = m21 * ip1, f3 = m31 * ip1;
    m22 = fma_(-f2, m12, m22); m23 = fma_(-f2, m13, m23); b2 = fma_(-f2, b1, b2);
    m32 = fma_(-f3, m12, m32); m33 = fma_(-f3, m13, m33); b3 = fma_(-f3, b1, b3);
    T ip2 = T(1.0) / m22;
    T f4 = m32 * ip2;
    m33 = fma_(-f4, m23, m33); b3 = fma_(-f4, b2, b3);
    T be[4];
    be[3] = b3 / m33;
    be[2] = fma_(-m23, be[3], b2) * ip2;
    be[1] = fma_(-m13, be[3], fma_(-m12, be[2], b1)) * ip1;
    be[0] = ((b0 - be[1]) - be[2]) - be[3];
    for (int p = 0; p < 4; ++p) {
      T ba = be[p] * al[p];
      W.s[p] = s[p];
      W.Z[p][0] = be[p];
      W.Z[p][1] = be[p] * s[p];
      W.Z[p][2] = be[p] * wb1;
      W.Z[p][3] = ba;
      W.Z[p][4] = ba * s[p];
      W.Z[p][5] = ba * wb2;
    }
    W.s[4] = ub1; W.Z[4][2] = fma_(-wb1, del1, dt1);
    W.s[5] = ub2; W.Z[5][5] = fma_(-wb2, del3, dt2);
    return;
  }
  // some layer dry on some side: each layer alone over its effective bottom
  T J1 = R.eta1 - L.eta1;
  T J2 = (R.eta2 - L.eta2) + T(P.r) * (R.h1 - L.h1);
  layer_alone(P, 1, L.wet1, R.wet1, false, false, L, R, J1, W);
  layer_alone(P, 2, L.wet2, R.wet2, !R.wet1, !L.wet1, L, R, J2, W);
}

// A- dQ (into the left cell) and A+ dQ (into the right cell); a tie at s = 0 is split.
// The shear waves (slots 4 and 5) have a single nonzero component (2 and 5), so
// sums over their components take that one term only.
inline bool wave_comp(int p, int c) { return p < 4 || (p == 4 && c == 2) || (p == 5 && c == 5); }

template <class T> void fluctuations(const Waves<T>& W, T am[6], T ap[6]) {
  for (int c = 0; c < 6; ++c) { am[c] = T(0.0); ap[c] = T(0.0); }
  for (int p = 0; p < 6; ++p) {
    double sv = val(W.s[p]);
    for (int c = 0; c < 6; ++c) {
      if (!wave_comp(p, c)) continue;
      // a tie adds half the wave: 0.5 Z is exact, so the fused form rounds once
      // like the plain sum
      if (W.mode[p] != 2) {
        if (sv < 0.0) am[c] = am[c] + W.Z[p][c];
        else if (sv == 0.0) am[c] = fma_(T(0.5), W.Z[p][c], am[c]);
      }
      if (W.mode[p] != 1) {
        if (sv > 0.0) ap[c] = ap[c] + W.Z[p][c];
        else if (sv == 0.0) ap[c] = fma_(T(0.5), W.Z[p][c], ap[c]);
      }
    }
  }
}

// Dot product of two 6-vectors, accumulated left to right with fused
// multiply-adds.
template <class T> inline T dot6(const T* a, const T* b) {
  T acc = a[0] * b[0];
  for (int c = 1; c < 6; ++c) acc = fma_(a[c], b[c], acc);
  return acc;
}

// Dot product of wave p of two edges over its components.
template <class T> inline T wave_dot(const Waves<T>& U, const Waves<T>& W, int p) {
  if (p == 4) return U.Z[4][2] * W.Z[4][2];
  if (p == 5) return U.Z[5][5] * W.Z[5][5];
  return dot6(U.Z[p], W.Z[p]);
}

// MC limiter phi(theta) = max(0, min((1+theta)/2, 2, 2 theta)).
template <class T> inline T mc_limiter(const T& th) {
  T a = T(0.5) * (T(1.0) + th);
  T b = T(2.0) * th;
  T m = minv(minv(a, T(2.0)), b);
  return maxv(T(0.0), m);
}

// Second-order correction flux at edge k from its waves and its two neighbour edges.
template <class T>
void correction(const Waves<T>& Wm, const Waves<T>& W, const Waves<T>& Wp, T nu, T F[6]) {
  for (int c = 0; c < 6; ++c) F[c] = T(0.0);
  for (int p = 0; p < 6; ++p) {
    double sv = val(W.s[p]);
    T coef = T(0.0);
    if (W.mode[p] == 0 && sv != 0.0) {
      T dd = wave_dot(W, W, p);
      if (val(dd) != 0.0) {
        const Waves<T>& U = (sv > 0.0) ? Wm : Wp;
        T dn = wave_dot(U, W, p);
        T th = dn / dd;
        T phi = mc_limiter(th);
        T sg = T(sv > 0.0 ? 0.5 : -0.5);
        coef = (sg * (T(1.0) - nu * absv(W.s[p]))) * phi;
      }
    }
    for (int c = 0; c < 6; ++c)
      if (wave_comp(p, c)) F[c] = fma_(coef, W.Z[p][c], F[c]);
  }
}

// Dry-state fix-up after a sweep: clip thin layers (bottom layer first), then
// restore the wet ordering (a layer may be wet only if all layers above it are).
template <class T> void fixup(const Params& P, T* q, bool count, Counters& C) {
  if (val(q[3]) < P.hdry) {
    if (count && val(q[3]) != 0.0) { C.nclip++; C.clip2 += val(q[3]); }
    q[3] = T(0.0); q[4] = T(0.0); q[5] = T(0.0);
  }
  if (val(q[0]) < P.hdry) {
    if (count && val(q[0]) != 0.0) { C.nclip++; C.clip1 += val(q[0]); }
    q[0] = T(0.0); q[1] = T(0.0); q[2] = T(0.0);
  }
  if (val(q[0]) == 0.0 && val(q[3]) > 0.0) {
    if (count) { C.repair++; C.clip2 += val(q[3]); }
    q[3] = T(0.0); q[4] = T(0.0); q[5] = T(0.0);
  }
}

// One 1-D sweep along a line of n interior cells with two ghost cells at each end.
// line[k][0..5] is the state in local order (h1 m1 t1 h2 m2 t2) for k = -2..n+1
// (stored at index k+2), Bl[k+2] the bathymetry.  Writes out[k][6] for k = 0..n-1
// (fix-up applied) and returns the largest wave speed at edges 0..n.
// g4 (optional, [n][4]): for each cell the depth parts (layers 1, 2) of the terms
// its update takes from its left edge (A+dQ - F) and from its right edge
// (A-dQ + F), for the mass fluxes of a flux correction at coarse-fine edges.
template <class T>
double sweep_line(const Params& P, int n, const T* line, const T* Bl, T nu, T* out, bool interior,
                  Counters& C, T* g4 = nullptr) {
  std::vector<CellV<T>> cells(n + 4);
  for (int k = 0; k < n + 4; ++k) cells[k] = make_cell(P, line + 6 * k, Bl[k]);
  // edges e = -1..n+1 at index e+1; edge e lies between cells e-1 and e
  std::vector<Waves<T>> W(n + 3);
  double smax = 0.0;
  for (int e = -1; e <= n + 1; ++e) {
    bool used = (e >= 0 && e <= n);
    riemann(P, cells[e - 1 + 2], cells[e + 2], W[e + 1], C, interior && used);
    if (used)
      for (int p = 0; p < 6; ++p) {
        double a = std::fabs(val(W[e + 1].s[p]));
        if (a > smax) smax = a;
      }
  }
  std::vector<T> am(6 * (n + 1)), ap(6 * (n + 1)), F(6 * (n + 1));
  for (int e = 0; e <= n; ++e) {
    fluctuations(W[e + 1], &am[6 * e], &ap[6 * e]);
    correction(W[e], W[e + 1], W[e + 2], nu, &F[6 * e]);
  }
  const T mnu = T(0.0) - nu;
  for (int k = 0; k < n; ++k) {
    const T* q = line + 6 * (k + 2);
    T* o = out + 6 * k;
    // Q - nu (A+dQ_left + A-dQ_right + F_right - F_left), grouped per edge, the
    // product and the sum rounded once
    for (int c = 0; c < 6; ++c) {
      T gl = ap[6 * k + c] - F[6 * k + c];
      T gr = am[6 * (k + 1) + c] + F[6 * (k + 1) + c];
      o[c] = fma_(mnu, gl + gr, q[c]);
      if (g4 && (c == 0 || c == 3)) {
        g4[4 * k + (c == 0 ? 0 : 1)] = gl;
        g4[4 * k + (c == 0 ? 2 : 3)] = gr;
      }
    }
    fixup(P, o, interior, C);
  }
  return smax;
}

// ---------------------------------------------------------------- level arrays
// A level array stores the six fields over the level's whole index space plus a
// two-cell frame, field-major, rows with x fastest.
struct Grid {
  int nx = 0, ny = 0;
  int pitch() const { return nx + 4; }
  size_t plane() const { return size_t(ny + 4) * size_t(nx + 4); }
  size_t idx(int i, int j) const { return size_t(j + 2) * size_t(nx + 4) + size_t(i + 2); }
};

struct Box {
  int ilo, jlo, nx, ny;
};

// Mirror image of a frame cell across the reflecting walls of the level domain.
inline void mirror_src(const Grid& G, int i, int j, int& si, int& sj, bool& fx, bool& fy) {
  fx = false; fy = false; si = i; sj = j;
  if (i < 0) { si = -1 - i; fx = true; }
  else if (i >= G.nx) { si = 2 * G.nx - 1 - i; fx = true; }
  if (j < 0) { sj = -1 - j; fy = true; }
  else if (j >= G.ny) { sj = 2 * G.ny - 1 - j; fy = true; }
}

// x-sweep of a box: the box rows and the two frame rows on each side, each
// line fixed up; writes the intermediate state qs (six planes of
// nx x (ny + 4), rows jlo-2 .. jlo+ny+1, columns ilo .. ilo+nx-1).
// mflux (optional, [8][plane] over the level): for every interior cell of the
// box, the mass flux of each layer through its left and right edges as its
// update sees it (normal momentum minus the left-edge term, plus the right-edge
// term): planes 0-1 left edge, 2-3 right edge (layers 1, 2).
template <class T>
double x_pass(const Params& P, const Grid& G, const T* q, const T* B, const Box& bx, T nux, T* qs,
              Counters& C, T* mflux = nullptr) {
  const size_t pl = G.plane();
  const int nx = bx.nx, ny = bx.ny;
  std::vector<T> line(6 * (nx + 4)), Bl(nx + 4), out(6 * nx), g4(4 * nx);
  double smax = 0.0;
  for (int jj = -2; jj < ny + 2; ++jj) {
    int j = bx.jlo + jj;
    for (int k = -2; k < nx + 2; ++k) {
      int i = bx.ilo + k;
      for (int c = 0; c < 6; ++c) line[6 * (k + 2) + c] = q[c * pl + G.idx(i, j)];
      Bl[k + 2] = B[G.idx(i, j)];
    }
    bool interior = (jj >= 0 && jj < ny);
    double s = sweep_line(P, nx, line.data(), Bl.data(), nux, out.data(), interior, C,
                          mflux && interior ? g4.data() : nullptr);
    if (interior && s > smax) smax = s;
    if (mflux && interior)
      for (int k = 0; k < nx; ++k) {
        const size_t id = G.idx(bx.ilo + k, j);
        const T m1 = line[6 * (k + 2) + 1], m2 = line[6 * (k + 2) + 4];
        mflux[0 * pl + id] = m1 - g4[4 * k + 0];
        mflux[1 * pl + id] = m2 - g4[4 * k + 1];
        mflux[2 * pl + id] = m1 + g4[4 * k + 2];
        mflux[3 * pl + id] = m2 + g4[4 * k + 3];
      }
    for (int k = 0; k < nx; ++k)
      for (int c = 0; c < 6; ++c)
        qs[(size_t(c) * (ny + 4) + (jj + 2)) * nx + k] = out[6 * k + c];
  }
  return smax;
}

// y-sweep of a box over the intermediate state: columns in the y orientation
// (normal momentum hv, transverse hu), each fixed up; writes the box interior
// of qo.
// mflux as for x_pass, planes 4-5 lower edge, 6-7 upper edge.
template <class T>
double y_pass(const Params& P, const Grid& G, const T* qs, const T* B, const Box& bx, T nuy, T* qo,
              Counters& C, T* mflux = nullptr) {
  const size_t pl = G.plane();
  const int nx = bx.nx, ny = bx.ny;
  static const int ymap[6] = {0, 2, 1, 3, 5, 4};
  std::vector<T> linev(6 * (ny + 4)), Bv(ny + 4), outv(6 * ny), g4(4 * ny);
  double smax = 0.0;
  for (int k = 0; k < nx; ++k) {
    int i = bx.ilo + k;
    for (int jj = -2; jj < ny + 2; ++jj) {
      for (int c = 0; c < 6; ++c)
        linev[6 * (jj + 2) + c] = qs[(size_t(ymap[c]) * (ny + 4) + (jj + 2)) * nx + k];
      Bv[jj + 2] = B[G.idx(i, bx.jlo + jj)];
    }
    double s = sweep_line(P, ny, linev.data(), Bv.data(), nuy, outv.data(), true, C,
                          mflux ? g4.data() : nullptr);
    if (s > smax) smax = s;
    if (mflux)
      for (int jj = 0; jj < ny; ++jj) {
        const size_t id = G.idx(i, bx.jlo + jj);
        const T m1 = linev[6 * (jj + 2) + 1], m2 = linev[6 * (jj + 2) + 4];
        mflux[4 * pl + id] = m1 - g4[4 * jj + 0];
        mflux[5 * pl + id] = m2 - g4[4 * jj + 1];
        mflux[6 * pl + id] = m1 + g4[4 * jj + 2];
        mflux[7 * pl + id] = m2 + g4[4 * jj + 3];
      }
    for (int jj = 0; jj < ny; ++jj)
      for (int c = 0; c < 6; ++c)
        qo[size_t(ymap[c]) * pl + G.idx(i, bx.jlo + jj)] = outv[6 * jj + c];
  }
  return smax;
}

// One split step of the box `bx` of a level: reads q (interior and two-cell frame
// valid around the box), writes the box interior of qo.  x-sweep over the box rows
// and the two frame rows on each side, fix-up, y-sweep, fix-up.
template <class T>
void step_box(const Params& P, const Grid& G, const T* q, const T* B, const Box& bx, double dx,
              double dy, double dt, T* qo, double smax[2], Counters& C, T* mflux = nullptr) {
  std::vector<T> qs(size_t(6) * size_t(bx.nx) * size_t(bx.ny + 4));
  smax[0] = x_pass(P, G, q, B, bx, T(dt / dx), qs.data(), C, mflux);
  smax[1] = y_pass(P, G, qs.data(), B, bx, T(dt / dy), qo, C, mflux);
}

// Reflecting-wall fill of every frame cell of a single-box level.
template <class T> void wall_fill_all(const Grid& G, T* q) {
  const size_t pl = G.plane();
  for (int j = -2; j < G.ny + 2; ++j)
    for (int i = -2; i < G.nx + 2; ++i) {
      if (i >= 0 && i < G.nx && j >= 0 && j < G.ny) continue;
      int si, sj; bool fx, fy;
      mirror_src(G, i, j, si, sj, fx, fy);
      for (int c = 0; c < 6; ++c) {
        T v = q[c * pl + G.idx(si, sj)];
        if ((fx && (c == F_HU1 || c == F_HU2)) || (fy && (c == F_HV1 || c == F_HV2))) v = T(0.0) - v;
        q[c * pl + G.idx(i, j)] = v;
      }
    }
}

template <class T> void wall_fill_B(const Grid& G, T* B) {
  for (int j = -2; j < G.ny + 2; ++j)
    for (int i = -2; i < G.nx + 2; ++i) {
      if (i >= 0 && i < G.nx && j >= 0 && j < G.ny) continue;
      int si, sj; bool fx, fy;
      mirror_src(G, i, j, si, sj, fx, fy);
      B[G.idx(i, j)] = B[G.idx(si, sj)];
    }
}

}  // namespace ora
