// Operation census of one fixed-grid step -- TEST AND MEASUREMENT INFRASTRUCTURE
// ONLY (never linked by the product library).
//
// Runs the oracle's own x- and y-passes of one split step (the same templated
// code as every other oracle entry point) in a number type that counts each
// FP64 operation the method performs: add/subtract, multiply, divide, square
// root, negation and fused multiply-add.  The totals, per sweep, give the
// algorithmic operation count per cell update of a workload, which prices the
// arithmetic roof of the sweeps the way 104 bytes per cell update prices their
// memory roof.
#include "ora_core.hpp"

namespace ora {

struct OpTally {
  long long add = 0, mul = 0, div = 0, sqrt = 0, neg = 0, fma = 0;
};
static OpTally g_tally;

struct Tally {
  double v;
  Tally() : v(0) {}
  Tally(double x) : v(x) {}
};
inline Tally operator+(Tally a, Tally b) { g_tally.add++; return Tally(a.v + b.v); }
inline Tally operator-(Tally a, Tally b) { g_tally.add++; return Tally(a.v - b.v); }
inline Tally operator-(Tally a) { g_tally.neg++; return Tally(-a.v); }
inline Tally operator*(Tally a, Tally b) { g_tally.mul++; return Tally(a.v * b.v); }
inline Tally operator/(Tally a, Tally b) { g_tally.div++; return Tally(a.v / b.v); }
inline double val(const Tally& x) { return x.v; }
inline Tally sqrt_(const Tally& x) { g_tally.sqrt++; return Tally(std::sqrt(x.v)); }
inline Tally fma_(const Tally& a, const Tally& b, const Tally& c) {
  g_tally.fma++;
  return Tally(std::fma(a.v, b.v, c.v));
}

}  // namespace ora

using namespace ora;

extern "C" {

// One step of an nx x ny wall-bounded grid (inputs as for ora_fixed_steps) with
// the census on: out[0..5] = add, mul, div, sqrt, neg, fma of the x-pass (ny + 4
// rows of nx cells), out[6..11] the same for the y-pass (nx columns of ny cells).
// Returns 0, or -1 for sizes below 2.
int ora_count_ops(int nx, int ny, double dx, double dy, double g, double r, double hdry, double kmin,
                  const double* Bi, const double* q, double dt, long long* out) {
  if (nx < 2 || ny < 2) return -1;
  Params P = make_params(g, r, hdry, kmin);
  Grid G; G.nx = nx; G.ny = ny;
  const size_t pl = G.plane();
  std::vector<Tally> a(6 * pl, Tally(0.0)), b(6 * pl, Tally(0.0)), B(pl, Tally(0.0));
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      B[G.idx(i, j)] = Tally(Bi[size_t(j) * nx + i]);
      for (int c = 0; c < 6; ++c) a[c * pl + G.idx(i, j)] = Tally(q[(size_t(c) * ny + j) * nx + i]);
    }
  wall_fill_B(G, B.data());
  wall_fill_all(G, a.data());
  Counters C;
  Box bx{0, 0, nx, ny};
  std::vector<Tally> qs(size_t(6) * size_t(nx) * size_t(ny + 4));
  const Tally nux(dt / dx), nuy(dt / dy);
  g_tally = OpTally();
  x_pass(P, G, a.data(), B.data(), bx, nux, qs.data(), C);
  const OpTally tx = g_tally;
  g_tally = OpTally();
  y_pass(P, G, qs.data(), B.data(), bx, nuy, b.data(), C);
  const OpTally ty = g_tally;
  const OpTally* t[2] = {&tx, &ty};
  for (int k = 0; k < 2; ++k) {
    out[6 * k + 0] = t[k]->add;
    out[6 * k + 1] = t[k]->mul;
    out[6 * k + 2] = t[k]->div;
    out[6 * k + 3] = t[k]->sqrt;
    out[6 * k + 4] = t[k]->neg;
    out[6 * k + 5] = t[k]->fma;
  }
  return 0;
}

}  // extern "C"
