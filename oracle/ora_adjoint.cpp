// Reference oracle for the two-layer shallow-water hot path -- TEST INFRASTRUCTURE ONLY.
// Gauge-misfit loss of a fixed-grid wall-bounded run and its directional
// derivative by forward-mode dual numbers through the same oracle step.  The
// derivative is exact for the discrete forward map with the dt sequence frozen;
// it is what the GPU adjoint (a reverse sweep) must reproduce as <grad L, v>.
#include "ora_core.hpp"

namespace ora {

// Parameters: initial top surface eta1_0 and bathymetry B (interior n x n, row
// major).  Initial state: h2 = eta2_0 - B, h1 = eta1_0 - eta2_0, at rest, with
// the interface eta2_0 held fixed when B varies; thin layers are dry.
template <class T>
T c5_loss(const Params& P, int n, double dx, const T* eta1_0, const T* Bi, double eta2_0, int nsteps,
          const double* dts, int every, int gi0, int gj0, int gn, const double* targets) {
  Grid G; G.nx = n; G.ny = n;
  const size_t pl = G.plane();
  std::vector<T> a(6 * pl, T(0.0)), b(6 * pl, T(0.0)), B(pl, T(0.0));
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      size_t k = G.idx(i, j);
      B[k] = Bi[size_t(j) * n + i];
      T h2 = T(eta2_0) - B[k];
      T h1 = eta1_0[size_t(j) * n + i] - T(eta2_0);
      if (val(h2) < P.hdry) h2 = T(0.0);
      if (val(h1) < P.hdry) h1 = T(0.0);
      a[F_H1 * pl + k] = h1;
      a[F_H2 * pl + k] = h2;
    }
  wall_fill_B(G, B.data());
  Counters C;
  Box bx{0, 0, n, n};
  T loss = T(0.0);
  int sample = 0;
  for (int s = 0; s < nsteps; ++s) {
    wall_fill_all(G, a.data());
    double sm[2];
    step_box(P, G, a.data(), B.data(), bx, dx, dx, dts[s], b.data(), sm, C);
    std::swap(a, b);
    if ((s + 1) % every == 0) {
      const double* tg = targets + size_t(sample) * gn * gn;
      for (int j = 0; j < gn; ++j)
        for (int i = 0; i < gn; ++i) {
          size_t k = G.idx(gi0 + i, gj0 + j);
          T eta1 = (B[k] + a[F_H2 * pl + k]) + a[F_H1 * pl + k];
          T d = eta1 - T(tg[j * gn + i]);
          loss = loss + d * d;
        }
      ++sample;
    }
  }
  return loss;
}

}  // namespace ora

using namespace ora;

extern "C" {

// Loss value; with v_eta / v_B non-null also its directional derivative along
// (v_eta, v_B) in *dloss.
double ora_gauge_loss(int n, double dx, double g, double r, double hdry, double kmin,
                      const double* eta1_0, const double* B, double eta2_0, int nsteps,
                      const double* dts, int every, int gi0, int gj0, int gn, const double* targets,
                      const double* v_eta, const double* v_B, double* dloss) {
  Params P = make_params(g, r, hdry, kmin);
  const size_t N = size_t(n) * n;
  if (!v_eta && !v_B) {
    return c5_loss<double>(P, n, dx, eta1_0, B, eta2_0, nsteps, dts, every, gi0, gj0, gn, targets);
  }
  std::vector<Dual> e(N), b(N);
  for (size_t k = 0; k < N; ++k) {
    e[k] = Dual(eta1_0[k], v_eta ? v_eta[k] : 0.0);
    b[k] = Dual(B[k], v_B ? v_B[k] : 0.0);
  }
  Dual L = c5_loss<Dual>(P, n, dx, e.data(), b.data(), eta2_0, nsteps, dts, every, gi0, gj0, gn, targets);
  if (dloss) *dloss = L.d;
  return L.v;
}

}  // extern "C"
