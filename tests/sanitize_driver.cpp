// Drives the oracle's C interface through a small three-level run (refine,
// flag, cluster, regrid, subcycled steps, coarsen, rejection bookkeeping), a
// refine point and a fixed-grid run, for a build with address and
// undefined-behaviour sanitizers.  Exits non-zero on a failed call.
#include <cmath>
#include <cstdio>
#include <vector>

extern "C" {
void* ora_create(double g, double r, double hdry, double kmin, double cfl, double cflmax, int nlev, const int* ratio,
                 int nx0, int ny0, double dx0, double dy0);
void ora_destroy(void* h);
int ora_set_bathymetry(void* h, const double* Bf);
int ora_set_state(void* h, int l, const double* q);
int ora_get_state(void* h, int l, double* q);
int ora_advance(void* h, int nsteps, int regrid_every, const double* tau, int nbuf, double* dts);
int ora_get_npatches(void* h, int l);
int ora_refine_point(double hdry, int r, int a, int b, const double* q5, int inx, int iny, double Bf, double* out);
int ora_fixed_steps(int nx, int ny, double dx, double dy, double g, double r, double hdry, double kmin,
                    const double* B, double* q, int nsteps, const double* dts, double* smax, double* cnt);
}

int main() {
  const int n0 = 24, ratio[2] = {2, 2};
  const int nf = n0 * 4;
  const double L = 48e3, dx0 = L / n0, dxf = L / nf;
  std::vector<double> Bf((size_t)nf * nf), q0((size_t)6 * n0 * n0, 0.0);
  for (int j = 0; j < nf; ++j)
    for (int i = 0; i < nf; ++i) {
      const double x = (i + 0.5) * dxf, y = (j + 0.5) * dxf;
      Bf[(size_t)j * nf + i] = -3000.0 + 3100.0 * x / L + 200.0 * std::sin(6.0 * y / L);
    }
  for (int j = 0; j < n0; ++j)
    for (int i = 0; i < n0; ++i) {
      double B = 0.0;
      for (int b = 0; b < 4; ++b)
        for (int a = 0; a < 4; ++a) B += Bf[(size_t)(4 * j + b) * nf + 4 * i + a];
      B /= 16.0;
      const double x = (i + 0.5) * dx0 - 0.3 * L, y = (j + 0.5) * dx0 - 0.5 * L;
      const double eta1 = 2.0 * std::exp(-(x * x + y * y) / (2.0 * 4e3 * 4e3)), eta2 = -150.0;
      double h2 = eta2 - B > 0.0 ? eta2 - B : 0.0;
      double h1 = eta1 - (B + h2) > 0.0 ? eta1 - (B + h2) : 0.0;
      if (h2 < 1e-3) h2 = 0.0;
      if (h1 < 1e-3) { h1 = 0.0; h2 = 0.0; }
      q0[(size_t)0 * n0 * n0 + j * n0 + i] = h1;
      q0[(size_t)3 * n0 * n0 + j * n0 + i] = h2;
    }
  void* h = ora_create(9.81, 0.95, 1e-3, 1e-6, 0.9, 1.0, 3, ratio, n0, n0, dx0, dx0);
  if (!h) return 2;
  if (ora_set_bathymetry(h, Bf.data()) || ora_set_state(h, 0, q0.data())) return 3;
  const double tau[2] = {2e-5, 4e-5};
  std::vector<double> dts(6);
  if (ora_advance(h, 6, 3, tau, 2, dts.data())) return 4;
  std::vector<double> q2((size_t)6 * nf * nf);
  if (ora_get_state(h, 2, q2.data())) return 5;
  std::printf("patches %d %d %d dt %g\n", ora_get_npatches(h, 0), ora_get_npatches(h, 1), ora_get_npatches(h, 2),
              dts[5]);
  ora_destroy(h);
  double q5[35] = {0}, out[6];
  for (int k = 0; k < 5; ++k) { q5[7 * k + 0] = 10.0 + k; q5[7 * k + 3] = 100.0; q5[7 * k + 6] = -200.0 - k; }
  for (int a = 0; a < 4; ++a) ora_refine_point(1e-3, 4, a, 3 - a, q5, 1, 0, -201.0, out);
  std::vector<double> qf(q0), sm(4), cnt(5);
  std::vector<double> B0((size_t)n0 * n0, -3000.0), dtf = {5.0, 5.0};
  if (ora_fixed_steps(n0, n0, dx0, dx0, 9.81, 0.95, 1e-3, 1e-6, B0.data(), qf.data(), 2, dtf.data(), sm.data(),
                      cnt.data()))
    return 6;
  std::printf("ok\n");
  return 0;
}
