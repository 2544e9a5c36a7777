// Reference oracle for the two-layer shallow-water hot path -- TEST INFRASTRUCTURE ONLY.
// Plain CPU FP64 implementation of the level hierarchy, the multilayer refine and
// coarsen operators, flagging, clustering, ghost filling and the subcycled
// (Berger-Oliger) advance.  Shares no code with the HIP library; only the tests,
// the smoke check and the benchmark's CPU-baseline leg call it.
//
// Paper passages followed:
//   level hierarchy and refinement ratios ......... Sec. 2, Eqs. (1)-(2)
//   time refinement r_t = max(r_x, r_y) ............ Sec. 2 (text after Eq. 2)
//   wet ordering of layers ......................... Sec. 2.1 (first paragraph)
//   refine surfaces, not depths; refine bathymetry . Sec. 2.1 (second paragraph)
//   surfaces and effective bathymetry .............. Sec. 2.1, Eqs. (3)-(9)
//   minmod-limited linear interpolant .............. Sec. 2.1, Eq. (10)
//   bottom layer first, then up through B-hat ...... Sec. 2.1 (last paragraph)
//   coarsening by averaging all quantities ......... Sec. 2.2, Eq. (11)
#include "ora_core.hpp"

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <limits>
#include <thread>

namespace ora {

enum { OK = 0, E_INVAL = -1, E_CFL = -4, E_NAN = -5 };

struct Level {
  Grid G;
  double dx = 0, dy = 0;
  std::vector<double> q[2];
  int cur = 0;
  std::vector<double> B;
  std::vector<Box> boxes;
  std::vector<uint8_t> mask;  // 1 where an interior cell is covered by a patch
  double smax[2] = {0, 0};    // largest speeds seen during the last coarse step
  std::vector<double> mflux;  // [8][plane]: edge mass fluxes of the last step (flux correction)
};

struct Hier {
  Params P;
  double cfl = 0.9, cflmax = 1.0;
  int nlev = 1;
  int ratio[8] = {0};
  std::vector<Level> L;
  Counters C;
  int64_t updates[8] = {0};
  double t = 0.0;
  bool have_smax = false;
  double cmax = 0.0;     // largest substep Courant number of the current coarse step
  int retries = 8;       // rejected coarse steps are retaken at most this often
  int64_t rejected = 0;  // coarse steps rejected so far
  bool reflux = false;   // mass flux correction at coarse-fine edges
  bool dyn_rt = false;   // time ratios chosen per coarse step from the last speeds
  int rt[8] = {0};       // substeps of level l + 1 per substep of level l (this coarse step)
};

// ---------------------------------------------------------------- refine (Sec. 2.1)
// minmod: zero unless both arguments have strictly the same sign, else the one
// of smaller modulus (Eq. 10 and the sentence after it).
inline double minmod(double a, double b) {
  if (a > 0.0 && b > 0.0) return a < b ? a : b;
  if (a < 0.0 && b < 0.0) return a > b ? a : b;
  return 0.0;
}

// Coarse data at time fraction th between two buffers (linear in time).
struct CoarseSrc {
  const Level* L;
  const double* qo;
  const double* qn;
  double th;
  void get(int I, int J, double out[7]) const {
    const size_t pl = L->G.plane(), k = L->G.idx(I, J);
    for (int c = 0; c < 6; ++c) out[c] = (1.0 - th) * qo[c * pl + k] + th * qn[c * pl + k];
    out[6] = L->B[k];
  }
};

// Fills one fine cell (child (a,b) of coarse cell (I,J), ratio r) from coarse data.
// Surfaces are interpolated bottom layer first (eta2 = B + h2, Eq. 9), the
// fine depths recovered through the fine bathymetry and the effective
// bathymetry B-hat = B + h2 (Eqs. 5, 8), then the wet ordering is enforced.
void refine_cell(const Params& P, const CoarseSrc& S, int r, int I, int J, int a, int b, double Bf,
                 double out[6], Counters& C) {
  const int nxc = S.L->G.nx, nyc = S.L->G.ny;
  const double fa = double(2 * a + 1 - r) / double(2 * r);
  const double fb = double(2 * b + 1 - r) / double(2 * r);
  double c0[7] = {0}, xl[7] = {0}, xr[7] = {0}, yd[7] = {0}, yu[7] = {0};
  const bool inx = (I - 1 >= 0) && (I + 1 < nxc);
  const bool iny = (J - 1 >= 0) && (J + 1 < nyc);
  S.get(I, J, c0);
  if (inx) { S.get(I - 1, J, xl); S.get(I + 1, J, xr); }
  if (iny) { S.get(I, J - 1, yd); S.get(I, J + 1, yu); }
  auto eta = [](const double* q, int m) { return m == 2 ? q[6] + q[3] : (q[6] + q[3]) + q[0]; };
  auto wet = [&](const double* q, int m) { return (m == 2 ? q[3] : q[0]) >= P.hdry; };
  double etaf[3] = {0, 0, 0};
  bool sxok[3], syok[3];
  for (int m = 2; m >= 1; --m) {
    sxok[m] = inx && wet(xl, m) && wet(c0, m) && wet(xr, m);
    syok[m] = iny && wet(yd, m) && wet(c0, m) && wet(yu, m);
    double e = eta(c0, m);
    double sx = sxok[m] ? minmod(e - eta(xl, m), eta(xr, m) - e) : 0.0;
    double sy = syok[m] ? minmod(e - eta(yd, m), eta(yu, m) - e) : 0.0;
    etaf[m] = (e + sx * fa) + sy * fb;
  }
  double h2 = wet(c0, 2) ? etaf[2] - Bf : 0.0;
  if (h2 < P.hdry) h2 = 0.0;
  double Bhat = Bf + h2;
  double h1 = wet(c0, 1) ? etaf[1] - Bhat : 0.0;
  if (h1 < P.hdry) h1 = 0.0;
  if (h1 == 0.0 && h2 > 0.0) { h2 = 0.0; C.repair++; }
  auto mom = [&](int f, int m) {
    double v = c0[f];
    double sx = sxok[m] ? minmod(v - xl[f], xr[f] - v) : 0.0;
    double sy = syok[m] ? minmod(v - yd[f], yu[f] - v) : 0.0;
    return (v + sx * fa) + sy * fb;
  };
  out[F_H1] = h1;
  out[F_HU1] = h1 > 0.0 ? mom(F_HU1, 1) : 0.0;
  out[F_HV1] = h1 > 0.0 ? mom(F_HV1, 1) : 0.0;
  out[F_H2] = h2;
  out[F_HU2] = h2 > 0.0 ? mom(F_HU2, 2) : 0.0;
  out[F_HV2] = h2 > 0.0 ? mom(F_HV2, 2) : 0.0;
}

// ---------------------------------------------------------------- hierarchy set-up
static void alloc_level(Level& L, int nx, int ny, double dx, double dy) {
  L.G.nx = nx; L.G.ny = ny; L.dx = dx; L.dy = dy;
  L.q[0].assign(6 * L.G.plane(), 0.0);
  L.q[1].assign(6 * L.G.plane(), 0.0);
  L.B.assign(L.G.plane(), 0.0);
  L.mask.assign(L.G.plane(), 0);
  L.cur = 0;
}

static void rebuild_mask(Level& L) {
  std::fill(L.mask.begin(), L.mask.end(), 0);
  for (const Box& b : L.boxes)
    for (int j = b.jlo; j < b.jlo + b.ny; ++j)
      for (int i = b.ilo; i < b.ilo + b.nx; ++i) L.mask[L.G.idx(i, j)] = 1;
}

static bool boxes_valid(const Level& L, int n, const int* bx) {
  std::vector<uint8_t> m(size_t(L.G.nx) * L.G.ny, 0);
  for (int k = 0; k < n; ++k) {
    int ilo = bx[4 * k], jlo = bx[4 * k + 1], nx = bx[4 * k + 2], ny = bx[4 * k + 3];
    if (nx <= 0 || ny <= 0 || ilo < 0 || jlo < 0 || ilo + nx > L.G.nx || jlo + ny > L.G.ny) return false;
    for (int j = jlo; j < jlo + ny; ++j)
      for (int i = ilo; i < ilo + nx; ++i) {
        if (m[size_t(j) * L.G.nx + i]) return false;  // overlap
        m[size_t(j) * L.G.nx + i] = 1;
      }
  }
  return true;
}

// Finest-level samples define the bathymetry; each coarser level holds block means
// (row-major sum of the r x r children times 1/r^2), so "refining the bathymetry"
// is a lookup of the finer level's values.
static void build_bathymetry(Hier& H, const double* Bf) {
  Level& F = H.L[H.nlev - 1];
  for (int j = 0; j < F.G.ny; ++j)
    for (int i = 0; i < F.G.nx; ++i) F.B[F.G.idx(i, j)] = Bf[size_t(j) * F.G.nx + i];
  wall_fill_B(F.G, F.B.data());
  for (int l = H.nlev - 2; l >= 0; --l) {
    Level& Lc = H.L[l];
    const Level& Lf = H.L[l + 1];
    const int r = H.ratio[l];
    const double inv = 1.0 / double(r * r);
    for (int J = 0; J < Lc.G.ny; ++J)
      for (int I = 0; I < Lc.G.nx; ++I) {
        double s = 0.0;
        for (int b = 0; b < r; ++b)
          for (int a = 0; a < r; ++a) s = s + Lf.B[Lf.G.idx(r * I + a, r * J + b)];
        Lc.B[Lc.G.idx(I, J)] = s * inv;
      }
    wall_fill_B(Lc.G, Lc.B.data());
  }
}

// New patches of a fine level: cells already covered by an old patch of that
// level keep their values, all other new cells are refined from the coarser level.
static int set_patches(Hier& H, int l, int n, const int* bx) {
  Level& L = H.L[l];
  if (!boxes_valid(L, n, bx)) return E_INVAL;
  std::vector<uint8_t> old = L.mask;
  L.boxes.clear();
  for (int k = 0; k < n; ++k) L.boxes.push_back(Box{bx[4 * k], bx[4 * k + 1], bx[4 * k + 2], bx[4 * k + 3]});
  rebuild_mask(L);
  if (l == 0) return OK;
  const Level& Lc = H.L[l - 1];
  const int r = H.ratio[l - 1];
  CoarseSrc S{&Lc, Lc.q[Lc.cur].data(), Lc.q[Lc.cur].data(), 0.0};
  double* q = L.q[L.cur].data();
  const size_t pl = L.G.plane();
  for (const Box& b : L.boxes)
    for (int j = b.jlo; j < b.jlo + b.ny; ++j)
      for (int i = b.ilo; i < b.ilo + b.nx; ++i) {
        size_t k = L.G.idx(i, j);
        if (old[k]) continue;
        double out[6];
        refine_cell(H.P, S, r, i / r, j / r, i % r, j % r, L.B[k], out, H.C);
        for (int c = 0; c < 6; ++c) q[c * pl + k] = out[c];
      }
  return OK;
}

// ---------------------------------------------------------------- ghost cells
// Frame cells of every patch of level l at time fraction th of the coarser
// level's last step: cells inside the domain not covered by a sibling patch are
// refined from time-interpolated coarse data; then cells outside the domain
// mirror the in-domain values (reflecting walls).
static void ghost_fill(Hier& H, int l, double th) {
  Level& L = H.L[l];
  double* q = L.q[L.cur].data();
  const size_t pl = L.G.plane();
  if (l > 0) {
    const Level& Lc = H.L[l - 1];
    const int r = H.ratio[l - 1];
    CoarseSrc S{&Lc, Lc.q[1 - Lc.cur].data(), Lc.q[Lc.cur].data(), th};
    for (const Box& b : L.boxes)
      for (int j = b.jlo - 2; j < b.jlo + b.ny + 2; ++j)
        for (int i = b.ilo - 2; i < b.ilo + b.nx + 2; ++i) {
          if (i < 0 || j < 0 || i >= L.G.nx || j >= L.G.ny) continue;
          size_t k = L.G.idx(i, j);
          if (L.mask[k]) continue;
          double out[6];
          refine_cell(H.P, S, r, i / r, j / r, i % r, j % r, L.B[k], out, H.C);
          for (int c = 0; c < 6; ++c) q[c * pl + k] = out[c];
        }
  }
  for (const Box& b : L.boxes)
    for (int j = b.jlo - 2; j < b.jlo + b.ny + 2; ++j)
      for (int i = b.ilo - 2; i < b.ilo + b.nx + 2; ++i) {
        if (i >= 0 && j >= 0 && i < L.G.nx && j < L.G.ny) continue;
        int si, sj; bool fx, fy;
        mirror_src(L.G, i, j, si, sj, fx, fy);
        for (int c = 0; c < 6; ++c) {
          double v = q[c * pl + L.G.idx(si, sj)];
          if ((fx && (c == F_HU1 || c == F_HU2)) || (fy && (c == F_HV1 || c == F_HV2))) v = 0.0 - v;
          q[c * pl + L.G.idx(i, j)] = v;
        }
      }
}

// ---------------------------------------------------------------- step one level
static int step_level(Hier& H, int l, double dt, double th, double smax[2]) {
  Level& L = H.L[l];
  ghost_fill(H, l, th);
  smax[0] = 0.0; smax[1] = 0.0;
  const double* q = L.q[L.cur].data();
  double* qo = L.q[1 - L.cur].data();
  double* mf = nullptr;
  if (H.reflux) {
    L.mflux.assign(8 * L.G.plane(), 0.0);
    mf = L.mflux.data();
  }
  for (const Box& b : L.boxes) {
    double s[2];
    step_box(H.P, L.G, q, L.B.data(), b, L.dx, L.dy, dt, qo, s, H.C, mf);
    smax[0] = std::max(smax[0], s[0]);
    smax[1] = std::max(smax[1], s[1]);
    H.updates[l] += int64_t(b.nx) * b.ny;
  }
  L.cur = 1 - L.cur;
  L.smax[0] = std::max(L.smax[0], smax[0]);
  L.smax[1] = std::max(L.smax[1], smax[1]);
  double courant = dt * std::max(smax[0] / L.dx, smax[1] / L.dy);
  if (courant > H.cmax || courant != courant) H.cmax = courant;
  if (!(courant <= H.cflmax)) return E_CFL;
  return OK;
}

// ---------------------------------------------------------------- coarsen (Sec. 2.2)
// Every coarse cell under a fine patch takes the average of its r x r children for
// all six quantities (Eq. 11 in two dimensions), followed by the dry-state fix-up.
static void coarsen(Hier& H, int lf) {
  const Level& Lf = H.L[lf];
  Level& Lc = H.L[lf - 1];
  const int r = H.ratio[lf - 1];
  const double inv = 1.0 / double(r * r);
  const double* qf = Lf.q[Lf.cur].data();
  double* qc = Lc.q[Lc.cur].data();
  const size_t pf = Lf.G.plane(), pc = Lc.G.plane();
  Counters dummy;
  for (const Box& b : Lf.boxes)
    for (int J = b.jlo / r; J < (b.jlo + b.ny) / r; ++J)
      for (int I = b.ilo / r; I < (b.ilo + b.nx) / r; ++I) {
        double v[6];
        for (int c = 0; c < 6; ++c) {
          double s = 0.0;
          for (int bb = 0; bb < r; ++bb)
            for (int aa = 0; aa < r; ++aa) s = s + qf[c * pf + Lf.G.idx(r * I + aa, r * J + bb)];
          v[c] = s * inv;
        }
        fixup(H.P, v, false, dummy);
        for (int c = 0; c < 6; ++c) qc[c * pc + Lc.G.idx(I, J)] = v[c];
      }
}

// ---------------------------------------------------------------- flag + buffer
// Cell flagged iff the top layer is wet in it and its four face neighbours (each
// covered by the level, or mirrored across a wall) and the centred |grad eta1|
// exceeds tau; then dilated by nbuf cells within the level's coverage.
static void flag(const Hier& H, int l, double tau, int nbuf, uint8_t* out) {
  const Level& L = H.L[l];
  const int nx = L.G.nx, ny = L.G.ny;
  const double* q = L.q[L.cur].data();
  const size_t pl = L.G.plane();
  auto mir = [&](int& i, int& j) {
    if (i < 0) i = -1 - i; else if (i >= nx) i = 2 * nx - 1 - i;
    if (j < 0) j = -1 - j; else if (j >= ny) j = 2 * ny - 1 - j;
  };
  auto ok = [&](int i, int j) {
    mir(i, j);
    size_t k = L.G.idx(i, j);
    return L.mask[k] && q[F_H1 * pl + k] >= H.P.hdry;
  };
  auto eta1 = [&](int i, int j) {
    mir(i, j);
    size_t k = L.G.idx(i, j);
    return (L.B[k] + q[F_H2 * pl + k]) + q[F_H1 * pl + k];
  };
  std::vector<uint8_t> raw(size_t(nx) * ny, 0);
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      if (!ok(i, j) || !ok(i - 1, j) || !ok(i + 1, j) || !ok(i, j - 1) || !ok(i, j + 1)) continue;
      double gx = std::fabs(eta1(i + 1, j) - eta1(i - 1, j)) / (2.0 * L.dx);
      double gy = std::fabs(eta1(i, j + 1) - eta1(i, j - 1)) / (2.0 * L.dy);
      double gm = gx > gy ? gx : gy;
      raw[size_t(j) * nx + i] = gm > tau ? 1 : 0;
    }
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      uint8_t f = 0;
      if (L.mask[L.G.idx(i, j)])
        for (int jj = std::max(0, j - nbuf); jj <= std::min(ny - 1, j + nbuf) && !f; ++jj)
          for (int ii = std::max(0, i - nbuf); ii <= std::min(nx - 1, i + nbuf); ++ii)
            if (raw[size_t(jj) * nx + ii]) { f = 1; break; }
      out[size_t(j) * nx + i] = f;
    }
}

// ---------------------------------------------------------------- cluster
// 16x16 fine tiles marked by any flagged coarse cell under them, kept if their
// coarse footprint grown by two coarse cells (clipped at the domain) lies inside
// the coarse level's coverage, then merged row-major into rectangles of at most
// 4x4 tiles.  Boxes are returned in fine index space.
static int cluster(const Hier& H, int l, const uint8_t* flags, std::vector<int>& boxes) {
  const Level& L = H.L[l];
  const int r = H.ratio[l];
  const int T = 16;
  const int nxf = L.G.nx * r, nyf = L.G.ny * r;
  const int ntx = (nxf + T - 1) / T, nty = (nyf + T - 1) / T;
  std::vector<uint8_t> keep(size_t(ntx) * nty, 0), used(size_t(ntx) * nty, 0);
  for (int J = 0; J < nty; ++J)
    for (int I = 0; I < ntx; ++I) {
      int i0 = (T * I) / r, i1 = std::min(L.G.nx, (T * (I + 1) + r - 1) / r);
      int j0 = (T * J) / r, j1 = std::min(L.G.ny, (T * (J + 1) + r - 1) / r);
      bool marked = false;
      for (int j = j0; j < j1 && !marked; ++j)
        for (int i = i0; i < i1; ++i)
          if (flags[size_t(j) * L.G.nx + i]) { marked = true; break; }
      if (!marked) continue;
      bool nested = true;
      for (int j = std::max(0, j0 - 2); j < std::min(L.G.ny, j1 + 2) && nested; ++j)
        for (int i = std::max(0, i0 - 2); i < std::min(L.G.nx, i1 + 2); ++i)
          if (!L.mask[L.G.idx(i, j)]) { nested = false; break; }
      keep[size_t(J) * ntx + I] = nested ? 1 : 0;
    }
  boxes.clear();
  auto avail = [&](int I, int J) { return keep[size_t(J) * ntx + I] && !used[size_t(J) * ntx + I]; };
  for (int J = 0; J < nty; ++J)
    for (int I = 0; I < ntx; ++I) {
      if (!avail(I, J)) continue;
      int w = 1;
      while (w < 4 && I + w < ntx && avail(I + w, J)) ++w;
      int h = 1;
      while (h < 4 && J + h < nty) {
        bool row = true;
        for (int k = 0; k < w; ++k)
          if (!avail(I + k, J + h)) { row = false; break; }
        if (!row) break;
        ++h;
      }
      for (int jj = 0; jj < h; ++jj)
        for (int k = 0; k < w; ++k) used[size_t(J + jj) * ntx + I + k] = 1;
      int ilo = T * I, jlo = T * J;
      int ihi = std::min(nxf, T * (I + w)), jhi = std::min(nyf, T * (J + h));
      boxes.push_back(ilo); boxes.push_back(jlo);
      boxes.push_back(ihi - ilo); boxes.push_back(jhi - jlo);
    }
  return int(boxes.size() / 4);
}

static int regrid(Hier& H, const double* tau, int nbuf) {
  for (int l = 0; l + 1 < H.nlev; ++l) {
    const Level& L = H.L[l];
    std::vector<uint8_t> f(size_t(L.G.nx) * L.G.ny);
    flag(H, l, tau[l], nbuf, f.data());
    std::vector<int> bx;
    int n = cluster(H, l, f.data(), bx);
    int rc = set_patches(H, l + 1, n, bx.data());
    if (rc) return rc;
  }
  return OK;
}

// ---------------------------------------------------------------- time step rule
static double initial_dt(const Hier& H) {
  double best = std::numeric_limits<double>::infinity();
  double fac = 1.0;
  for (int l = 0; l < H.nlev; ++l) {
    const Level& L = H.L[l];
    if (l > 0) fac *= H.ratio[l - 1];
    if (L.boxes.empty()) continue;
    const double* q = L.q[L.cur].data();
    const size_t pl = L.G.plane();
    double smx = 0.0;
    for (const Box& b : L.boxes)
      for (int j = b.jlo; j < b.jlo + b.ny; ++j)
        for (int i = b.ilo; i < b.ilo + b.nx; ++i) {
          size_t k = L.G.idx(i, j);
          double h1 = q[F_H1 * pl + k], h2 = q[F_H2 * pl + k];
          double vm = 0.0;
          if (h1 >= H.P.hdry) {
            double inv = 1.0 / h1;
            vm = std::max(vm, std::max(std::fabs(q[F_HU1 * pl + k] * inv), std::fabs(q[F_HV1 * pl + k] * inv)));
          }
          if (h2 >= H.P.hdry) {
            double inv = 1.0 / h2;
            vm = std::max(vm, std::max(std::fabs(q[F_HU2 * pl + k] * inv), std::fabs(q[F_HV2 * pl + k] * inv)));
          }
          if (h1 >= H.P.hdry || h2 >= H.P.hdry) {
            double s = vm + std::sqrt(H.P.g * (h1 + h2));
            if (s > smx) smx = s;
          }
        }
    if (smx > 0.0) best = std::min(best, fac * ((H.cfl * std::min(L.dx, L.dy)) / smx));
  }
  return best;
}

static double next_dt(const Hier& H) {
  if (!H.have_smax) return initial_dt(H);
  double best = std::numeric_limits<double>::infinity();
  double fac = 1.0;
  for (int l = 0; l < H.nlev; ++l) {
    const Level& L = H.L[l];
    if (l > 0) fac *= H.ratio[l - 1];
    double a = L.smax[0] > 0.0 ? L.dx / L.smax[0] : std::numeric_limits<double>::infinity();
    double b = L.smax[1] > 0.0 ? L.dy / L.smax[1] : std::numeric_limits<double>::infinity();
    double m = std::min(a, b);
    if (m < std::numeric_limits<double>::infinity()) best = std::min(best, fac * (H.cfl * m));
  }
  return best;
}

// ---------------------------------------------------------------- flux correction
// Mass flux correction at coarse-fine edges (the paper is silent; optional).  A
// coarse cell O of level l outside the finer level, with a face neighbour N
// covered by it, took the coarse mass flux Gc through the face O|N in its own
// update; the fine cells along that face took the fine fluxes of the r fine
// faces in each of the r fine substeps.  After coarsening, O's depths get
// nu_c (Gc - (sum of the fine fluxes) / r^2), added when O lies left of (below)
// the face and subtracted when it lies right of (above) it, so each layer's
// mass on the composite grid changes only through the domain walls.  Faces in
// the order +x, -x, +y, -y; the fine fluxes of a substep summed along the face
// first, then added to the running sum.
struct RefluxCell {
  int i, j, dirs;  // dirs bit d: face neighbour in direction d is covered by the finer level
  double gc[4][2], acc[4][2];
};

static std::vector<RefluxCell> reflux_begin(const Hier& H, int l) {
  const Level& L = H.L[l];
  const Level& F = H.L[l + 1];
  const int r = H.ratio[l];
  const size_t pl = L.G.plane();
  auto fine = [&](int I, int J) {
    return I >= 0 && J >= 0 && I < L.G.nx && J < L.G.ny && F.mask[F.G.idx(r * I, r * J)] != 0;
  };
  static const int di[4] = {1, -1, 0, 0}, dj[4] = {0, 0, 1, -1};
  static const int plane_of[4] = {2, 0, 6, 4};  // O's flux through the face: right, left, upper, lower
  std::vector<RefluxCell> out;
  for (int j = 0; j < L.G.ny; ++j)
    for (int i = 0; i < L.G.nx; ++i) {
      const size_t id = L.G.idx(i, j);
      if (!L.mask[id] || fine(i, j)) continue;
      RefluxCell c{};
      c.i = i; c.j = j; c.dirs = 0;
      for (int d = 0; d < 4; ++d) {
        if (!fine(i + di[d], j + dj[d])) continue;
        c.dirs |= 1 << d;
        for (int m = 0; m < 2; ++m) {
          c.gc[d][m] = L.mflux[(plane_of[d] + m) * pl + id];
          c.acc[d][m] = 0.0;
        }
      }
      if (c.dirs) out.push_back(c);
    }
  return out;
}

// After a fine substep: add the fine fluxes through each recorded face.
static void reflux_accumulate(const Hier& H, int l, std::vector<RefluxCell>& cells) {
  const Level& F = H.L[l + 1];
  const int r = H.ratio[l];
  const size_t pl = F.G.plane();
  static const int plane_of[4] = {0, 2, 4, 6};  // the fine cells' flux through the face: left, right, lower, upper
  for (RefluxCell& c : cells)
    for (int d = 0; d < 4; ++d) {
      if (!(c.dirs >> d & 1)) continue;
      for (int m = 0; m < 2; ++m) {
        double s = 0.0;
        for (int k = 0; k < r; ++k) {
          int fi, fj;
          if (d == 0) { fi = r * (c.i + 1); fj = r * c.j + k; }
          else if (d == 1) { fi = r * c.i - 1; fj = r * c.j + k; }
          else if (d == 2) { fi = r * c.i + k; fj = r * (c.j + 1); }
          else { fi = r * c.i + k; fj = r * c.j - 1; }
          const double g = F.mflux[(plane_of[d] + m) * pl + F.G.idx(fi, fj)];
          s = k == 0 ? g : s + g;
        }
        c.acc[d][m] = c.acc[d][m] + s;
      }
    }
}

static void reflux_apply(Hier& H, int l, const std::vector<RefluxCell>& cells, double dt) {
  Level& L = H.L[l];
  const double inv = 1.0 / double(H.ratio[l] * H.rt[l]);  // r fine faces in each of rt substeps
  const double nux = dt / L.dx, nuy = dt / L.dy;
  double* q = L.q[L.cur].data();
  const size_t pl = L.G.plane();
  for (const RefluxCell& c : cells) {
    const size_t id = L.G.idx(c.i, c.j);
    for (int d = 0; d < 4; ++d) {
      if (!(c.dirs >> d & 1)) continue;
      const double nu = d < 2 ? nux : nuy;
      for (int m = 0; m < 2; ++m) {
        const double corr = nu * (c.gc[d][m] - c.acc[d][m] * inv);
        double& h = q[(m == 0 ? F_H1 : F_H2) * pl + id];
        h = (d % 2 == 0) ? h + corr : h - corr;
      }
    }
  }
}

// ---------------------------------------------------------------- time ratio
// Time-refinement ratios of a coarse step of length dt (Sec. 2, text after Eq.
// 2).  By default each equals the space ratio.  With the dynamic choice on and
// speeds of a last coarse step known, level l (>= 1) takes the fewest substeps
// per substep of level l - 1, at most the space ratio, that keep its substep
// within the Courant limit of its own last speeds and leave every finer level
// able to meet its own with full ratios: with a_l = cfl * min(dx / sx, dy / sy)
// of the last coarse step (infinite without speeds) and A_l = min(a_l, r_l
// A_{l+1}) from the finest level up, rt = ceil(dt_{l-1} / A_l) clipped to [1, r].
static void choose_rt(Hier& H, double dt) {
  for (int l = 0; l + 1 < H.nlev; ++l) H.rt[l] = H.ratio[l];
  if (!H.dyn_rt || !H.have_smax) return;
  // A level with patches but no speeds of the last coarse step (one a regrid
  // has just populated) has no Courant bound of its own: then every level keeps
  // its space ratio, as on the first step, so that the new level's substep is
  // no longer than with fixed ratios.
  for (int l = 1; l < H.nlev; ++l)
    if (!H.L[l].boxes.empty() && !(H.L[l].smax[0] > 0.0) && !(H.L[l].smax[1] > 0.0)) return;
  const double inf = std::numeric_limits<double>::infinity();
  double A[8];
  for (int l = H.nlev - 1; l >= 0; --l) {
    const Level& L = H.L[l];
    const double a = L.smax[0] > 0.0 ? L.dx / L.smax[0] : inf;
    const double b = L.smax[1] > 0.0 ? L.dy / L.smax[1] : inf;
    const double m = std::min(a, b);
    const double al = m < inf ? H.cfl * m : inf;
    A[l] = l + 1 < H.nlev ? std::min(al, double(H.ratio[l]) * A[l + 1]) : al;
  }
  double dtp = dt;
  for (int l = 1; l < H.nlev; ++l) {
    const double q = dtp / A[l];
    int k = H.ratio[l - 1];
    if (q < double(k)) {
      const double c = std::ceil(q);
      k = c < 1.0 ? 1 : int(c);
    }
    H.rt[l - 1] = k;
    dtp = dtp / double(k);
  }
}

// Subcycled recursion: fill and step level l, then rt substeps of level l+1
// (the time ratio of this coarse step), then average level l+1 back onto level l
// (and, with the flux correction on, correct the coarse cells beside it).
// A substep above the Courant limit does not stop the step: the whole coarse
// step is completed and judged by its largest substep Courant number.
static int adv(Hier& H, int l, double dt, double th) {
  double s[2];
  int rc = step_level(H, l, dt, th, s);
  if (rc && rc != E_CFL) return rc;
  if (l + 1 < H.nlev && !H.L[l + 1].boxes.empty()) {
    const int r = H.rt[l];
    const double dtf = dt / double(r);
    std::vector<RefluxCell> rf;
    if (H.reflux) rf = reflux_begin(H, l);
    for (int k = 0; k < r; ++k) {
      rc = adv(H, l + 1, dtf, double(k) / double(r));
      if (rc && rc != E_CFL) return rc;
      if (H.reflux) reflux_accumulate(H, l, rf);
    }
    coarsen(H, l + 1);
    if (H.reflux) reflux_apply(H, l, rf, dt);
  }
  return OK;
}

// Coarse steps with rejection: a step whose largest substep Courant number
// exceeds cflmax is undone and retaken with dt scaled by cfl / (that number).
static int advance(Hier& H, int nsteps, int regrid_every, const double* tau, int nbuf, double* dts) {
  for (int n = 0; n < nsteps; ++n) {
    if (regrid_every > 0 && n % regrid_every == 0) {
      int rc = regrid(H, tau, nbuf);
      if (rc) return rc;
    }
    double dt = next_dt(H);
    choose_rt(H, dt);
    std::vector<std::vector<double>> save(H.nlev);
    std::vector<int> save_cur(H.nlev);
    Counters save_c = H.C;
    int64_t save_u[8];
    std::copy(H.updates, H.updates + 8, save_u);
    for (int l = 0; l < H.nlev; ++l) { save[l] = H.L[l].q[H.L[l].cur]; save_cur[l] = H.L[l].cur; }
    for (int attempt = 0;; ++attempt) {
      for (int l = 0; l < H.nlev; ++l) { H.L[l].smax[0] = 0.0; H.L[l].smax[1] = 0.0; }
      H.cmax = 0.0;
      int rc = adv(H, 0, dt, 0.0);
      if (rc) return rc;
      if (H.cmax <= H.cflmax) break;
      if (attempt + 1 > H.retries || !(H.cmax == H.cmax)) return E_CFL;
      for (int l = 0; l < H.nlev; ++l) { H.L[l].cur = save_cur[l]; H.L[l].q[save_cur[l]] = save[l]; }
      H.C = save_c;
      std::copy(save_u, save_u + 8, H.updates);
      H.rejected++;
      dt = dt * (H.cfl / H.cmax);
    }
    H.have_smax = true;
    H.t += dt;
    if (dts) dts[n] = dt;
  }
  return OK;
}

}  // namespace ora

// ================================================================ C interface
using namespace ora;

extern "C" {

void* ora_create(double g, double r, double hdry, double kmin, double cfl, double cflmax, int nlev,
                 const int* ratios, int nx0, int ny0, double dx0, double dy0) {
  // two reflecting ghost cells need at least two cells across the domain
  if (nlev < 1 || nlev > 8 || nx0 < 2 || ny0 < 2) return nullptr;
  Hier* H = new Hier;
  H->P = make_params(g, r, hdry, kmin);
  H->cfl = cfl; H->cflmax = cflmax;
  H->nlev = nlev;
  H->L.resize(nlev);
  int nx = nx0, ny = ny0;
  double dx = dx0, dy = dy0;
  for (int l = 0; l < nlev; ++l) {
    if (l > 0) {
      H->ratio[l - 1] = ratios[l - 1];
      H->rt[l - 1] = ratios[l - 1];
      nx *= ratios[l - 1]; ny *= ratios[l - 1];
      dx = dx / ratios[l - 1]; dy = dy / ratios[l - 1];
    }
    alloc_level(H->L[l], nx, ny, dx, dy);
  }
  // level 0 is one patch over the whole domain unless set otherwise
  H->L[0].boxes.push_back(Box{0, 0, nx0, ny0});
  rebuild_mask(H->L[0]);
  return H;
}

void ora_destroy(void* h) { delete static_cast<Hier*>(h); }

int ora_level_shape(void* h, int l, int* nx, int* ny, double* dx, double* dy) {
  Hier* H = static_cast<Hier*>(h);
  if (l < 0 || l >= H->nlev) return E_INVAL;
  *nx = H->L[l].G.nx; *ny = H->L[l].G.ny; *dx = H->L[l].dx; *dy = H->L[l].dy;
  return OK;
}

int ora_set_bathymetry(void* h, const double* Bf) {
  build_bathymetry(*static_cast<Hier*>(h), Bf);
  return OK;
}

int ora_get_bathymetry(void* h, int l, double* B) {
  Hier* H = static_cast<Hier*>(h);
  if (l < 0 || l >= H->nlev) return E_INVAL;
  const Level& L = H->L[l];
  for (int j = 0; j < L.G.ny; ++j)
    for (int i = 0; i < L.G.nx; ++i) B[size_t(j) * L.G.nx + i] = L.B[L.G.idx(i, j)];
  return OK;
}

// State of a level, [6][ny][nx]; written over the level's current buffer.
int ora_set_state(void* h, int l, const double* q) {
  Hier* H = static_cast<Hier*>(h);
  if (l < 0 || l >= H->nlev) return E_INVAL;
  Level& L = H->L[l];
  const size_t pl = L.G.plane();
  for (int c = 0; c < 6; ++c)
    for (int j = 0; j < L.G.ny; ++j)
      for (int i = 0; i < L.G.nx; ++i)
        L.q[L.cur][c * pl + L.G.idx(i, j)] = q[(size_t(c) * L.G.ny + j) * L.G.nx + i];
  return OK;
}

// State of a level, [6][ny][nx]; cells not covered by a patch read NaN.
int ora_get_state(void* h, int l, double* q) {
  Hier* H = static_cast<Hier*>(h);
  if (l < 0 || l >= H->nlev) return E_INVAL;
  const Level& L = H->L[l];
  const size_t pl = L.G.plane();
  const double nan = std::numeric_limits<double>::quiet_NaN();
  for (int c = 0; c < 6; ++c)
    for (int j = 0; j < L.G.ny; ++j)
      for (int i = 0; i < L.G.nx; ++i) {
        size_t k = L.G.idx(i, j);
        q[(size_t(c) * L.G.ny + j) * L.G.nx + i] = L.mask[k] ? L.q[L.cur][c * pl + k] : nan;
      }
  return OK;
}

int ora_set_patches(void* h, int l, int n, const int* boxes) {
  Hier* H = static_cast<Hier*>(h);
  if (l < 0 || l >= H->nlev || n < 0) return E_INVAL;
  return set_patches(*H, l, n, boxes);
}

int ora_get_npatches(void* h, int l) {
  Hier* H = static_cast<Hier*>(h);
  if (l < 0 || l >= H->nlev) return E_INVAL;
  return int(H->L[l].boxes.size());
}

int ora_get_patches(void* h, int l, int* boxes) {
  Hier* H = static_cast<Hier*>(h);
  if (l < 0 || l >= H->nlev) return E_INVAL;
  int k = 0;
  for (const Box& b : H->L[l].boxes) {
    boxes[k++] = b.ilo; boxes[k++] = b.jlo; boxes[k++] = b.nx; boxes[k++] = b.ny;
  }
  return int(H->L[l].boxes.size());
}

int ora_step_level(void* h, int l, double dt, double th, double* smax) {
  Hier* H = static_cast<Hier*>(h);
  if (l < 0 || l >= H->nlev) return E_INVAL;
  double s[2];
  int rc = step_level(*H, l, dt, th, s);
  if (smax) { smax[0] = s[0]; smax[1] = s[1]; }
  return rc;
}

int ora_coarsen(void* h, int lf) {
  Hier* H = static_cast<Hier*>(h);
  if (lf < 1 || lf >= H->nlev) return E_INVAL;
  coarsen(*H, lf);
  return OK;
}

int ora_flag(void* h, int l, double tau, int nbuf, unsigned char* out) {
  Hier* H = static_cast<Hier*>(h);
  if (l < 0 || l >= H->nlev) return E_INVAL;
  flag(*H, l, tau, nbuf, out);
  return OK;
}

int ora_cluster(void* h, int l, const unsigned char* flags, int* boxes, int cap) {
  Hier* H = static_cast<Hier*>(h);
  if (l < 0 || l + 1 >= H->nlev) return E_INVAL;
  std::vector<int> bx;
  int n = cluster(*H, l, flags, bx);
  if (n > cap) return E_INVAL;
  std::copy(bx.begin(), bx.end(), boxes);
  return n;
}

int ora_regrid(void* h, const double* tau, int nbuf) { return regrid(*static_cast<Hier*>(h), tau, nbuf); }

int ora_advance(void* h, int nsteps, int regrid_every, const double* tau, int nbuf, double* dts) {
  return advance(*static_cast<Hier*>(h), nsteps, regrid_every, tau, nbuf, dts);
}

double ora_next_dt(void* h) { return next_dt(*static_cast<Hier*>(h)); }

void ora_set_reflux(void* h, int on) { static_cast<Hier*>(h)->reflux = on != 0; }

void ora_set_dynamic_rt(void* h, int on) { static_cast<Hier*>(h)->dyn_rt = on != 0; }

// Rejected coarse steps are retaken at most n times (n < 0: never).
void ora_set_retries(void* h, int n) { static_cast<Hier*>(h)->retries = n < 0 ? 0 : n; }

// Test hooks: the ghost fill of level l at time fraction th on its own, and a
// level's raw buffers with their frames (which = 0: current, 1: the other one,
// i.e. the state before the level's last step), [6][ny + 4][nx + 4].
void ora_ghost_fill(void* h, int l, double th) { ghost_fill(*static_cast<Hier*>(h), l, th); }

void ora_get_level_raw(void* h, int l, int which, double* out) {
  const Level& L = static_cast<Hier*>(h)->L[l];
  const std::vector<double>& q = L.q[which ? 1 - L.cur : L.cur];
  std::copy(q.begin(), q.end(), out);
}

double ora_mc_limiter(double th) { return mc_limiter<double>(th); }

// Time ratios of the last coarse step: out[nlev - 1].
void ora_get_rt(void* h, int* out) {
  Hier* H = static_cast<Hier*>(h);
  for (int l = 0; l + 1 < H->nlev; ++l) out[l] = H->rt[l];
}

// Time-stepping state for checkpoint and resume: t, whether the next coarse
// step takes its dt from the last step's speeds (else from the state), and each
// level's largest x / y speeds over the last coarse step.  out / in:
// [2 + 2 * nlev].
void ora_get_step_state(void* h, double* out) {
  Hier* H = static_cast<Hier*>(h);
  out[0] = H->t;
  out[1] = H->have_smax ? 1.0 : 0.0;
  for (int l = 0; l < H->nlev; ++l) { out[2 + 2 * l] = H->L[l].smax[0]; out[3 + 2 * l] = H->L[l].smax[1]; }
}

void ora_set_step_state(void* h, const double* in) {
  Hier* H = static_cast<Hier*>(h);
  H->t = in[0];
  H->have_smax = in[1] != 0.0;
  for (int l = 0; l < H->nlev; ++l) { H->L[l].smax[0] = in[2 + 2 * l]; H->L[l].smax[1] = in[3 + 2 * l]; }
}

// [hyp, nclip, repair, clip1, clip2, t, updates level 0..7, rejected steps]
void ora_counters(void* h, double* out) {
  Hier* H = static_cast<Hier*>(h);
  out[0] = double(H->C.hyp); out[1] = double(H->C.nclip); out[2] = double(H->C.repair);
  out[3] = H->C.clip1; out[4] = H->C.clip2; out[5] = H->t;
  for (int l = 0; l < 8; ++l) out[6 + l] = double(H->updates[l]);
  out[14] = double(H->rejected);
}

// Refine one fine cell from explicit coarse data: q5 = 5 cells x 7 values
// (h1 hu1 hv1 h2 hu2 hv2 B) for centre, left, right, down, up; inx / iny say
// whether the x / y neighbours exist (a missing pair means the centre touches the
// domain edge in that direction).  Returns the number of wet-order repairs.
int ora_refine_point(double hdry, int r, int a, int b, const double* q5, int inx, int iny, double Bf,
                     double* out) {
  Params P = make_params(9.81, 0.95, hdry, 1e-6);
  const int nx = inx ? 3 : 1, ny = iny ? 3 : 1;
  const int I = inx ? 1 : 0, J = iny ? 1 : 0;
  Level L;
  alloc_level(L, nx, ny, 1.0, 1.0);
  const int off[5][2] = {{0, 0}, {-1, 0}, {1, 0}, {0, -1}, {0, 1}};
  for (int k = 0; k < 5; ++k) {
    int i = I + off[k][0], j = J + off[k][1];
    if (i < 0 || j < 0 || i >= nx || j >= ny) continue;
    size_t id = L.G.idx(i, j);
    for (int c = 0; c < 6; ++c) L.q[0][c * L.G.plane() + id] = q5[7 * k + c];
    L.B[id] = q5[7 * k + 6];
  }
  CoarseSrc S{&L, L.q[0].data(), L.q[0].data(), 0.0};
  Counters C;
  refine_cell(P, S, r, I, J, a, b, Bf, out, C);
  return int(C.repair);
}

// Single-edge solve for unit tests.  qL/qR: h1 m1 t1 h2 m2 t2 B (normal momentum m,
// transverse t).  Outputs 6 speeds, 6x6 waves, 6 modes, A-dQ and A+dQ.
int ora_riemann(double g, double r, double hdry, double kmin, const double* qL, const double* qR,
                double* s, double* Z, int* mode, double* amdq, double* apdq) {
  Params P = make_params(g, r, hdry, kmin);
  CellV<double> L = make_cell<double>(P, qL, qL[6]);
  CellV<double> R = make_cell<double>(P, qR, qR[6]);
  Waves<double> W;
  Counters C;
  riemann(P, L, R, W, C, true);
  for (int p = 0; p < 6; ++p) {
    s[p] = W.s[p];
    mode[p] = W.mode[p];
    for (int c = 0; c < 6; ++c) Z[6 * p + c] = W.Z[p][c];
  }
  fluctuations(W, amdq, apdq);
  return int(C.hyp);
}

// Fixed-grid wall-bounded run with a frozen dt sequence, in double; used by the
// pins (conservation, symmetry) without the level machinery.
int ora_fixed_steps(int nx, int ny, double dx, double dy, double g, double r, double hdry, double kmin,
                    const double* Bi, double* q /*[6][ny][nx] in/out*/, int nsteps, const double* dts,
                    double* smax /*[2*nsteps] or null*/, double* cnt /*[5] or null*/) {
  Params P = make_params(g, r, hdry, kmin);
  Grid G; G.nx = nx; G.ny = ny;
  const size_t pl = G.plane();
  std::vector<double> a(6 * pl, 0.0), b(6 * pl, 0.0), B(pl, 0.0);
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      B[G.idx(i, j)] = Bi[size_t(j) * nx + i];
      for (int c = 0; c < 6; ++c) a[c * pl + G.idx(i, j)] = q[(size_t(c) * ny + j) * nx + i];
    }
  wall_fill_B(G, B.data());
  Counters C;
  Box bx{0, 0, nx, ny};
  for (int n = 0; n < nsteps; ++n) {
    wall_fill_all(G, a.data());
    double s[2];
    step_box(P, G, a.data(), B.data(), bx, dx, dy, dts[n], b.data(), s, C);
    std::swap(a, b);
    if (smax) { smax[2 * n] = s[0]; smax[2 * n + 1] = s[1]; }
  }
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i)
      for (int c = 0; c < 6; ++c) q[(size_t(c) * ny + j) * nx + i] = a[c * pl + G.idx(i, j)];
  if (cnt) { cnt[0] = double(C.hyp); cnt[1] = double(C.nclip); cnt[2] = double(C.repair); cnt[3] = C.clip1; cnt[4] = C.clip2; }
  return OK;
}

// Wall-clock rate of the oracle's fixed-grid step (cell updates per second) on an
// nx x ny wall-bounded grid, for the benchmark's CPU baseline.
double ora_time_fixed(int nx, int ny, double dx, double dy, double g, double r, double hdry, double kmin,
                      const double* Bi, const double* q0, int nsteps, double dt, double* seconds) {
  Params P = make_params(g, r, hdry, kmin);
  Grid G; G.nx = nx; G.ny = ny;
  const size_t pl = G.plane();
  std::vector<double> a(6 * pl, 0.0), b(6 * pl, 0.0), B(pl, 0.0);
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      B[G.idx(i, j)] = Bi[size_t(j) * nx + i];
      for (int c = 0; c < 6; ++c) a[c * pl + G.idx(i, j)] = q0[(size_t(c) * ny + j) * nx + i];
    }
  wall_fill_B(G, B.data());
  Counters C;
  Box bx{0, 0, nx, ny};
  auto t0 = std::chrono::steady_clock::now();
  for (int n = 0; n < nsteps; ++n) {
    wall_fill_all(G, a.data());
    double s[2];
    step_box(P, G, a.data(), B.data(), bx, dx, dy, dt, b.data(), s, C);
    std::swap(a, b);
  }
  auto t1 = std::chrono::steady_clock::now();
  double sec = std::chrono::duration<double>(t1 - t0).count();
  if (seconds) *seconds = sec;
  return double(nx) * ny * nsteps / sec;
}

// The same stepping with nthreads host threads, the paper's multi-threaded
// mode (Sec. 3 times its runs with one and with four threads): each step cuts
// the level into nthreads strips of whole rows and steps every strip as a box
// of its own on its own thread (frame rows come from the neighbouring strips of
// the full state, as for any patch), so the results are those of the one-box
// step bit for bit.  q_out (nullable, [6][ny][nx]) receives the final state.
double ora_time_fixed_mt(int nx, int ny, double dx, double dy, double g, double r, double hdry, double kmin,
                         const double* Bi, const double* q0, int nsteps, double dt, int nthreads, double* seconds,
                         double* q_out) {
  Params P = make_params(g, r, hdry, kmin);
  Grid G; G.nx = nx; G.ny = ny;
  const size_t pl = G.plane();
  std::vector<double> a(6 * pl, 0.0), b(6 * pl, 0.0), B(pl, 0.0);
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      B[G.idx(i, j)] = Bi[size_t(j) * nx + i];
      for (int c = 0; c < 6; ++c) a[c * pl + G.idx(i, j)] = q0[(size_t(c) * ny + j) * nx + i];
    }
  wall_fill_B(G, B.data());
  const int nt = std::max(1, std::min(nthreads, ny));
  std::vector<Counters> C(nt);
  auto t0 = std::chrono::steady_clock::now();
  for (int n = 0; n < nsteps; ++n) {
    wall_fill_all(G, a.data());
    std::vector<std::thread> pool;
    for (int t = 0; t < nt; ++t) {
      const int j0 = int((long long)ny * t / nt), j1 = int((long long)ny * (t + 1) / nt);
      pool.emplace_back([&, t, j0, j1] {
        double s[2];
        step_box(P, G, a.data(), B.data(), Box{0, j0, nx, j1 - j0}, dx, dy, dt, b.data(), s, C[t]);
      });
    }
    for (std::thread& th : pool) th.join();
    std::swap(a, b);
  }
  auto t1 = std::chrono::steady_clock::now();
  double sec = std::chrono::duration<double>(t1 - t0).count();
  if (seconds) *seconds = sec;
  if (q_out)
    for (int c = 0; c < 6; ++c)
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) q_out[(size_t(c) * ny + j) * nx + i] = a[c * pl + G.idx(i, j)];
  return double(nx) * ny * nsteps / sec;
}

}  // extern "C"

extern "C" {

// One step of the sub-box `box` (ilo, jlo, nx, ny) of a wall-bounded single
// level whose full state is given: frame cells of the box come from the
// neighbouring cells of the level or, outside the domain, from the walls.
// Writes the box's new state, [6][box ny][box nx].  Lets a test check sampled
// windows of a grid too large for a full oracle step.
int ora_step_window(int nx, int ny, double dx, double dy, double g, double r, double hdry, double kmin,
                    const double* Bi, const double* q, const int* box, double dt, double* out,
                    double* smax) {
  Params P = make_params(g, r, hdry, kmin);
  const int bi = box[0], bj = box[1], bnx = box[2], bny = box[3];
  if (bi < 0 || bj < 0 || bnx <= 0 || bny <= 0 || bi + bnx > nx || bj + bny > ny) return E_INVAL;
  // local level = window grown by 2 cells, clipped to the domain; cells beyond the
  // domain are mirror images
  Grid G; G.nx = nx; G.ny = ny;
  const int x0 = bi - 2, y0 = bj - 2, wx = bnx + 4, wy = bny + 4;
  Grid W; W.nx = wx - 4; W.ny = wy - 4;  // frame of W holds the window's ghosts
  const size_t pl = W.plane();
  std::vector<double> a(6 * pl, 0.0), b(6 * pl, 0.0), B(pl, 0.0);
  for (int jj = 0; jj < wy; ++jj)
    for (int ii = 0; ii < wx; ++ii) {
      int i = x0 + ii, j = y0 + jj;
      int si, sj; bool fx, fy;
      mirror_src(G, i, j, si, sj, fx, fy);
      size_t k = W.idx(ii - 2, jj - 2);
      B[k] = Bi[size_t(sj) * nx + si];
      for (int c = 0; c < 6; ++c) {
        double v = q[(size_t(c) * ny + sj) * nx + si];
        if ((fx && (c == F_HU1 || c == F_HU2)) || (fy && (c == F_HV1 || c == F_HV2))) v = 0.0 - v;
        a[c * pl + k] = v;
      }
    }
  Counters C;
  Box bx{0, 0, bnx, bny};
  double s[2];
  step_box(P, W, a.data(), B.data(), bx, dx, dy, dt, b.data(), s, C);
  for (int c = 0; c < 6; ++c)
    for (int j = 0; j < bny; ++j)
      for (int i = 0; i < bnx; ++i) out[(size_t(c) * bny + j) * bnx + i] = b[c * pl + W.idx(i, j)];
  if (smax) { smax[0] = s[0]; smax[1] = s[1]; }
  return OK;
}

}  // extern "C"
