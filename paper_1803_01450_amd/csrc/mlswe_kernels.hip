// HIP kernels (gfx950) of the two-layer shallow-water step and the multilayer
// AMR operators.  Level arrays are dense per (problem, level), field-major SoA
// with a two-cell frame; row j, column i sits at (j + 2) * pitch + (i + XOFF),
// XOFF = 8 so that interior rows start on a 64-byte boundary.
#include "mlswe_kernels.hpp"

namespace mlswe {

__device__ __forceinline__ long long cidx(long long pitch, int i, int j) {
  return (long long)(j + 2) * pitch + (long long)(i + XOFF);
}

// ---------------------------------------------------------------- wave helpers
__device__ __forceinline__ double shup(double v) { return __shfl_up(v, 1, 64); }
__device__ __forceinline__ double shdn(double v) { return __shfl_down(v, 1, 64); }
__device__ __forceinline__ int shup_i(int v) { return __shfl_up(v, 1, 64); }

__device__ __forceinline__ CellX shup_cell(const CellX& c) {
  CellX o;
  o.h1 = shup(c.h1); o.m1 = shup(c.m1); o.t1 = shup(c.t1);
  o.h2 = shup(c.h2); o.m2 = shup(c.m2); o.t2 = shup(c.t2); o.B = shup(c.B);
  o.u1 = shup(c.u1); o.w1 = shup(c.w1); o.u2 = shup(c.u2); o.w2 = shup(c.w2);
  o.s1 = shup(c.s1); o.s2 = shup(c.s2); o.e1 = shup(c.e1); o.e2 = shup(c.e2);
  int f = shup_i((c.wet1 ? 1 : 0) | (c.wet2 ? 2 : 0));
  o.wet1 = (f & 1) != 0; o.wet2 = (f & 2) != 0;
  return o;
}

__device__ __forceinline__ EdgeW shup_edge(const EdgeW& w) {
  EdgeW o;
#pragma unroll
  for (int p = 0; p < 6; ++p) o.s[p] = shup(w.s[p]);
#pragma unroll
  for (int p = 0; p < 4; ++p) { o.A[p] = shup(w.A[p]); o.C[p] = shup(w.C[p]); }
  o.v1 = shup(w.v1); o.v2 = shup(w.v2); o.z4 = shup(w.z4); o.z5 = shup(w.z5);
  int m = shup_i(w.mode1 | (w.mode2 << 4));
  o.mode1 = m & 15; o.mode2 = m >> 4;
  return o;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) { double t = __shfl_xor(v, o, 64); v = t > v ? t : v; }
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ int wave_isum(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ void flush_counts(Counters* cnt, LevelCtl* ctl, int axis, double smax, int hyp,
                                             const FixCount& K, int lane) {
  double sm = wave_max(smax);
  int h = wave_isum(hyp);
  int nc = wave_isum(K.nclip);
  int rp = wave_isum(K.repair);
  double c1 = wave_sum(K.clip1);
  double c2 = wave_sum(K.clip2);
  if (lane == 0) {
    atomicMax(&ctl->step_smax[axis], (unsigned long long)__double_as_longlong(sm));
    if (h) atomicAdd(&cnt->hyp, (unsigned long long)h);
    if (nc) atomicAdd(&cnt->nclip, (unsigned long long)nc);
    if (rp) atomicAdd(&cnt->repair, (unsigned long long)rp);
    if (c1 != 0.0) atomicAdd(&cnt->clip1, c1);
    if (c2 != 0.0) atomicAdd(&cnt->clip2, c2);
  }
}

// Branch code of wave p's limiter and speed sign at an edge, weighted by a hash
// of the edge position; sums of these over a run change (almost surely) when any
// limiter branch or wave direction changes.
__device__ __forceinline__ unsigned long long mix64(unsigned long long x) {
  x += 0x9e3779b97f4a7c15ull;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
  return x ^ (x >> 31);
}

__device__ __forceinline__ unsigned long long branch_sig(const EdgeW& W, const double dd[6], const double dl[6],
                                                         const double dr[6], int i, int j, int axis) {
  unsigned long long acc = 0;
#pragma unroll
  for (int p = 0; p < 6; ++p) {
    const double sv = W.s[p];
    unsigned code = sv > 0.0 ? 1u : (sv < 0.0 ? 2u : 3u);
    if (slot_mode(W, p) == 0 && sv != 0.0 && dd[p] != 0.0) {
      const double th = (sv > 0.0 ? dl[p] : dr[p]) / dd[p];
      const double a = 0.5 * (1.0 + th), b = 2.0 * th;
      const double m1 = a < 2.0 ? a : 2.0;
      const double m = m1 < b ? m1 : b;
      unsigned br = (0.0 > m) ? 1u : (m1 < b ? (a < 2.0 ? 2u : 3u) : 4u);
      code |= br << 2;
    }
    const unsigned long long key =
        ((unsigned long long)(unsigned)i << 32) ^ ((unsigned long long)(unsigned)j << 4) ^ (unsigned)(axis * 8 + p);
    acc += (unsigned long long)code * mix64(key);
  }
  return acc;
}

__device__ __forceinline__ unsigned long long wave_usum(unsigned long long v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double edge_smax(const EdgeW& W) {
  double m = 0.0;
#pragma unroll
  for (int p = 0; p < 6; ++p) {
    double a = W.s[p] < 0.0 ? 0.0 - W.s[p] : W.s[p];
    if (a > m) m = a;
  }
  return m;
}

// ---------------------------------------------------------------- x-sweep
// One wave per tile: lane l holds column i0 - 2 + l of each row; the edge at
// lane l lies between columns i0 - 3 + l and i0 - 2 + l.  Lanes 2..ncols+1 own
// the tile's interior cells.  Writes the x-swept, fixed-up state of the tile's
// rows (interior and frame rows of the patch) into the intermediate buffer.
__device__ __forceinline__ void sweep_x_tile(const PatchDev* __restrict__ patches, const XTile* __restrict__ tiles,
                                             int wv, int lane) {
  const XTile T = tiles[wv];
  const PatchDev& Pd = patches[T.patch];
  const PhysParams P = Pd.P;
  const long long pitch = Pd.pitch, plane = Pd.plane;
  const double* __restrict__ q = Pd.q;
  const double* __restrict__ Bp = Pd.B;
  double* __restrict__ qs = Pd.qs;
  const int c = T.i0 - 2 + lane;
  const bool act = lane < T.ncols + 4;
  const bool upd = lane >= 2 && lane < T.ncols + 2;
  const bool own = upd || (lane == T.ncols + 2 && T.i0 + T.ncols == Pd.ilo + Pd.nx);
  const double nu = Pd.ctl->dt / Pd.dx;
  double smax = 0.0;
  int hyp = 0;
  unsigned long long sig = 0;
  FixCount K = {0, 0, 0.0, 0.0};

  double nq[7];
  if (act) {
    const long long id = cidx(pitch, c, T.j0);
#pragma unroll
    for (int f = 0; f < 6; ++f) nq[f] = q[f * plane + id];
    nq[6] = Bp[id];
  } else {
#pragma unroll
    for (int f = 0; f < 7; ++f) nq[f] = 0.0;
  }
  for (int r = 0; r < T.nrows; ++r) {
    const int j = T.j0 + r;
    double cq[7];
#pragma unroll
    for (int f = 0; f < 7; ++f) cq[f] = nq[f];
    if (act && r + 1 < T.nrows) {  // prefetch the next row
      const long long id = cidx(pitch, c, j + 1);
#pragma unroll
      for (int f = 0; f < 6; ++f) nq[f] = q[f * plane + id];
      nq[6] = Bp[id];
    }
    const bool irow = j >= Pd.jlo && j < Pd.jlo + Pd.ny;
    CellX C = load_cell(P, cq[0], cq[1], cq[2], cq[3], cq[4], cq[5], cq[6]);
    CellX CL = shup_cell(C);
    EdgeW W;
    bool cl = riemann(P, CL, C, W);
    if (irow && own) {
      double e = edge_smax(W);
      smax = e > smax ? e : smax;
      hyp += cl ? 1 : 0;
    }
    double dd[6], dl[6], dr[6];
    EdgeW WL = shup_edge(W);
#pragma unroll
    for (int p = 0; p < 6; ++p) {
      dd[p] = wdot(W, W, p);
      dl[p] = wdot(WL, W, p);
    }
#pragma unroll
    for (int p = 0; p < 6; ++p) dr[p] = shdn(dl[p]);
    double coef[6], F[6], am[6], ap[6];
#pragma unroll
    for (int p = 0; p < 6; ++p) coef[p] = corr_coef(W, p, dd[p], dl[p], dr[p], nu);
    if (Pd.sig_on && own) sig += branch_sig(W, dd, dl, dr, c, j, 0);
    correction_flux(W, coef, F);
    fluctuations(W, am, ap);
    double gl[6], gr[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      gl[k] = ap[k] - F[k];
      gr[k] = shdn(am[k] + F[k]);
    }
    if (upd) {
      double o[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) o[k] = cq[k] - nu * (gl[k] + gr[k]);
      fixup(P, o, irow, K);
      const long long id = cidx(pitch, c, j);
#pragma unroll
      for (int f = 0; f < 6; ++f) qs[f * plane + id] = o[f];
    }
  }
  flush_counts(Pd.cnt, Pd.ctl, 0, smax, hyp, K, lane);
  if (Pd.sig_on) {
    sig = wave_usum(sig);
    if (lane == 0) atomicAdd(&Pd.cnt->sig, sig);
  }
}

// ---------------------------------------------------------------- y-sweep
// One wave per tile: lane l owns column i0 + l and marches up the rows
// j0 - 2 .. j0 + nrows + 1 of the intermediate state, keeping the last edge's
// waves in registers; row k is updated once the edges k, k + 1 and their
// neighbours are known.
__device__ __forceinline__ void sweep_y_tile(const PatchDev* __restrict__ patches, const YTile* __restrict__ tiles,
                                             int wv, int lane) {
  const YTile T = tiles[wv];
  const PatchDev& Pd = patches[T.patch];
  const PhysParams P = Pd.P;
  const long long pitch = Pd.pitch, plane = Pd.plane;
  const double* __restrict__ qs = Pd.qs;
  const double* __restrict__ Bp = Pd.B;
  double* __restrict__ qo = Pd.qo;
  const int i = T.i0 + lane;
  const bool act = lane < T.ncols;
  const double nu = Pd.ctl->dt / Pd.dy;
  double smax = 0.0;
  int hyp = 0;
  unsigned long long sig = 0;
  FixCount K = {0, 0, 0.0, 0.0};

  CellX Cp;
  EdgeW Wp;
  double qm2[6], qm1[6], ddp[6], dlp[6], glo[6];
  double nq[7];
  auto load_row = [&](int jj, double* v) {
    if (act) {
      const long long id = cidx(pitch, i, jj);
#pragma unroll
      for (int f = 0; f < 6; ++f) v[f] = qs[f * plane + id];
      v[6] = Bp[id];
    } else {
#pragma unroll
      for (int f = 0; f < 7; ++f) v[f] = 0.0;
    }
  };
  load_row(T.j0 - 2, nq);
  const int nk = T.nrows + 4;
  for (int k = 0; k < nk; ++k) {
    const int jj = T.j0 - 2 + k;
    double cq[7];
#pragma unroll
    for (int f = 0; f < 7; ++f) cq[f] = nq[f];
    if (k + 1 < nk) load_row(jj + 1, nq);
    // y orientation: normal momentum hv, transverse hu
    CellX Cc = load_cell(P, cq[0], cq[2], cq[1], cq[3], cq[5], cq[4], cq[6]);
    if (k >= 1) {
      EdgeW Wc;
      bool cl = riemann(P, Cp, Cc, Wc);
      const bool own = (jj >= T.j0 && jj < T.j0 + T.nrows) || (T.last && jj == T.j0 + T.nrows);
      if (own) {
        double e = edge_smax(Wc);
        smax = e > smax ? e : smax;
        hyp += cl ? 1 : 0;
      }
      double ddc[6];
#pragma unroll
      for (int p = 0; p < 6; ++p) ddc[p] = wdot(Wc, Wc, p);
      if (k >= 2) {
        double dlc[6];
#pragma unroll
        for (int p = 0; p < 6; ++p) dlc[p] = wdot(Wp, Wc, p);
        if (k >= 3) {
          // edge jj-1 is complete: its correction flux and fluctuations
          double coef[6], F[6], am[6], ap[6];
#pragma unroll
          for (int p = 0; p < 6; ++p) coef[p] = corr_coef(Wp, p, ddp[p], dlp[p], dlc[p], nu);
          if (Pd.sig_on && act) sig += branch_sig(Wp, ddp, dlp, dlc, i, jj - 1, 1);
          correction_flux(Wp, coef, F);
          fluctuations(Wp, am, ap);
          if (k >= 4 && act) {
            // row jj-2: lower edge jj-2 (glo), upper edge jj-1
            double o[6];
#pragma unroll
            for (int c = 0; c < 6; ++c) o[c] = qm2[c] - nu * (glo[c] + (am[c] + F[c]));
            fixup(P, o, true, K);
            const long long id = cidx(pitch, i, jj - 2);
            qo[0 * plane + id] = o[0];
            qo[1 * plane + id] = o[2];
            qo[2 * plane + id] = o[1];
            qo[3 * plane + id] = o[3];
            qo[4 * plane + id] = o[5];
            qo[5 * plane + id] = o[4];
          }
#pragma unroll
          for (int c = 0; c < 6; ++c) glo[c] = ap[c] - F[c];
        }
#pragma unroll
        for (int p = 0; p < 6; ++p) dlp[p] = dlc[p];
      }
      Wp = Wc;
#pragma unroll
      for (int p = 0; p < 6; ++p) ddp[p] = ddc[p];
    }
    // local y order of the row just read: h1, hv1, hu1, h2, hv2, hu2
#pragma unroll
    for (int c = 0; c < 6; ++c) qm2[c] = qm1[c];
    qm1[0] = cq[0]; qm1[1] = cq[2]; qm1[2] = cq[1];
    qm1[3] = cq[3]; qm1[4] = cq[5]; qm1[5] = cq[4];
    Cp = Cc;
  }
  flush_counts(Pd.cnt, Pd.ctl, 1, smax, hyp, K, lane);
  if (Pd.sig_on) {
    sig = wave_usum(sig);
    if (lane == 0) atomicAdd(&Pd.cnt->sig, sig);
  }
}

// ---------------------------------------------------------------- sweep launches
// sched 0: one wave per tile; 1: persistent waves over the tile list with a
// static stride; 2: persistent waves taking tiles from an atomic ticket (every
// wave leaves once the ticket passes the list, so the grid always drains).
template <int AXIS>
__device__ __forceinline__ void run_tiles(const PatchDev* __restrict__ patches, const void* __restrict__ tiles,
                                          int ntiles, int sched, unsigned* ticket) {
  const int lane = threadIdx.x & 63;
  const int w0 = blockIdx.x * 4 + (threadIdx.x >> 6);
  auto one = [&](int wv) {
    if (AXIS == 0) sweep_x_tile(patches, (const XTile*)tiles, wv, lane);
    else sweep_y_tile(patches, (const YTile*)tiles, wv, lane);
  };
  if (sched == 0) {
    if (w0 < ntiles) one(w0);
    return;
  }
  if (sched == 1) {
    for (int wv = w0; wv < ntiles; wv += gridDim.x * 4) one(wv);
    return;
  }
  for (;;) {
    int wv = 0;
    if (lane == 0) wv = (int)atomicAdd(ticket, 1u);
    wv = __shfl(wv, 0, 64);
    if (wv >= ntiles) break;
    one(wv);
  }
}

__global__ __launch_bounds__(256) void k_sweep_x(const PatchDev* __restrict__ patches, const XTile* __restrict__ tiles,
                                                 int ntiles, int sched, unsigned* ticket) {
  run_tiles<0>(patches, tiles, ntiles, sched, ticket);
}

__global__ __launch_bounds__(256) void k_sweep_y(const PatchDev* __restrict__ patches, const YTile* __restrict__ tiles,
                                                 int ntiles, int sched, unsigned* ticket) {
  run_tiles<1>(patches, tiles, ntiles, sched, ticket);
}

__global__ void k_zero_u32(unsigned* p, int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = 0u;
}

// ---------------------------------------------------------------- ghost cells
// Frame ring of a patch: 2 rows below (width nx+4), 2 cells each side of every
// interior row, 2 rows above.
__device__ __forceinline__ void ring_cell(int k, int ilo, int jlo, int bnx, int bny, int& i, int& j) {
  const int W = bnx + 4;
  if (k < 2 * W) { j = jlo - 2 + k / W; i = ilo - 2 + k % W; return; }
  k -= 2 * W;
  if (k < 4 * bny) {
    j = jlo + k / 4;
    int s = k % 4;
    i = s < 2 ? ilo - 2 + s : ilo + bnx + (s - 2);
    return;
  }
  k -= 4 * bny;
  j = jlo + bny + k / W;
  i = ilo - 2 + k % W;
}

__device__ __forceinline__ void coarse_value(const FillPatch& F, int I, int J, double th, double out[7]) {
  const long long id = cidx(F.cpitch, I, J);
#pragma unroll
  for (int c = 0; c < 6; ++c) out[c] = (1.0 - th) * F.qco[c * F.cplane + id] + th * F.qcn[c * F.cplane + id];
  out[6] = F.Bc[id];
}

// Refines fine cell (i, j) (inside the domain) from the coarse level at time
// fraction th and writes it.
__device__ __forceinline__ bool refine_cell_into(const FillPatch& F, int i, int j, double th, double* dst,
                                                 long long dplane) {
  const int r = F.r;
  const int I = i / r, J = j / r;
  const int a = i - r * I, b = j - r * J;
  const double fa = double(2 * a + 1 - r) / double(2 * r);
  const double fb = double(2 * b + 1 - r) / double(2 * r);
  const bool inx = (I - 1 >= 0) && (I + 1 < F.ncx);
  const bool iny = (J - 1 >= 0) && (J + 1 < F.ncy);
  double st[5][7];
  coarse_value(F, I, J, th, st[0]);
  if (inx) { coarse_value(F, I - 1, J, th, st[1]); coarse_value(F, I + 1, J, th, st[2]); }
  else {
#pragma unroll
    for (int c = 0; c < 7; ++c) { st[1][c] = 0.0; st[2][c] = 0.0; }
  }
  if (iny) { coarse_value(F, I, J - 1, th, st[3]); coarse_value(F, I, J + 1, th, st[4]); }
  else {
#pragma unroll
    for (int c = 0; c < 7; ++c) { st[3][c] = 0.0; st[4][c] = 0.0; }
  }
  const long long id = cidx(F.pitch, i, j);
  double out[6];
  bool rep = refine_from_stencil(F.P, st, inx, iny, fa, fb, F.B[id], out);
#pragma unroll
  for (int c = 0; c < 6; ++c) dst[c * dplane + id] = out[c];
  return rep;
}

// pass 0: in-domain frame cells not covered by a patch of the level are refined
// from the coarser level; pass 1: frame cells outside the domain mirror the
// in-domain cells across the walls (normal momentum negated).
__global__ __launch_bounds__(256) void k_ghost_fill(const FillPatch* __restrict__ fills, int pass) {
  const FillPatch& F = fills[blockIdx.y];
  const int ring = 4 * (F.bnx + 4) + 4 * F.bny;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ring) return;
  int i, j;
  ring_cell(k, F.ilo, F.jlo, F.bnx, F.bny, i, j);
  const bool indom = i >= 0 && j >= 0 && i < F.nx && j < F.ny;
  if (pass == 0) {
    if (!indom || F.coarse_none) return;
    if (F.mask[cidx(F.pitch, i, j)]) return;
    bool rep = refine_cell_into(F, i, j, *F.theta, F.q, F.plane);
    if (rep && F.cnt) atomicAdd(&F.cnt->repair, 1ull);
    return;
  }
  if (indom) return;
  int si = i, sj = j;
  bool fx = false, fy = false;
  if (i < 0) { si = -1 - i; fx = true; } else if (i >= F.nx) { si = 2 * F.nx - 1 - i; fx = true; }
  if (j < 0) { sj = -1 - j; fy = true; } else if (j >= F.ny) { sj = 2 * F.ny - 1 - j; fy = true; }
  const long long s = cidx(F.pitch, si, sj), d = cidx(F.pitch, i, j);
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    double v = F.q[c * F.plane + s];
    if ((fx && (c == 1 || c == 4)) || (fy && (c == 2 || c == 5))) v = 0.0 - v;
    F.q[c * F.plane + d] = v;
  }
}

// Regrid fill: every cell of a new fine patch not covered by an old patch is
// refined from the coarser level's current state.
__global__ __launch_bounds__(256) void k_refine_new(const FillPatch* __restrict__ fills,
                                                    const unsigned char* __restrict__ old_mask) {
  const FillPatch& F = fills[blockIdx.y];
  const int n = F.bnx * F.bny;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int i = F.ilo + k % F.bnx, j = F.jlo + k / F.bnx;
  if (old_mask[cidx(F.pitch, i, j)]) return;
  bool rep = refine_cell_into(F, i, j, 0.0, F.q, F.plane);
  if (rep && F.cnt) atomicAdd(&F.cnt->repair, 1ull);
}

// ---------------------------------------------------------------- coarsen
// Each coarse cell under a fine patch takes the mean of its r x r children
// (row-major sum times 1/r^2) for all six fields, then the dry-state fix-up.
__global__ __launch_bounds__(256) void k_coarsen(const CoarsenPatch* __restrict__ cps) {
  const CoarsenPatch& C = cps[blockIdx.y];
  const int r = C.r;
  const int cnx = C.bnx / r, cny = C.bny / r;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= cnx * cny) return;
  const int I = C.ilo / r + k % cnx, J = C.jlo / r + k / cnx;
  const double inv = 1.0 / double(r * r);
  double v[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    double s = 0.0;
    for (int bb = 0; bb < r; ++bb)
      for (int aa = 0; aa < r; ++aa) s = s + C.qf[c * C.fplane + cidx(C.fpitch, r * I + aa, r * J + bb)];
    v[c] = s * inv;
  }
  FixCount K = {0, 0, 0.0, 0.0};
  fixup(C.P, v, false, K);
  const long long d = cidx(C.cpitch, I, J);
#pragma unroll
  for (int c = 0; c < 6; ++c) C.qc[c * C.cplane + d] = v[c];
}

// ---------------------------------------------------------------- flag
__device__ __forceinline__ void mirror_ij(int nx, int ny, int& i, int& j) {
  if (i < 0) i = -1 - i; else if (i >= nx) i = 2 * nx - 1 - i;
  if (j < 0) j = -1 - j; else if (j >= ny) j = 2 * ny - 1 - j;
}

__global__ __launch_bounds__(256) void k_flag_raw(FlagLevel F) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= F.nx) return;
  auto ok = [&](int a, int b) {
    mirror_ij(F.nx, F.ny, a, b);
    const long long id = cidx(F.pitch, a, b);
    return F.mask[id] != 0 && F.q[id] >= F.hdry;  // F.q: field 0 (h1)
  };
  auto eta1 = [&](int a, int b) {
    mirror_ij(F.nx, F.ny, a, b);
    const long long id = cidx(F.pitch, a, b);
    return (F.B[id] + F.q[3 * F.plane + id]) + F.q[id];
  };
  unsigned char f = 0;
  if (ok(i, j) && ok(i - 1, j) && ok(i + 1, j) && ok(i, j - 1) && ok(i, j + 1)) {
    double gx = fabs(eta1(i + 1, j) - eta1(i - 1, j)) / (2.0 * F.dx);
    double gy = fabs(eta1(i, j + 1) - eta1(i, j - 1)) / (2.0 * F.dy);
    double gm = gx > gy ? gx : gy;
    f = gm > F.tau ? 1 : 0;
  }
  F.raw[(long long)j * F.nx + i] = f;
}

__global__ __launch_bounds__(256) void k_flag_dilate(FlagLevel F) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= F.nx) return;
  unsigned char f = 0;
  if (F.mask[cidx(F.pitch, i, j)]) {
    const int j0 = j - F.nbuf < 0 ? 0 : j - F.nbuf, j1 = j + F.nbuf > F.ny - 1 ? F.ny - 1 : j + F.nbuf;
    const int i0 = i - F.nbuf < 0 ? 0 : i - F.nbuf, i1 = i + F.nbuf > F.nx - 1 ? F.nx - 1 : i + F.nbuf;
    for (int b = j0; b <= j1 && !f; ++b)
      for (int a = i0; a <= i1; ++a)
        if (F.raw[(long long)b * F.nx + a]) { f = 1; break; }
  }
  F.out[(long long)j * F.nx + i] = f;
}

// ---------------------------------------------------------------- time step
// After a level substep: Courant check with this substep's speeds, fold them
// into the coarse-step maximum, clear them.
__global__ void k_after_substep(LevelCtl* ctls, const LevelInfo* infos, int n, double cflmax) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  LevelCtl& C = ctls[infos[k].ctl];
  const double sx = __longlong_as_double((long long)C.step_smax[0]);
  const double sy = __longlong_as_double((long long)C.step_smax[1]);
  const double ax = sx / infos[k].dx, ay = sy / infos[k].dy;
  const double courant = C.dt * (ax > ay ? ax : ay);
  if (courant > C.cmax || courant != courant) C.cmax = courant;
  if (!(courant <= cflmax)) C.status |= STATUS_CFL;
  C.last_smax[0] = C.step_smax[0];
  C.last_smax[1] = C.step_smax[1];
  if (C.step_smax[0] > C.acc_smax[0]) C.acc_smax[0] = C.step_smax[0];
  if (C.step_smax[1] > C.acc_smax[1]) C.acc_smax[1] = C.step_smax[1];
  C.step_smax[0] = 0ull;
  C.step_smax[1] = 0ull;
}

// Largest initial signal speed max(|u|,|v|) + sqrt(g (h1 + h2)) over covered cells.
__global__ __launch_bounds__(256) void k_initial_speed(const SpeedLevel* __restrict__ sl) {
  const SpeedLevel& S = sl[blockIdx.y];
  const long long n = (long long)S.nx * S.ny;
  double best = 0.0;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(k % S.nx), j = (int)(k / S.nx);
    const long long id = cidx(S.pitch, i, j);
    if (!S.mask[id]) continue;
    const double h1 = S.q[id], h2 = S.q[3 * S.plane + id];
    double vm = 0.0;
    if (h1 >= S.hdry) {
      double inv = 1.0 / h1;
      double a = fabs(S.q[1 * S.plane + id] * inv), b = fabs(S.q[2 * S.plane + id] * inv);
      double m = a > b ? a : b;
      vm = vm > m ? vm : m;
    }
    if (h2 >= S.hdry) {
      double inv = 1.0 / h2;
      double a = fabs(S.q[4 * S.plane + id] * inv), b = fabs(S.q[5 * S.plane + id] * inv);
      double m = a > b ? a : b;
      vm = vm > m ? vm : m;
    }
    if (h1 >= S.hdry || h2 >= S.hdry) {
      double s = vm + __builtin_sqrt(S.g * (h1 + h2));
      best = s > best ? s : best;
    }
  }
  best = wave_max(best);
  if ((threadIdx.x & 63) == 0)
    atomicMax(&S.ctl->acc_smax[0], (unsigned long long)__double_as_longlong(best));
}

// Next coarse dt of each problem from the speeds of its last coarse step (or, on
// the first step, the initial signal speed), then the levels' substep dt.
__global__ void k_next_dt(LevelCtl* ctls, const ProbDt* __restrict__ pd, int nprob, double cfl, int initial) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nprob) return;
  const ProbDt& D = pd[p];
  const double inf = __longlong_as_double(0x7ff0000000000000ll);
  double best = inf;
  double fac = 1.0;
  for (int l = 0; l < D.nlev; ++l) {
    LevelCtl& C = ctls[D.ctl0 + l];
    if (l > 0) fac *= (double)D.ratio[l - 1];
    if (initial) {
      if (!D.active[l]) continue;
      const double smx = __longlong_as_double((long long)C.acc_smax[0]);
      const double m = D.dx[l] < D.dy[l] ? D.dx[l] : D.dy[l];
      if (smx > 0.0) { double v = fac * ((cfl * m) / smx); best = v < best ? v : best; }
    } else {
      const double sx = __longlong_as_double((long long)C.acc_smax[0]);
      const double sy = __longlong_as_double((long long)C.acc_smax[1]);
      const double a = sx > 0.0 ? D.dx[l] / sx : inf;
      const double b = sy > 0.0 ? D.dy[l] / sy : inf;
      const double m = a < b ? a : b;
      if (m < inf) { double v = fac * (cfl * m); best = v < best ? v : best; }
    }
  }
  double dt = best;
  for (int l = 0; l < D.nlev; ++l) {
    LevelCtl& C = ctls[D.ctl0 + l];
    if (l > 0) dt = dt / (double)D.ratio[l - 1];
    C.dt = dt;
    C.acc_smax[0] = 0ull;
    C.acc_smax[1] = 0ull;
    C.cmax = 0.0;
  }
  ctls[D.ctl0].t += best;
  if (D.dt_out) D.dt_out[0] = best;
}

// Retake of a rejected coarse step: the given coarse dt, the levels' substeps,
// cleared speeds and Courant maximum.
__global__ void k_set_dt0(LevelCtl* ctls, const ProbDt* __restrict__ pd, const double* __restrict__ dt0, int nprob) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nprob) return;
  const ProbDt& D = pd[p];
  double dt = dt0[p];
  for (int l = 0; l < D.nlev; ++l) {
    LevelCtl& C = ctls[D.ctl0 + l];
    if (l > 0) dt = dt / (double)D.ratio[l - 1];
    C.dt = dt;
    C.acc_smax[0] = 0ull;
    C.acc_smax[1] = 0ull;
    C.cmax = 0.0;
  }
  ctls[D.ctl0].t += dt0[p];
}

__global__ void k_reset_acc(LevelCtl* ctls, const ProbDt* __restrict__ pd, int nprob) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nprob) return;
  for (int l = 0; l < pd[p].nlev; ++l) {
    ctls[pd[p].ctl0 + l].acc_smax[0] = 0ull;
    ctls[pd[p].ctl0 + l].acc_smax[1] = 0ull;
  }
}

__global__ void k_set_theta(double* th, double v) { *th = v; }

// Cells of a level-wide copy [6][ny][nx] that no patch covers read NaN.
__global__ __launch_bounds__(256) void k_nan_uncovered(double* q, const unsigned char* __restrict__ mask,
                                                       long long pitch, int nx, int ny) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long pu = (long long)nx * ny;
  if (t >= pu) return;
  const int i = (int)(t % nx), j = (int)(t / nx);
  if (mask[cidx(pitch, i, j)]) return;
  const double nan = __longlong_as_double(0x7ff8000000000000ll);
#pragma unroll
  for (int f = 0; f < 6; ++f) q[f * pu + t] = nan;
}

}  // namespace mlswe
