// HIP kernels (gfx950) of the two-layer shallow-water step and the multilayer
// AMR operators.  Level arrays are dense per (problem, level), field-major SoA
// with a two-cell frame; row j, column i sits at (j + 2) * pitch + (i + XOFF),
// XOFF = 8 so that interior rows start on a 64-byte boundary.
#include "mlswe_kernels.hpp"
#include "mlswe_wave.hpp"

namespace mlswe {


#define MLSWE_KX k_sweep_x
#define MLSWE_KY k_sweep_y
#define MLSWE_KX1 k_sweep_x1
#define MLSWE_KY1 k_sweep_y1
#define MLSWE_KXR k_sweep_xr
#define MLSWE_KYR k_sweep_yr
#include "mlswe_sweeps.inc"

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
// in-domain cells across the walls (normal momentum negated).  With dt_ctl
// set, the launch also stores the level's time step (dt_ctl->dt = dt) for the
// sweeps that follow it: a caller-given step costs no launch of its own.
__global__ __launch_bounds__(256) void k_ghost_fill(const FillPatch* __restrict__ fills, int pass, double theta,
                                                    LevelCtl* dt_ctl, double dt) {
  if (dt_ctl && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) dt_ctl->dt = dt;
  const FillPatch& F = fills[blockIdx.y];
  if (F.skip && *F.skip) return;
  const int ring = 4 * (F.bnx + 4) + 4 * F.bny;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ring) return;
  int i, j;
  ring_cell(k, F.ilo, F.jlo, F.bnx, F.bny, i, j);
  const bool indom = i >= 0 && j >= 0 && i < F.nx && j < F.ny;
  if (pass == 0) {
    if (!indom || F.coarse_none) return;
    if (F.mask[cidx(F.pitch, i, j)]) return;
    bool rep = refine_cell_into(F, i, j, theta, F.q, F.plane);
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
__global__ __launch_bounds__(256) void k_refine_new(const FillPatch* __restrict__ fills) {
  const FillPatch& F = fills[blockIdx.y];
  const int n = F.bnx * F.bny;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int i = F.ilo + k % F.bnx, j = F.jlo + k / F.bnx;
  if (F.mask_old[cidx(F.pitch, i, j)]) return;
  bool rep = refine_cell_into(F, i, j, 0.0, F.q, F.plane);
  if (rep && F.cnt) atomicAdd(&F.cnt->repair, 1ull);
}

// ---------------------------------------------------------------- coarsen
// Each coarse cell under a fine patch takes the mean of its r x r children
// (row-major sum times 1/r^2) for all six fields, then the dry-state fix-up.
__global__ __launch_bounds__(256) void k_coarsen(const CoarsenPatch* __restrict__ cps) {
  const CoarsenPatch& C = cps[blockIdx.y];
  if (C.halt[HALT_SET] || *C.skip) return;
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
  FixCount K = {0, 0, 0.0, 0.0, 0};
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

// Undilated flag of cell (i, j): the top layer wet in the cell and its four
// neighbours (mirrored at the domain edge) and the larger centred difference
// of eta1 above tau.
__device__ __forceinline__ unsigned char flag_raw_cell(const FlagLevel& F, int i, int j) {
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
  return f;
}

// Flag of covered cell (i, j) dilated by nbuf cells (clipped to the level)
// over the undilated flags F.raw.
__device__ __forceinline__ unsigned char flag_dilate_cell(const FlagLevel& F, int i, int j) {
  unsigned char f = 0;
  if (F.mask[cidx(F.pitch, i, j)]) {
    const int j0 = j - F.nbuf < 0 ? 0 : j - F.nbuf, j1 = j + F.nbuf > F.ny - 1 ? F.ny - 1 : j + F.nbuf;
    const int i0 = i - F.nbuf < 0 ? 0 : i - F.nbuf, i1 = i + F.nbuf > F.nx - 1 ? F.nx - 1 : i + F.nbuf;
    for (int b = j0; b <= j1 && !f; ++b)
      for (int a = i0; a <= i1; ++a)
        if (F.raw[(long long)b * F.nx + a]) { f = 1; break; }
  }
  return f;
}

// Flags of level blockIdx.z of a list (one launch for many problems).
__global__ __launch_bounds__(256) void k_flag_raw(const FlagLevel* __restrict__ Fs) {
  const FlagLevel F = Fs[blockIdx.z];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= F.nx || j >= F.ny) return;
  F.raw[(long long)j * F.nx + i] = flag_raw_cell(F, i, j);
}

__global__ __launch_bounds__(256) void k_flag_dilate(const FlagLevel* __restrict__ Fs) {
  const FlagLevel F = Fs[blockIdx.z];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= F.nx || j >= F.ny) return;
  F.out[(long long)j * F.nx + i] = flag_dilate_cell(F, i, j);
}

// The same two passes over one level with the descriptor passed by value and
// one thread per cell of a flat grid (cell k = j nx + i), for callers whose
// launches may use no device memory of the library's own.
__global__ __launch_bounds__(256) void k_flag_raw_v(FlagLevel F) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (long long)F.nx * F.ny) return;
  const int i = (int)(k % F.nx), j = (int)(k / F.nx);
  F.raw[k] = flag_raw_cell(F, i, j);
}

__global__ __launch_bounds__(256) void k_flag_dilate_v(FlagLevel F) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (long long)F.nx * F.ny) return;
  const int i = (int)(k % F.nx), j = (int)(k / F.nx);
  F.out[k] = flag_dilate_cell(F, i, j);
}

// Tile summary for clustering (block row y: problem y of the list): one
// thread per tile of the finer level.
__global__ __launch_bounds__(256) void k_flag_tiles(const FlagTiles* __restrict__ Ts) {
  const FlagTiles F = Ts[blockIdx.y];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= F.tx * F.ty) return;
  const int I = t % F.tx, J = t / F.tx, r = F.r;
  const int ci0 = (CLUSTER_TILE * I) / r, cj0 = (CLUSTER_TILE * J) / r;
  const int ci1 = min(F.nx, (CLUSTER_TILE * (I + 1) + r - 1) / r);
  const int cj1 = min(F.ny, (CLUSTER_TILE * (J + 1) + r - 1) / r);
  int any = 0;
  for (int j = cj0; j < cj1; ++j)
    for (int i = ci0; i < ci1; ++i) any |= F.flags[(long long)j * F.nx + i];
  int inside = 1;
  const int a0 = max(0, ci0 - 2), a1 = min(F.nx, ci1 + 2);
  const int b0 = max(0, cj0 - 2), b1 = min(F.ny, cj1 + 2);
  for (int j = b0; j < b1; ++j)
    for (int i = a0; i < a1; ++i) inside &= F.mask[cidx(F.pitch, i, j)] != 0 ? 1 : 0;
  F.out[t] = (unsigned char)((any != 0 ? 1 : 0) | (inside << 1));
}

// ---------------------------------------------------------------- time step
// After a substep: one block per (problem, level) reduces the partials of that
// problem's x and y tiles (each wave a strided share, then across the waves),
// then records the largest speeds, the Courant number and the CFL status, and
// adds the fix-up and clamp counts to the problem's counters.  Speeds are kept
// as the bit patterns of non-negative doubles.  Block size: a multiple of 64,
// at most 1024.
// The end of a (problem, level)'s substep reduction: the Courant check,
// status bits, speeds and counters from the reduced partials.  The words it
// reads are loaded together first (tail_load, issued before the partials are
// reduced) so that the reduction's end waits on one round trip to memory, not
// on one per read-modify-write.
struct TailIn {
  unsigned set, armed;
  double dt, cmax;
  int status;
  unsigned long long acc0, acc1, hyp, nclip, repair;
  double clip1, clip2;
};

__device__ __forceinline__ TailIn tail_load(const LevelCtl* ctls, const Counters* cnts, const LevelInfo& I,
                                            const unsigned* halt) {
  TailIn t;
  t.set = halt[HALT_SET];
  t.armed = halt[HALT_ARMED];
  const LevelCtl& C = ctls[I.ctl];
  t.dt = C.dt;
  t.cmax = C.cmax;
  t.status = C.status;
  t.acc0 = C.acc_smax[0];
  t.acc1 = C.acc_smax[1];
  const Counters& K = cnts[I.cnt];
  t.hyp = K.hyp;
  t.nclip = K.nclip;
  t.repair = K.repair;
  t.clip1 = K.clip1;
  t.clip2 = K.clip2;
  return t;
}

__device__ __forceinline__ void after_tail(LevelCtl* ctls, Counters* cnts, const LevelInfo& I, const TailIn& t,
                                           double sx, double sy, double c1, double c2, unsigned long long h,
                                           unsigned long long nc, unsigned long long rp, unsigned long long nf,
                                           double cflmax, unsigned* halt) {
  // a halted window keeps the failing substep's control block and counters
  if (t.set) return;
  LevelCtl& C = ctls[I.ctl];
  const double ax = sx / I.dx, ay = sy / I.dy;
  const double courant = t.dt * (ax > ay ? ax : ay);
  if (t.armed && (!(courant <= cflmax) || nf)) halt[HALT_SET] = 1u;
  if (courant > t.cmax || courant != courant) C.cmax = courant;
  int st = t.status;
  if (!(courant <= cflmax)) st |= STATUS_CFL;
  if (nf) st |= STATUS_NAN;
  C.status = st;
  const unsigned long long bx = (unsigned long long)__double_as_longlong(sx);
  const unsigned long long by = (unsigned long long)__double_as_longlong(sy);
  C.last_smax[0] = bx;
  C.last_smax[1] = by;
  if (bx > t.acc0) C.acc_smax[0] = bx;
  if (by > t.acc1) C.acc_smax[1] = by;
  Counters& K = cnts[I.cnt];
  K.hyp = t.hyp + h;
  K.nclip = t.nclip + nc;
  K.repair = t.repair + rp;
  if (c1 != 0.0) K.clip1 = t.clip1 + c1;
  if (c2 != 0.0) K.clip2 = t.clip2 + c2;
}

// Block (x, y) of a grid of (problems, slices) reduces slice y of problem x's
// partials (its x tiles, then its y tiles, cut into gridDim.y equal slices).
// With one slice the block finishes the problem itself; with several, each
// block leaves its slice's result in red and k_after_combine, launched next,
// combines the slices in slice order.
__global__ __launch_bounds__(1024) void k_after_substep(LevelCtl* ctls, Counters* cnts, const LevelInfo* infos,
                                                        const TilePart* parts, double cflmax, SliceRed* red,
                                                        unsigned* halt, const unsigned* skip) {
  __shared__ double red_d[4][16];
  __shared__ unsigned long long red_u[4][16];
  const LevelInfo I = infos[blockIdx.x];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int ns = (int)gridDim.y, sl = (int)blockIdx.y;
  // the skip flag, the tail's words and the partials are all requested before
  // the first wait; a problem a retake leaves alone is dropped at the end
  const unsigned sk = skip[I.prob];
  const TailIn tin = tail_load(ctls, cnts, I, halt);
  double sx = 0.0, sy = 0.0, c1 = 0.0, c2 = 0.0;
  unsigned long long h = 0, nc = 0, rp = 0, nf = 0;
  const int ntot = I.nx + I.ny, step = blockDim.x;
  const int kb = (int)((long long)ntot * sl / ns), ke = (int)((long long)ntot * (sl + 1) / ns);
  // four independent loads in flight per pass (the passes are latency bound)
  for (int k0 = kb + (int)threadIdx.x; k0 < ke; k0 += 4 * step) {
    TilePart T[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = k0 + u * step;
      if (k < ke) T[u] = parts[k < I.nx ? I.x0 + k : I.y0 + (k - I.nx)];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = k0 + u * step;
      if (k >= ke) continue;
      if (k < I.nx) sx = T[u].smax > sx ? T[u].smax : sx;
      else sy = T[u].smax > sy ? T[u].smax : sy;
      c1 += T[u].clip1;
      c2 += T[u].clip2;
      h += T[u].hyp;
      nc += T[u].nclip;
      rp += T[u].repair;
      nf += T[u].nonfinite;
    }
  }
  sx = wave_max(sx);
  sy = wave_max(sy);
  c1 = wave_sum(c1);
  c2 = wave_sum(c2);
  h = wave_usum(h);
  nc = wave_usum(nc);
  rp = wave_usum(rp);
  nf = wave_usum(nf);
  if (lane == 0) {
    red_d[0][wave] = sx; red_d[1][wave] = sy; red_d[2][wave] = c1; red_d[3][wave] = c2;
    red_u[0][wave] = h; red_u[1][wave] = nc; red_u[2][wave] = rp; red_u[3][wave] = nf;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int w = 1; w < nw; ++w) {
    sx = red_d[0][w] > sx ? red_d[0][w] : sx;
    sy = red_d[1][w] > sy ? red_d[1][w] : sy;
    c1 += red_d[2][w]; c2 += red_d[3][w];
    h += red_u[0][w]; nc += red_u[1][w]; rp += red_u[2][w]; nf += red_u[3][w];
  }
  if (sk) return;  // a problem a retake leaves alone
  if (ns > 1) {
    red[(size_t)blockIdx.x * ns + sl] = SliceRed{sx, sy, c1, c2, h, nc, rp, nf};
    return;
  }
  after_tail(ctls, cnts, I, tin, sx, sy, c1, c2, h, nc, rp, nf, cflmax, halt);
}

// One thread per problem: its ns slice results combined in slice order, then
// the end of the reduction.
__global__ void k_after_combine(LevelCtl* ctls, Counters* cnts, const LevelInfo* infos, int n, int ns,
                                const SliceRed* __restrict__ red, double cflmax, unsigned* halt,
                                const unsigned* skip) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const LevelInfo I = infos[i];
  const unsigned sk = skip[I.prob];
  const TailIn tin = tail_load(ctls, cnts, I, halt);
  const SliceRed* R = red + (size_t)i * ns;
  double sx = R[0].sx, sy = R[0].sy, c1 = R[0].c1, c2 = R[0].c2;
  unsigned long long h = R[0].h, nc = R[0].nc, rp = R[0].rp, nf = R[0].nf;
  for (int k = 1; k < ns; ++k) {
    sx = R[k].sx > sx ? R[k].sx : sx;
    sy = R[k].sy > sy ? R[k].sy : sy;
    c1 += R[k].c1; c2 += R[k].c2;
    h += R[k].h; nc += R[k].nc; rp += R[k].rp; nf += R[k].nf;
  }
  if (sk) return;
  after_tail(ctls, cnts, I, tin, sx, sy, c1, c2, h, nc, rp, nf, cflmax, halt);
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
__global__ void k_next_dt(LevelCtl* ctls, const ProbDt* __restrict__ pd, int nprob, double cfl, int initial,
                          const unsigned* halt) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nprob || halt[HALT_SET]) return;
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
    if (l > 0) dt = dt / (double)D.rt[l - 1];
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
__global__ void k_set_dt0(LevelCtl* ctls, const ProbDt* __restrict__ pd, const double* __restrict__ dt0, int nprob,
                          const unsigned* skip) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nprob || skip[p]) return;
  const ProbDt& D = pd[p];
  double dt = dt0[p];
  for (int l = 0; l < D.nlev; ++l) {
    LevelCtl& C = ctls[D.ctl0 + l];
    if (l > 0) dt = dt / (double)D.rt[l - 1];
    C.dt = dt;
    C.acc_smax[0] = 0ull;
    C.acc_smax[1] = 0ull;
    C.cmax = 0.0;
  }
  ctls[D.ctl0].t += dt0[p];
}

__global__ void k_set_skip(unsigned* skip, const unsigned char* __restrict__ fail, int n) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) skip[p] = fail ? (fail[p] ? 0u : 1u) : 0u;
}

__global__ void k_reset_acc(LevelCtl* ctls, const ProbDt* __restrict__ pd, int nprob) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nprob) return;
  for (int l = 0; l < pd[p].nlev; ++l) {
    ctls[pd[p].ctl0 + l].acc_smax[0] = 0ull;
    ctls[pd[p].ctl0 + l].acc_smax[1] = 0ull;
  }
}


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

// ---------------------------------------------------------------- flux correction
// A cell of the sweeps' line from a level buffer: x lines take (h, hu, hv) per
// layer, y lines (h, hv, hu), as the sweeps load them.
__device__ __forceinline__ CellX line_cell(const PhysParams& P, const double* q, const double* B, long long plane,
                                           long long k, bool ydir) {
  const double h1 = q[k], a1 = q[plane + k], b1 = q[2 * plane + k];
  const double h2 = q[3 * plane + k], a2 = q[4 * plane + k], b2 = q[5 * plane + k];
  return ydir ? load_cell(P, h1, b1, a1, h2, b2, a2, B[k]) : load_cell(P, h1, a1, b1, h2, a2, b2, B[k]);
}

// Depth parts (layers 1, 2) of the terms the sweeps give the cell before a face
// (A-dQ + F) and the cell after it (A+dQ - F), from the four cells around the
// face (the face lies between c[1] and c[2]).
__device__ __forceinline__ void face_terms(const PhysParams& P, const CellX* c, double nu, double gr[2],
                                           double gl[2]) {
  EdgeW Wm, W, Wp;
  riemann(P, c[0], c[1], Wm);
  riemann(P, c[1], c[2], W);
  riemann(P, c[2], c[3], Wp);
  double coef[6], F[6], am[6], ap[6];
#pragma unroll
  for (int p = 0; p < 6; ++p) coef[p] = corr_coef(W, p, wdot(W, W, p), wdot(Wm, W, p), wdot(W, Wp, p), nu);
  correction_flux(W, coef, F);
  fluctuations(W, am, ap);
  gr[0] = am[0] + F[0];
  gr[1] = am[3] + F[3];
  gl[0] = ap[0] - F[0];
  gl[1] = ap[3] - F[3];
}

// Coarse face fluxes of each record's cell O after a level-l substep (x faces
// from the x-sweep's input, y faces from the x-swept state), running sums
// cleared; one thread per (record, direction).  The flux is O's normal
// momentum plus (face after O) or minus (face before O) O's term from that face.
__global__ __launch_bounds__(64) void k_reflux_coarse(const RefluxCell* __restrict__ rcs, int n, int parity) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 4LL * n) return;
  const RefluxCell& R = rcs[t >> 2];
  if (*R.skip) return;
  const int d = (int)(t & 3);
  if (!((R.dirs >> d) & 1)) return;
  const long long o = cidx(R.cpitch, R.i, R.j);
  const bool ydir = d >= 2, plus = (d & 1) == 0;
  const long long st = ydir ? R.cpitch : 1;
  const double* q = ydir ? R.cqs : R.cq[parity];
  const double nu = R.cctl->dt / (ydir ? R.cdy : R.cdx);
  const long long k0 = plus ? o - st : o - 2 * st;
  CellX c[4];
  for (int u = 0; u < 4; ++u) c[u] = line_cell(R.P, q, R.cB, R.cplane, k0 + u * st, ydir);
  double gr[2], gl[2];
  face_terms(R.P, c, nu, gr, gl);
  const int mf = ydir ? 2 : 1;
  for (int m = 0; m < 2; ++m) {
    const double mo = q[(3 * m + mf) * R.cplane + o];
    R.reg[2 * d + m] = plus ? mo + gr[m] : mo - gl[m];
    R.reg[8 + 2 * d + m] = 0.0;
  }
}

// After a level-(l+1) substep: the fine flux through each of the r fine faces
// along each recorded face (the fine cell beside the face: its normal momentum
// minus its term from a face before it, plus its term from a face after it),
// one thread per (record, direction, fine face), into the record's slots.
__global__ __launch_bounds__(64) void k_reflux_fine(const RefluxCell* __restrict__ rcs, int n, int parity) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 64LL * n) return;
  const RefluxCell& R = rcs[t >> 6];
  if (*R.skip) return;
  const int d = (int)((t >> 4) & 3), k = (int)(t & 15);
  const int r = R.r;
  if (!((R.dirs >> d) & 1) || k >= r) return;
  const bool ydir = d >= 2, plus = (d & 1) == 0;
  const long long st = ydir ? R.fpitch : 1;
  const double* q = ydir ? R.fqs : R.fq[parity];
  const double nu = R.fctl->dt / (ydir ? R.fdy : R.fdx);
  int fi, fj;
  if (d == 0) { fi = r * (R.i + 1); fj = r * R.j + k; }
  else if (d == 1) { fi = r * R.i - 1; fj = r * R.j + k; }
  else if (d == 2) { fi = r * R.i + k; fj = r * (R.j + 1); }
  else { fi = r * R.i + k; fj = r * R.j - 1; }
  const long long f = cidx(R.fpitch, fi, fj);
  const long long k0 = plus ? f - 2 * st : f - st;
  CellX c[4];
  for (int u = 0; u < 4; ++u) c[u] = line_cell(R.P, q, R.fB, R.fplane, k0 + u * st, ydir);
  double gr[2], gl[2];
  face_terms(R.P, c, nu, gr, gl);
  const int mf = ydir ? 2 : 1;
  for (int m = 0; m < 2; ++m) {
    const double mF = q[(3 * m + mf) * R.fplane + f];
    R.reg[16 + (d * 16 + k) * 2 + m] = plus ? mF - gl[m] : mF + gr[m];
  }
}

// The fine fluxes of a substep summed along each face (in face order) and
// added to the running sums; one thread per record.
__global__ __launch_bounds__(64) void k_reflux_fsum(const RefluxCell* __restrict__ rcs, int n) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const RefluxCell& R = rcs[t];
  if (*R.skip) return;
  for (int d = 0; d < 4; ++d) {
    if (!((R.dirs >> d) & 1)) continue;
    for (int m = 0; m < 2; ++m) {
      double s = R.reg[16 + (d * 16) * 2 + m];
      for (int k = 1; k < R.r; ++k) s = s + R.reg[16 + (d * 16 + k) * 2 + m];
      R.reg[8 + 2 * d + m] = R.reg[8 + 2 * d + m] + s;
    }
  }
}

// After coarsening: nu_c (gc - acc / (r rt)) added to (faces after O) or
// subtracted from (faces before O) O's depths, faces in the order +x, -x, +y, -y.
__global__ __launch_bounds__(64) void k_reflux_apply(const RefluxCell* __restrict__ rcs, int n, int parity, int rt) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const RefluxCell& R = rcs[t];
  if (*R.skip) return;
  const long long o = cidx(R.cpitch, R.i, R.j);
  const double dt = R.cctl->dt;
  const double inv = 1.0 / double(R.r * rt);  // r fine faces in each of rt substeps
  const double nux = dt / R.cdx, nuy = dt / R.cdy;
  double* q = R.cq[parity];
  double h[2] = {q[o], q[3 * R.cplane + o]};
  for (int d = 0; d < 4; ++d) {
    if (!((R.dirs >> d) & 1)) continue;
    const double nu = d < 2 ? nux : nuy;
    for (int m = 0; m < 2; ++m) {
      const double corr = nu * (R.reg[2 * d + m] - R.reg[8 + 2 * d + m] * inv);
      h[m] = (d & 1) == 0 ? h[m] + corr : h[m] - corr;
    }
  }
  q[o] = h[0];
  q[3 * R.cplane + o] = h[1];
}

// Cells of a level that no patch covers set to zero (all six fields) in the
// level's own buffer: values handed in there are never used, and a non-finite
// one would otherwise reach the non-finite check of the union-tile x-sweep.
__global__ __launch_bounds__(256) void k_zero_uncovered(double* q, const unsigned char* __restrict__ mask,
                                                        long long pitch, long long plane, int nx, int ny) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)nx * ny) return;
  const int i = (int)(t % nx), j = (int)(t / nx);
  const long long k = cidx(pitch, i, j);
  if (mask[k]) return;
#pragma unroll
  for (int f = 0; f < 6; ++f) q[f * plane + k] = 0.0;
}

// Byte runs in one launch (block row y: run y), copied or filled.
__global__ __launch_bounds__(256) void k_byte_segs(const ByteSeg* __restrict__ segs) {
  const ByteSeg S = segs[blockIdx.y];
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < S.n; k += (long long)gridDim.x * blockDim.x)
    S.dst[k] = S.src ? S.src[k] : (unsigned char)S.value;
}

// Coverage bytes of patch boxes (block row y: box y): interior, first column
// and first row bits.
__global__ __launch_bounds__(256) void k_mask_boxes(const MaskBox* __restrict__ boxes) {
  const MaskBox M = boxes[blockIdx.y];
  const int n = M.nx * M.ny;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    const int a = k % M.nx, b = k / M.nx;
    M.mask[cidx(M.pitch, M.ilo + a, M.jlo + b)] = COV_IN | (a == 0 ? COV_COL0 : 0) | (b == 0 ? COV_ROW0 : 0);
  }
}

// Many box copies in one launch: block row y copies box y; its elements are
// numbered column-fastest over the (field, row) lines and strided over the
// block row's threads.
// halt (nullable): a backup of a coarse step's start, skipped once a deferred
// window has halted; mark: this launch counts the backup in HALT_MARKS.
__global__ __launch_bounds__(256) void k_copy_boxes(const CopyBox* __restrict__ boxes, unsigned* halt, int mark) {
  if (halt) {
    if (halt[HALT_SET]) return;
    if (mark && halt[HALT_ARMED] && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) halt[HALT_MARKS] += 1u;
  }
  const CopyBox C = boxes[blockIdx.y];
  if (C.skip && *C.skip) return;
  const unsigned nx = (unsigned)C.nx, ny = (unsigned)C.ny;
  const unsigned n = nx * ny * (unsigned)C.nf;
  for (unsigned k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    const unsigned line = k / nx, a = k - line * nx;
    const unsigned f = line / ny, b = line - f * ny;
    const long long off = (long long)f * C.plane + (long long)b * C.pitch + a;
    C.dst[off] = C.src[off];
  }
}

// Halt words cleared, armed (1) for a deferred window or disarmed (0).
__global__ void k_set_halt(unsigned* halt, unsigned armed) {
  if (threadIdx.x == 0) {
    halt[HALT_SET] = 0u;
    halt[HALT_MARKS] = 0u;
    halt[HALT_ARMED] = armed;
  }
}

// Six fields between a level array (interior cells, padded rows) and the
// compact [6][ny][nx] layout of the interface; dir 0: compact -> level,
// 1: level -> compact.  One launch instead of one strided copy per field.
__global__ __launch_bounds__(256) void k_copy6(double* lv, long long pitch, long long plane, double* cq, int nx,
                                               int ny, int dir) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long pu = (long long)nx * ny;
  if (t >= pu) return;
  const int i = (int)(t % nx), j = (int)(t / nx);
  const long long id = cidx(pitch, i, j);
  if (dir == 0) {
#pragma unroll
    for (int f = 0; f < 6; ++f) lv[f * plane + id] = cq[f * pu + t];
  } else {
#pragma unroll
    for (int f = 0; f < 6; ++f) cq[f * pu + t] = lv[f * plane + id];
  }
}

}  // namespace mlswe
