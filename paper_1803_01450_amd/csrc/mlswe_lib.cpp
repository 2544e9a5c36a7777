// Host side of the MI355X two-layer shallow-water AMR library: contexts,
// problems, dense per-level device arrays, launch descriptors, clustering,
// regridding and the subcycled (Berger-Oliger) advance, behind the C ABI of
// include/mlswe.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <limits>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/mlswe.h"
#include "mlswe_kernels.hpp"
#include "mlswe_layers.hpp"

using namespace mlswe;

namespace {

constexpr int MAXLEV = 8;
constexpr int TILE = CLUSTER_TILE;  // clustering tile (fine cells per side)

struct Box { int ilo, jlo, nx, ny; };

struct LevelH {
  int nx = 0, ny = 0;
  double dx = 0, dy = 0;
  long long pitch = 0, plane = 0;
  double* q[2] = {nullptr, nullptr};
  int cur = 0;
  double* qs = nullptr;
  double* B = nullptr;
  unsigned char* mask = nullptr;
  unsigned char* mask_old = nullptr;
  unsigned char* fraw = nullptr;
  unsigned char* fout = nullptr;
  double* bk = nullptr;  // copy of the current buffer for a rejected coarse step
  std::vector<unsigned char> mask_h;  // host copy of the coverage, rebuilt when needed
  bool mask_h_ok = true;
  std::vector<Box> boxes;
};

// Device buffers of the adjoint step (level layout), allocated on first use.
struct AdjBuf {
  double* lam1 = nullptr;  // adjoint of the step's output
  double* lamS = nullptr;  // adjoint of the x-swept state
  double* lamG = nullptr;  // adjoint of the wall-filled state
  double* cL = nullptr;    // per-edge contributions (7 planes)
  double* cR = nullptr;
  double* Bbx = nullptr;
  double* Bby = nullptr;
  int* status = nullptr;        // device: set by the edge kernel on a non-wet edge (sticky)
  int* status_host = nullptr;   // pinned copy of status, written after each adjoint step
  hipEvent_t status_ev = nullptr;
};

struct ProblemH {
  AdjBuf adj;
  PhysParams P;
  int nlev = 1;
  int ratio[MAXLEV] = {0};
  int rt[MAXLEV] = {0};  // time ratios of the current coarse step (the space ratios unless chosen)
  // largest speeds of the last coarse step as read back after its Courant
  // check (valid until the device copies may have changed)
  unsigned long long last_acc[MAXLEV][2] = {};
  bool acc_known = false;
  LevelH L[MAXLEV];
  int ctl0 = 0;  // index of level 0's LevelCtl
  int cnt = 0;   // index of the problem's counters
  double t = 0.0;
  long long updates[MAXLEV] = {0};
  long long rejected = 0;
  bool bathy = false;
  bool state = false;
  bool have_dt = false;
};

// Launch data of one level index across all problems (rebuilt on patch change).
struct LevelLaunch {
  bool dirty = true;
  int nptch = 0;
  std::vector<int> patch_prob;               // problem of each patch
  std::vector<std::pair<int, int>> xr, yr;   // per patch: tile ranges
  PatchDev* pd[2] = {nullptr, nullptr};      // by buffer parity of the level
  XTile* xt = nullptr;                       // patch tiles, then run tiles
  YTile* yt = nullptr;
  int nxt = 0, nyt = 0;                      // all tiles
  int nxt_p = 0, nyt_p = 0;                  // patch tiles
  bool use_runs = false;                     // some problem has several patches on the level
  std::vector<std::pair<int, int>> xrun, yrun;  // per problem: run tile ranges
  int rows_x = 0, rows_y = 0;                // rows per sweep wave in the current tiles
  int rows_xr = 0, rows_yr = 0;              // the same for the run tiles
  // the layout size at the last evaluation of the tile-height model and its
  // choices (patch x / y, run x / y), kept while the layout stays similar
  long long model_cells = -1, model_patches = 0;
  bool model_runs = false;
  int model_rows[4] = {0, 0, 0, 0};
  TilePart* parts = nullptr;                 // per tile: x tiles, then y tiles
  int cap_parts = 0;
  int max_info_tiles = 0;                    // most tiles of one problem on the level
  FillPatch* fp[4] = {nullptr, nullptr, nullptr, nullptr};   // [fine parity * 2 + coarse parity]
  CoarsenPatch* cp[4] = {nullptr, nullptr, nullptr, nullptr};
  std::vector<int> fill_first;               // per problem: first fill entry (or -1) and count
  std::vector<int> fill_count;
  std::vector<int> crs_first, crs_count;     // per problem: coarsen entries (row chunks of patches)
  int ncrs = 0, cap_cp = 0;
  LevelInfo* li = nullptr;                   // ctl / dx / dy of every problem having the level; four
                                             // copies (x ranges of patch / run tiles, times y ranges)
  int nli = 0;
  std::vector<int> li_first;
  int cap_pd = 0, cap_xt = 0, cap_yt = 0, cap_fp = 0, cap_li = 0;
  // flux correction (config reflux): records of the coarser level's cells
  // beside this level's patches, per problem contiguous, and their registers
  RefluxCell* rfx = nullptr;
  double* rfx_reg = nullptr;
  int nrfx = 0, cap_rfx = 0, cap_rfx_reg = 0;
  std::vector<int> rfx_first, rfx_count;
};

}  // namespace

struct mlswe_ctx {
  mlswe_config cfg;
  hipStream_t stream = nullptr;
  int device = 0;
  std::vector<ProblemH> probs;
  LevelCtl* ctl = nullptr;
  int ctl_cap = 0;
  Counters* cnt = nullptr;
  int cnt_cap = 0;
  ProbDt* pdt = nullptr;
  int pdt_cap = 0;
  bool pdt_dirty = true;
  SpeedLevel* spd = nullptr;
  int spd_cap = 0;
  LevelLaunch launch[MAXLEV];
  std::string err;
  long long bytes = 0;
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_used;
  // timed classes: 0 x-sweep, 1 y-sweep, 2 ghost fill, 3 substep reduction,
  // 4 coarsening, 5 flux correction, 6 dt rule, 7 regrid (host wall time)
  double kms[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  long long klaunch[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  double* dt_stage = nullptr;
  int dt_stage_cap = 0;
  int sig_on = 0;
  // launch shape of the sweeps (autotuned or set)
  mlswe_tuning tune;
  int ncu = 256;
  unsigned* tickets = nullptr;  // [2] atomic work tickets of the persistent sweeps
  // graph replay of whole coarse steps
  hipStream_t cap_stream = nullptr;
  long long generation = 0;      // bumped whenever launch data may have changed
  struct GraphRec {
    unsigned long long key;
    long long gen;
    int p0, p1;
    hipGraphExec_t exec;
    std::vector<long long> upd;  // per problem, per level update increments
    std::vector<int> flips;      // per problem, per level parity flips (0/1)
  };
  std::vector<GraphRec> graphs;
  long long graph_launches = 0, graph_captures = 0;
  LevelCtl* ctl_bk = nullptr;
  Counters* cnt_bk = nullptr;
  int bk_cap = 0, cbk_cap = 0;
  double* dt0_d = nullptr;
  int dt0_cap = 0;
  CopyBox* boxes_d = nullptr;  // copy list of a coarse step's backup / restore
  int boxes_cap = 0;
  LevelCtl* ctl_pin = nullptr;  // pinned readback of the control blocks
  size_t ctl_pin_cap = 0;
  unsigned char* pin = nullptr;  // pinned staging of the regrid flags
  size_t pin_cap = 0;
  ByteSeg* bsegs_d = nullptr;    // regrid descriptor lists
  int bsegs_cap = 0;
  MaskBox* mboxes_d = nullptr;
  int mboxes_cap = 0;
  FillPatch* rfills_d = nullptr;
  int rfills_cap = 0;
  FlagLevel* flv_d = nullptr;    // flag descriptors
  int flv_cap = 0;
  FlagTiles* ftl_d = nullptr;    // tile-summary descriptors and their output
  int ftl_cap = 0;
  unsigned char* tbits_d = nullptr;
  int tbits_cap = 0;
  unsigned long long* lrep_d = nullptr;  // repair counter of the M-layer refine
  int lrep_cap = 0;
};

namespace {

int fail(mlswe_ctx* c, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return code;
}

#define HIPCHK(c, call)                                                                      \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess) return fail((c), MLSWE_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

int dalloc(mlswe_ctx* c, void** p, size_t bytes) {
  if (c->cfg.max_device_bytes > 0 && c->bytes + (long long)bytes > c->cfg.max_device_bytes)
    return fail(c, MLSWE_ENOMEM, "device memory cap of %lld bytes exceeded", (long long)c->cfg.max_device_bytes);
  hipError_t e = hipMalloc(p, bytes ? bytes : 8);
  if (e != hipSuccess) return fail(c, MLSWE_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
  c->bytes += (long long)bytes;
  return MLSWE_OK;
}

void dfree(void* p) {
  if (p) (void)hipFree(p);
}

long long idx(const LevelH& L, int i, int j) { return (long long)(j + 2) * L.pitch + (i + XOFF); }
unsigned blocks(long long n) { return (unsigned)((n + 255) / 256); }

bool valid_prob(mlswe_ctx* c, int p) { return p >= 0 && p < (int)c->probs.size(); }

// grow-only device array
template <class T>
int ensure(mlswe_ctx* c, T** p, int* cap, int n) {
  if (n <= *cap && *p) return MLSWE_OK;
  int nc = std::max(n, std::max(16, *cap * 2));
  dfree(*p);
  *p = nullptr;
  int rc = dalloc(c, (void**)p, sizeof(T) * (size_t)nc);
  if (rc) return rc;
  *cap = nc;
  return MLSWE_OK;
}

// ------------------------------------------------------------ bathymetry
void mirror_frame_host(const LevelH& L, std::vector<double>& a) {
  for (int j = -2; j < L.ny + 2; ++j)
    for (int i = -2; i < L.nx + 2; ++i) {
      if (i >= 0 && j >= 0 && i < L.nx && j < L.ny) continue;
      int si = i < 0 ? -1 - i : (i >= L.nx ? 2 * L.nx - 1 - i : i);
      int sj = j < 0 ? -1 - j : (j >= L.ny ? 2 * L.ny - 1 - j : j);
      a[idx(L, i, j)] = a[idx(L, si, sj)];
    }
}

// ------------------------------------------------------------ clustering
// 16x16 fine tiles marked by a flagged coarse cell, kept if their coarse
// footprint grown by two coarse cells (clipped at the domain) is covered by the
// coarse level (the two bits k_flag_tiles computes per tile), merged greedily
// row-major into rectangles of at most 4x4 tiles.  fnx x fny: the finer level.
std::vector<Box> cluster_tiles(int fnx, int fny, const unsigned char* bits) {
  const int tx = (fnx + TILE - 1) / TILE, ty = (fny + TILE - 1) / TILE;
  std::vector<char> keep((size_t)tx * ty, 0), taken((size_t)tx * ty, 0);
  for (size_t t = 0; t < keep.size(); ++t) keep[t] = (bits[t] & 3) == 3;
  auto free_tile = [&](int I, int J) { return keep[(size_t)J * tx + I] && !taken[(size_t)J * tx + I]; };
  std::vector<Box> out;
  for (int J = 0; J < ty; ++J)
    for (int I = 0; I < tx; ++I) {
      if (!free_tile(I, J)) continue;
      int w = 1;
      while (w < 4 && I + w < tx && free_tile(I + w, J)) ++w;
      int h = 1;
      for (; h < 4 && J + h < ty; ++h) {
        bool full = true;
        for (int a = 0; a < w; ++a) full = full && free_tile(I + a, J + h);
        if (!full) break;
      }
      for (int b = 0; b < h; ++b)
        for (int a = 0; a < w; ++a) taken[(size_t)(J + b) * tx + I + a] = 1;
      Box bx;
      bx.ilo = TILE * I;
      bx.jlo = TILE * J;
      bx.nx = std::min(fnx, TILE * (I + w)) - bx.ilo;
      bx.ny = std::min(fny, TILE * (J + h)) - bx.jlo;
      out.push_back(bx);
    }
  return out;
}

// ------------------------------------------------------------ launch data
// Run tiles of one level of one problem: fixed blocks over the union of its
// patches, x blocks of XTILE_COLS columns by `rows` rows counted from row -2
// (the patches' rows and two frame rows on each side), y blocks of 64 columns
// by `rows` interior rows.  A block is kept where a patch region meets it; bit
// 0 of flags (x) / last (y) marks a block whose successor to the right (x) or
// above (y) is not kept, so that it owns the edge after its last column / row.
// Returns the number of blocks kept; appends tiles when the vectors are given.
long long run_blocks(const LevelH& L, int axis, int rows, int pdi, std::vector<XTile>* xo, std::vector<YTile>* yo,
                     std::vector<int>* rows_out = nullptr) {
  const int w = axis == 0 ? XTILE_COLS : 64;
  const int ns = (L.nx + w - 1) / w;
  const int r0 = axis == 0 ? -2 : 0, hy = axis == 0 ? L.ny + 4 : L.ny;
  const int nc = (hy + rows - 1) / rows;
  std::vector<char> keep((size_t)ns * nc, 0);
  for (const Box& b : L.boxes) {
    const int ja = axis == 0 ? b.jlo - 2 : b.jlo, jb = axis == 0 ? b.jlo + b.ny + 2 : b.jlo + b.ny;
    for (int k = (ja - r0) / rows; k <= (jb - 1 - r0) / rows; ++k)
      for (int s = b.ilo / w; s <= (b.ilo + b.nx - 1) / w; ++s) keep[(size_t)k * ns + s] = 1;
  }
  long long n = 0;
  for (int k = 0; k < nc; ++k)
    for (int s = 0; s < ns; ++s) {
      if (!keep[(size_t)k * ns + s]) continue;
      ++n;
      const int i0 = s * w, j0 = r0 + k * rows;
      const int ncol = std::min(w, L.nx - i0), nrow = std::min(rows, r0 + hy - j0);
      if (rows_out) rows_out->push_back(nrow);
      if (axis == 0 && xo) {
        const bool next = s + 1 < ns && keep[(size_t)k * ns + s + 1];
        xo->push_back(XTile{pdi, i0, ncol, j0, nrow, next ? 0 : 1});
      } else if (axis == 1 && yo) {
        const bool next = k + 1 < nc && keep[(size_t)(k + 1) * ns + s];
        yo->push_back(YTile{pdi, i0, ncol, j0, nrow, next ? 0 : 1});
      }
    }
  return n;
}

// Completion time of tiles started in list order, each on the earliest free of
// `slots` slots, a tile taking 4 time units per row plus `extra` (its start and,
// for y, its halo rows).  Integer times: a count of slots freed at each time.
long long tile_makespan(const std::vector<int>& rows, int extra, long long slots) {
  if (rows.empty() || slots <= 0) return 0;
  std::vector<long long> freed(256, 0);
  freed[0] = slots;
  size_t t = 0;
  long long end = 0;
  for (int r : rows) {
    while (freed[t] == 0) ++t;
    --freed[t];
    const size_t done = t + (size_t)(4 * r + extra);
    if (done >= freed.size()) freed.resize(2 * done + 1, 0);
    ++freed[done];
    end = std::max(end, (long long)done);
  }
  return end;
}

// Flux-correction records of level l (>= 1): every interior cell O of level
// l - 1 outside level l with a face neighbour covered by level l, per problem.
int build_reflux(mlswe_ctx* c, int l, std::vector<RefluxCell>& out) {
  LevelLaunch& LL = c->launch[l];
  const int np = (int)c->probs.size();
  LL.rfx_first.assign(np, 0);
  LL.rfx_count.assign(np, 0);
  out.clear();
  for (int p = 0; p < np; ++p) {
    ProblemH& P = c->probs[p];
    LL.rfx_first[p] = (int)out.size();
    if (l >= P.nlev || P.L[l].boxes.empty()) continue;
    LevelH& Lc = P.L[l - 1];
    LevelH& Lf = P.L[l];
    const int r = P.ratio[l - 1];
    const int nx = Lc.nx, ny = Lc.ny;
    std::vector<unsigned char> inc((size_t)nx * ny, 0), fin((size_t)nx * ny, 0);
    for (const Box& b : Lc.boxes)
      for (int j = b.jlo; j < b.jlo + b.ny; ++j)
        for (int i = b.ilo; i < b.ilo + b.nx; ++i) inc[(size_t)j * nx + i] = 1;
    for (const Box& b : Lf.boxes)
      for (int j = b.jlo / r; j < (b.jlo + b.ny) / r; ++j)
        for (int i = b.ilo / r; i < (b.ilo + b.nx) / r; ++i) fin[(size_t)j * nx + i] = 1;
    std::vector<int> at((size_t)nx * ny, -1);
    const int di[4] = {-1, 1, 0, 0}, dj[4] = {0, 0, -1, 1};  // O = N + (di, dj) for direction d
    for (const Box& b : Lf.boxes) {
      const int I0 = b.ilo / r, I1 = (b.ilo + b.nx) / r - 1, J0 = b.jlo / r, J1 = (b.jlo + b.ny) / r - 1;
      for (int d = 0; d < 4; ++d) {
        const int n = d < 2 ? J1 - J0 + 1 : I1 - I0 + 1;
        for (int k = 0; k < n; ++k) {
          // N on the box side facing O
          const int Ni = d == 0 ? I0 : d == 1 ? I1 : I0 + k;
          const int Nj = d < 2 ? J0 + k : d == 2 ? J0 : J1;
          const int Oi = Ni + di[d], Oj = Nj + dj[d];
          if (Oi < 0 || Oj < 0 || Oi >= nx || Oj >= ny) continue;
          const size_t o = (size_t)Oj * nx + Oi;
          if (!inc[o] || fin[o]) continue;
          if (at[o] < 0) {
            RefluxCell R;
            std::memset(&R, 0, sizeof R);
            R.cq[0] = Lc.q[0]; R.cq[1] = Lc.q[1]; R.cqs = Lc.qs; R.cB = Lc.B;
            R.fq[0] = Lf.q[0]; R.fq[1] = Lf.q[1]; R.fqs = Lf.qs; R.fB = Lf.B;
            R.cctl = c->ctl + P.ctl0 + (l - 1);
            R.fctl = c->ctl + P.ctl0 + l;
            R.cpitch = Lc.pitch; R.cplane = Lc.plane; R.fpitch = Lf.pitch; R.fplane = Lf.plane;
            R.i = Oi; R.j = Oj; R.dirs = 0; R.r = r;
            R.cdx = Lc.dx; R.cdy = Lc.dy; R.fdx = Lf.dx; R.fdy = Lf.dy;
            R.P = P.P;
            at[o] = (int)out.size();
            out.push_back(R);
          }
          out[at[o]].dirs |= 1 << d;
        }
      }
    }
    LL.rfx_count[p] = (int)out.size() - LL.rfx_first[p];
  }
  LL.nrfx = (int)out.size();
  return MLSWE_OK;
}

int build_launch(mlswe_ctx* c, int l) {
  LevelLaunch& LL = c->launch[l];
  if (!LL.dirty) return MLSWE_OK;
  // Rows per sweep wave: the tuned value, or (0) the candidate whose tiles, in
  // launch order, finish first by the list-schedule model above, with 24 (x) /
  // 16 (y) slots per compute unit (twice the lean kernels' resident waves: a
  // SIMD's waves share it, so it balances finer than whole tiles) and a tile's
  // start worth half a row (x) or its halo worth 2.5 rows (y), values fitted to
  // sweep times of uniform grids, batches of uneven problems and their union
  // tiles.  Ties keep the taller tiles.
  const int xc[4] = {32, 16, 8, 4}, yc[5] = {128, 64, 32, 16, 8};
  auto pick = [&](int axis, int tuned, const std::function<void(int, std::vector<int>&)>& rows_of) {
    if (tuned > 0) return tuned;
    const int* cand = axis == 0 ? xc : yc;
    const int nc = axis == 0 ? 4 : 5;
    const long long slots = (axis == 0 ? 24LL : 16LL) * c->ncu;
    long long best = -1;
    int br = cand[0];
    std::vector<int> d;
    for (int k = 0; k < nc; ++k) {
      d.clear();
      rows_of(cand[k], d);
      const long long m = tile_makespan(d, axis == 0 ? 2 : 10, slots);
      if (best < 0 || m < best) { best = m; br = cand[k]; }
    }
    return br;
  };
  auto patch_rows = [&](int axis, int rows, std::vector<int>& d) {
    for (const ProblemH& P : c->probs) {
      if (l >= P.nlev) continue;
      for (const Box& b : P.L[l].boxes) {
        const int ns = axis == 0 ? (b.nx + XTILE_COLS - 1) / XTILE_COLS : (b.nx + 63) / 64;
        const int h = axis == 0 ? b.ny + 4 : b.ny;
        for (int j = 0; j < h; j += rows)
          for (int s = 0; s < ns; ++s) d.push_back(std::min(rows, h - j));
      }
    }
  };
  // run tiles serve levels where some problem has several patches; their rows
  // follow the same rule over the run blocks.  The patch tiles of such a level
  // serve only plain launches (one patch per launch, a few waves each) and
  // persistent schedules (balanced by the schedule): both do best with the
  // shortest tiles, 4 (x) and 8 (y) rows.
  LL.use_runs = false;
  size_t npatch = 0;
  for (const ProblemH& P : c->probs)
    if (l < P.nlev) {
      if (P.L[l].boxes.size() > 1) LL.use_runs = true;
      npatch += P.L[l].boxes.size();
    }
  // the model's choices are kept while the level's cells and patch count stay
  // within a quarter of those it was last evaluated on (a regrid moves the
  // patches, the best heights change only with the layout's scale)
  long long cells = 0;
  for (const ProblemH& P : c->probs)
    if (l < P.nlev)
      for (const Box& b : P.L[l].boxes) cells += (long long)b.nx * b.ny;
  const bool similar = LL.model_cells > 0 && LL.model_runs == LL.use_runs &&
                       4 * std::llabs(cells - LL.model_cells) <= LL.model_cells &&
                       4 * std::llabs((long long)npatch - LL.model_patches) <= LL.model_patches;
  if (!similar) {
    LL.model_cells = cells;
    LL.model_patches = (long long)npatch;
    LL.model_runs = LL.use_runs;
    if (LL.use_runs) {
      LL.model_rows[0] = 4;
      LL.model_rows[1] = 8;
    } else {
      LL.model_rows[0] = pick(0, 0, [&](int r, std::vector<int>& d) { patch_rows(0, r, d); });
      LL.model_rows[1] = pick(1, 0, [&](int r, std::vector<int>& d) { patch_rows(1, r, d); });
    }
  }
  LL.rows_x = c->tune.x_rows > 0 ? c->tune.x_rows : LL.model_rows[0];
  LL.rows_y = c->tune.y_rows > 0 ? c->tune.y_rows : LL.model_rows[1];
  auto run_rows = [&](int axis, int rows, std::vector<int>& d) {
    for (const ProblemH& P : c->probs)
      if (l < P.nlev && !P.L[l].boxes.empty()) run_blocks(P.L[l], axis, rows, 0, nullptr, nullptr, &d);
  };
  if (!similar && LL.use_runs) {
    LL.model_rows[2] = pick(0, 0, [&](int r, std::vector<int>& d) { run_rows(0, r, d); });
    LL.model_rows[3] = pick(1, 0, [&](int r, std::vector<int>& d) { run_rows(1, r, d); });
  }
  LL.rows_xr = LL.use_runs ? (c->tune.x_rows > 0 ? c->tune.x_rows : LL.model_rows[2]) : 0;
  LL.rows_yr = LL.use_runs ? (c->tune.y_rows > 0 ? c->tune.y_rows : LL.model_rows[3]) : 0;
  const int xrows = LL.rows_x, yrows = LL.rows_y;
  std::vector<PatchDev> pd[2];
  std::vector<XTile> xt;
  std::vector<YTile> yt;
  std::vector<FillPatch> fp[4];
  std::vector<CoarsenPatch> cp[4];
  std::vector<LevelInfo> li;
  LL.patch_prob.clear(); LL.xr.clear(); LL.yr.clear();
  for (int par = 0; par < 2; ++par) pd[par].reserve(npatch + c->probs.size());
  for (int k = 0; k < 4; ++k) { fp[k].reserve(npatch); cp[k].reserve(npatch); }
  LL.patch_prob.reserve(npatch); LL.xr.reserve(npatch); LL.yr.reserve(npatch);
  xt.reserve(8 * npatch); yt.reserve(4 * npatch);
  li.reserve(c->probs.size());
  LL.fill_first.assign(c->probs.size(), -1);
  LL.fill_count.assign(c->probs.size(), 0);
  LL.crs_first.assign(c->probs.size(), -1);
  LL.crs_count.assign(c->probs.size(), 0);
  LL.li_first.assign(c->probs.size(), -1);
  for (size_t pi = 0; pi < c->probs.size(); ++pi) {
    ProblemH& P = c->probs[pi];
    if (l >= P.nlev) continue;
    LevelH& L = P.L[l];
    LL.li_first[pi] = (int)li.size();
    LevelInfo info;
    info.ctl = P.ctl0 + l; info.cnt = P.cnt; info.dx = L.dx; info.dy = L.dy;
    info.x0 = (int)xt.size(); info.nx = 0; info.y0 = (int)yt.size(); info.ny = 0;  // y0: offset added below
    li.push_back(info);
    if (L.boxes.empty()) continue;
    LL.fill_first[pi] = (int)fp[0].size();
    LL.fill_count[pi] = (int)L.boxes.size();
    LL.crs_first[pi] = (int)cp[0].size();
    for (const Box& b : L.boxes) {
      const int id = (int)pd[0].size();
      for (int par = 0; par < 2; ++par) {
        PatchDev d;
        d.q = L.q[par]; d.qo = L.q[1 - par]; d.qs = L.qs; d.B = L.B;
        d.ctl = c->ctl + P.ctl0 + l; d.cnt = c->cnt + P.cnt;
        d.pitch = L.pitch; d.plane = L.plane;
        d.ilo = b.ilo; d.jlo = b.jlo; d.nx = b.nx; d.ny = b.ny;
        d.dx = L.dx; d.dy = L.dy; d.P = P.P;
        d.sig_on = c->sig_on;
        d.mask = L.mask;
        pd[par].push_back(d);
      }
      LL.patch_prob.push_back((int)pi);
      const int x0 = (int)xt.size();
      // tiles row-major within the patch (the launch hands contiguous bands of
      // them to the XCDs, so a band is a strip of whole tile rows)
      for (int j0 = b.jlo - 2; j0 < b.jlo + b.ny + 2; j0 += xrows)
        for (int i0 = b.ilo; i0 < b.ilo + b.nx; i0 += XTILE_COLS)
          xt.push_back(XTile{id, i0, std::min(XTILE_COLS, b.ilo + b.nx - i0), j0,
                             std::min(xrows, b.jlo + b.ny + 2 - j0)});
      const int y0 = (int)yt.size();
      for (int j0 = b.jlo; j0 < b.jlo + b.ny; j0 += yrows) {
        const int nr = std::min(yrows, b.jlo + b.ny - j0);
        for (int i0 = b.ilo; i0 < b.ilo + b.nx; i0 += 64)
          yt.push_back(YTile{id, i0, std::min(64, b.ilo + b.nx - i0), j0, nr, (j0 + nr == b.jlo + b.ny) ? 1 : 0});
      }
      LL.xr.push_back({x0, (int)xt.size() - x0});
      LL.yr.push_back({y0, (int)yt.size() - y0});
      // fill and coarsen descriptors for the four buffer parities (fine, coarse)
      FillPatch f;
      std::memset(&f, 0, sizeof f);
      f.B = L.B; f.mask = L.mask;
      f.cnt = c->cnt + P.cnt;
      f.pitch = L.pitch; f.plane = L.plane;
      f.nx = L.nx; f.ny = L.ny;
      f.ilo = b.ilo; f.jlo = b.jlo; f.bnx = b.nx; f.bny = b.ny;
      f.P = P.P;
      CoarsenPatch cc;
      std::memset(&cc, 0, sizeof cc);
      const LevelH* Cl = l > 0 ? &P.L[l - 1] : nullptr;
      if (Cl) {
        f.Bc = Cl->B;
        f.cpitch = Cl->pitch; f.cplane = Cl->plane; f.ncx = Cl->nx; f.ncy = Cl->ny;
        f.r = P.ratio[l - 1];
        f.coarse_none = 0;
        cc.fpitch = L.pitch; cc.fplane = L.plane; cc.cpitch = Cl->pitch; cc.cplane = Cl->plane;
        cc.ilo = b.ilo; cc.jlo = b.jlo; cc.bnx = b.nx; cc.bny = b.ny; cc.r = P.ratio[l - 1];
        cc.P = P.P;
      } else {
        f.coarse_none = 1;
        f.r = 1;
      }
      for (int fpar = 0; fpar < 2; ++fpar)
        for (int cpar = 0; cpar < 2; ++cpar) {
          f.q = L.q[fpar];
          if (Cl) { f.qco = Cl->q[1 - cpar]; f.qcn = Cl->q[cpar]; }
          fp[fpar * 2 + cpar].push_back(f);
        }
      // coarsening in chunks of whole coarse rows, about 256 coarse cells each,
      // so that every block of its launch has work
      if (Cl) {
        const int r = P.ratio[l - 1], cnx = b.nx / r, cny = b.ny / r;
        const int rows = std::max(1, 256 / std::max(1, cnx));
        for (int j = 0; j < cny; j += rows) {
          cc.jlo = b.jlo + j * r;
          cc.bny = std::min(rows, cny - j) * r;
          for (int fpar = 0; fpar < 2; ++fpar)
            for (int cpar = 0; cpar < 2; ++cpar) {
              cc.qf = L.q[fpar]; cc.qc = Cl->q[cpar];
              cp[fpar * 2 + cpar].push_back(cc);
            }
        }
      }
    }
    LL.crs_count[pi] = (int)cp[0].size() - LL.crs_first[pi];
    li.back().nx = (int)xt.size() - li.back().x0;
    li.back().ny = (int)yt.size() - li.back().y0;
  }
  LL.nptch = (int)pd[0].size();
  LL.nxt_p = (int)xt.size();
  LL.nyt_p = (int)yt.size();
  // run tiles of each problem, over a level descriptor that follows the patch
  // descriptors (the patch extent fields are unused there)
  LL.xrun.assign(c->probs.size(), {0, 0});
  LL.yrun.assign(c->probs.size(), {0, 0});
  std::vector<LevelInfo> li_run = li;
  if (LL.use_runs) {
    int k = 0;
    for (size_t pi = 0; pi < c->probs.size(); ++pi) {
      ProblemH& P = c->probs[pi];
      if (l >= P.nlev) continue;
      LevelH& L = P.L[l];
      LevelInfo& info = li_run[k++];
      info.x0 = (int)xt.size(); info.y0 = (int)yt.size();
      if (!L.boxes.empty()) {
        const int id = (int)pd[0].size();
        for (int par = 0; par < 2; ++par) {
          PatchDev d = pd[par][LL.fill_first[pi]];  // the problem's first patch
          d.ilo = 0; d.jlo = 0; d.nx = L.nx; d.ny = L.ny;
          pd[par].push_back(d);
        }
        run_blocks(L, 0, LL.rows_xr, id, &xt, nullptr);
        run_blocks(L, 1, LL.rows_yr, id, nullptr, &yt);
      }
      info.nx = (int)xt.size() - info.x0;
      info.ny = (int)yt.size() - info.y0;
      LL.xrun[pi] = {info.x0, info.nx};
      LL.yrun[pi] = {info.y0, info.ny};
    }
  }
  LL.nxt = (int)xt.size();
  LL.nyt = (int)yt.size();
  LL.nli = (int)li.size();
  LL.max_info_tiles = 0;
  // four copies: x ranges of patch (0) or run (1) tiles, plus 2 for run y ranges
  std::vector<LevelInfo> li4(4 * (size_t)LL.nli);
  for (int k = 0; k < LL.nli; ++k)
    for (int v = 0; v < 4; ++v) {
      LevelInfo info = li[k];
      const LevelInfo& rinfo = li_run[k];
      if ((v & 1) && LL.use_runs) { info.x0 = rinfo.x0; info.nx = rinfo.nx; }
      if ((v & 2) && LL.use_runs) { info.y0 = rinfo.y0; info.ny = rinfo.ny; }
      info.y0 += LL.nxt;
      LL.max_info_tiles = std::max(LL.max_info_tiles, info.nx + info.ny);
      li4[(size_t)v * LL.nli + k] = info;
    }
  const int npd = (int)pd[0].size();
  int rc;
  int cap_pd1 = LL.cap_pd;
  if ((rc = ensure(c, &LL.pd[0], &LL.cap_pd, npd))) return rc;
  if ((rc = ensure(c, &LL.pd[1], &cap_pd1, npd))) return rc;
  if ((rc = ensure(c, &LL.xt, &LL.cap_xt, LL.nxt))) return rc;
  if ((rc = ensure(c, &LL.yt, &LL.cap_yt, LL.nyt))) return rc;
  LL.ncrs = (int)cp[0].size();
  int capf[4] = {LL.cap_fp, LL.cap_fp, LL.cap_fp, LL.cap_fp};
  int capc[4] = {LL.cap_cp, LL.cap_cp, LL.cap_cp, LL.cap_cp};
  for (int k = 0; k < 4; ++k) {
    if ((rc = ensure(c, &LL.fp[k], &capf[k], LL.nptch))) return rc;
    if ((rc = ensure(c, &LL.cp[k], &capc[k], std::max(1, LL.ncrs)))) return rc;
  }
  LL.cap_fp = capf[0];
  LL.cap_cp = capc[0];
  if ((rc = ensure(c, &LL.li, &LL.cap_li, 4 * LL.nli))) return rc;
  if ((rc = ensure(c, &LL.parts, &LL.cap_parts, LL.nxt + LL.nyt))) return rc;
  if (LL.nptch) {
    HIPCHK(c, hipMemcpyAsync(LL.pd[0], pd[0].data(), sizeof(PatchDev) * npd, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(LL.pd[1], pd[1].data(), sizeof(PatchDev) * npd, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(LL.xt, xt.data(), sizeof(XTile) * LL.nxt, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(LL.yt, yt.data(), sizeof(YTile) * LL.nyt, hipMemcpyHostToDevice, c->stream));
    for (int k = 0; k < 4; ++k) {
      HIPCHK(c, hipMemcpyAsync(LL.fp[k], fp[k].data(), sizeof(FillPatch) * LL.nptch, hipMemcpyHostToDevice, c->stream));
      if (LL.ncrs)
        HIPCHK(c, hipMemcpyAsync(LL.cp[k], cp[k].data(), sizeof(CoarsenPatch) * LL.ncrs, hipMemcpyHostToDevice, c->stream));
    }
  }
  if (LL.nli)
    HIPCHK(c, hipMemcpyAsync(LL.li, li4.data(), sizeof(LevelInfo) * li4.size(), hipMemcpyHostToDevice, c->stream));
  std::vector<RefluxCell> rfx;
  if (c->cfg.reflux && l >= 1) {
    if ((rc = build_reflux(c, l, rfx))) return rc;
    if ((rc = ensure(c, &LL.rfx, &LL.cap_rfx, std::max(1, LL.nrfx)))) return rc;
    if ((rc = ensure(c, &LL.rfx_reg, &LL.cap_rfx_reg, REFLUX_REG * std::max(1, LL.nrfx)))) return rc;
    for (int k = 0; k < LL.nrfx; ++k) rfx[k].reg = LL.rfx_reg + REFLUX_REG * (size_t)k;
    if (LL.nrfx)
      HIPCHK(c, hipMemcpyAsync(LL.rfx, rfx.data(), sizeof(RefluxCell) * LL.nrfx, hipMemcpyHostToDevice, c->stream));
  }
  // host vectors must outlive the asynchronous copies
  HIPCHK(c, hipStreamSynchronize(c->stream));
  LL.dirty = false;
  return MLSWE_OK;
}

void mark_dirty(mlswe_ctx* c, int l) {
  c->generation++;
  if (l >= 0 && l < MAXLEV) c->launch[l].dirty = true;
  if (l + 1 < MAXLEV) c->launch[l + 1].dirty = true;  // fill/coarsen descriptors of the finer level
  c->pdt_dirty = true;
}

int build_pdt(mlswe_ctx* c) {
  if (!c->pdt_dirty) return MLSWE_OK;
  std::vector<ProbDt> v(c->probs.size());
  for (size_t i = 0; i < c->probs.size(); ++i) {
    const ProblemH& P = c->probs[i];
    ProbDt d;
    std::memset(&d, 0, sizeof d);
    d.ctl0 = P.ctl0; d.nlev = P.nlev;
    for (int l = 0; l < P.nlev; ++l) {
      d.ratio[l] = P.ratio[l];
      d.rt[l] = P.rt[l];
      d.active[l] = P.L[l].boxes.empty() ? 0 : 1;
      d.dx[l] = P.L[l].dx; d.dy[l] = P.L[l].dy;
    }
    d.dt_out = nullptr;
    v[i] = d;
  }
  int rc = ensure(c, &c->pdt, &c->pdt_cap, (int)v.size());
  if (rc) return rc;
  HIPCHK(c, hipMemcpyAsync(c->pdt, v.data(), sizeof(ProbDt) * v.size(), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->pdt_dirty = false;
  return MLSWE_OK;
}

// ------------------------------------------------------------ timing
int ev_begin(mlswe_ctx* c, hipEvent_t* e) {
  if (c->ev_pool.empty()) {
    hipEvent_t a;
    HIPCHK(c, hipEventCreate(&a));
    c->ev_pool.push_back(a);
  }
  *e = c->ev_pool.back();
  c->ev_pool.pop_back();
  HIPCHK(c, hipEventRecord(*e, c->stream));
  return MLSWE_OK;
}

int collect_events(mlswe_ctx* c) {
  if (c->ev_used.empty()) return MLSWE_OK;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (auto& u : c->ev_used) {
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, u.second.first, u.second.second));
    c->kms[u.first] += ms;
    c->klaunch[u.first] += 1;
    c->ev_pool.push_back(u.second.first);
    c->ev_pool.push_back(u.second.second);
  }
  c->ev_used.clear();
  return MLSWE_OK;
}

// Brackets the launches that fn queues with two events of class cls when timing
// is on (never inside a graph capture: timing runs the eager path).
template <class F>
int timed(mlswe_ctx* c, int cls, F&& fn) {
  if (!c->timing) return fn();
  hipEvent_t e0, e1;
  int rc;
  if ((rc = ev_begin(c, &e0))) return rc;
  if ((rc = fn())) return rc;
  if ((rc = ev_begin(c, &e1))) return rc;
  c->ev_used.push_back({cls, {e0, e1}});
  if (c->ev_used.size() > 4096) return collect_events(c);
  return MLSWE_OK;
}

// ------------------------------------------------------------ launches
// Sweeps over tile ranges of level l; rx / ry: the ranges are run tiles.
int launch_sweeps(mlswe_ctx* c, int l, int parity, int xt0, int nxt, int yt0, int nyt, bool rx = false,
                  bool ry = false) {
  LevelLaunch& LL = c->launch[l];
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc;
  const int sx = c->tune.sched_x, sy = c->tune.sched_y;
  // one wave per tile: a multiple of eight blocks (the kernels hand each XCD a
  // band of the tiles); persistent schedules: a multiple of the compute units
  auto grid_of = [&](int ntiles, int sched, int mult) {
    const int need = (ntiles + 3) / 4;
    if (sched == 0) return (need + 7) / 8 * 8;
    const int g = std::max(1, mult) * c->ncu;
    return std::min(need, g);
  };
  if ((sx == 2 && nxt > 0) || (sy == 2 && nyt > 0))
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, c->stream, c->tickets, 2);
  if (nxt > 0) {
    if (c->timing && (rc = ev_begin(c, &e0))) return rc;
    if (rx)
      hipLaunchKernelGGL(c->tune.fast ? k_sweep_xr_fast : k_sweep_xr, dim3(grid_of(nxt, 0, 0)), dim3(256), 0,
                         c->stream, LL.pd[parity], LL.xt + xt0, nxt, LL.parts + xt0);
    else if (sx == 0 && !c->sig_on)  // one wave per tile, no signature: the lean kernels
      hipLaunchKernelGGL(c->tune.fast ? k_sweep_x1_fast : k_sweep_x1, dim3(grid_of(nxt, 0, 0)), dim3(256), 0,
                         c->stream, LL.pd[parity], LL.xt + xt0, nxt, LL.parts + xt0);
    else
      hipLaunchKernelGGL(c->tune.fast ? k_sweep_x_fast : k_sweep_x, dim3(grid_of(nxt, sx, c->tune.grid_x)), dim3(256),
                         0, c->stream, LL.pd[parity], LL.xt + xt0, nxt, sx, c->tickets, LL.parts + xt0);
    HIPCHK(c, hipGetLastError());
    if (c->timing) {
      if ((rc = ev_begin(c, &e1))) return rc;
      c->ev_used.push_back({0, {e0, e1}});
    }
  }
  if (nyt > 0) {
    if (c->timing && (rc = ev_begin(c, &e0))) return rc;
    if (ry)
      hipLaunchKernelGGL(c->tune.fast ? k_sweep_yr_fast : k_sweep_yr, dim3(grid_of(nyt, 0, 0)), dim3(256), 0,
                         c->stream, LL.pd[parity], LL.yt + yt0, nyt, LL.parts + LL.nxt + yt0);
    else if (sy == 0 && !c->sig_on)
      hipLaunchKernelGGL(c->tune.fast ? k_sweep_y1_fast : k_sweep_y1, dim3(grid_of(nyt, 0, 0)), dim3(256), 0,
                         c->stream, LL.pd[parity], LL.yt + yt0, nyt, LL.parts + LL.nxt + yt0);
    else
      hipLaunchKernelGGL(c->tune.fast ? k_sweep_y_fast : k_sweep_y, dim3(grid_of(nyt, sy, c->tune.grid_y)), dim3(256),
                         0, c->stream, LL.pd[parity], LL.yt + yt0, nyt, sy, c->tickets + 1, LL.parts + LL.nxt + yt0);
    HIPCHK(c, hipGetLastError());
    if (c->timing) {
      if ((rc = ev_begin(c, &e1))) return rc;
      c->ev_used.push_back({1, {e0, e1}});
    }
  }
  if (c->ev_used.size() > 4096) return collect_events(c);
  return MLSWE_OK;
}

// Ghost fill of level l for the problems in [p0, p1) (all with the level).
int launch_fill(mlswe_ctx* c, int l, int p0, int p1, double theta) {
  LevelLaunch& LL = c->launch[l];
  const ProblemH& P0 = c->probs[p0];
  const int fpar = P0.L[l].cur;
  const int cpar = l > 0 ? P0.L[l - 1].cur : 0;
  int first = -1, count = 0, maxring = 0;
  bool walls = false;  // some patch's two-cell frame leaves the domain
  for (int p = p0; p < p1; ++p) {
    if (LL.fill_first[p] < 0) continue;
    if (first < 0) first = LL.fill_first[p];
    count = LL.fill_first[p] + LL.fill_count[p] - first;
    const LevelH& L = c->probs[p].L[l];
    for (const Box& b : L.boxes) {
      maxring = std::max(maxring, 4 * (b.nx + 4) + 4 * b.ny);
      walls = walls || b.ilo < 2 || b.jlo < 2 || b.ilo + b.nx > L.nx - 2 || b.jlo + b.ny > L.ny - 2;
    }
  }
  if (count == 0) return MLSWE_OK;
  const FillPatch* f = LL.fp[fpar * 2 + cpar] + first;
  if (l > 0) {
    hipLaunchKernelGGL(k_ghost_fill, dim3((maxring + 255) / 256, count), dim3(256), 0, c->stream, f, 0, theta);
    HIPCHK(c, hipGetLastError());
  }
  // the second pass only mirrors frame cells outside the domain
  if (walls) {
    hipLaunchKernelGGL(k_ghost_fill, dim3((maxring + 255) / 256, count), dim3(256), 0, c->stream, f, 1, theta);
    HIPCHK(c, hipGetLastError());
  }
  return MLSWE_OK;
}

// runs: bit 0 the x tiles were run tiles, bit 1 the y tiles.
int launch_after(mlswe_ctx* c, int l, int p0, int p1, int runs) {
  LevelLaunch& LL = c->launch[l];
  int first = -1, n = 0;
  for (int p = p0; p < p1; ++p) {
    if (LL.li_first[p] < 0) continue;
    if (first < 0) first = LL.li_first[p];
    n = LL.li_first[p] + 1 - first;
  }
  if (n == 0) return MLSWE_OK;
  // one wave per problem suffices for a few tiles; a problem with many gets 16
  hipLaunchKernelGGL(k_after_substep, dim3(n), dim3(LL.max_info_tiles > 256 ? 1024 : 64), 0, c->stream, c->ctl, c->cnt,
                     LL.li + (size_t)runs * LL.nli + first, LL.parts, c->cfg.cfl_max);
  HIPCHK(c, hipGetLastError());
  return MLSWE_OK;
}

// Flux-correction launch over the records of level lf for problems [p0, p1):
// which 0 coarse face fluxes (after a level lf - 1 substep), 1 fine face fluxes
// (after a level lf substep), 2 the correction (after coarsening level lf).
int launch_reflux(mlswe_ctx* c, int lf, int p0, int p1, int which, int parity) {
  if (!c->cfg.reflux || lf < 1 || lf >= MAXLEV) return MLSWE_OK;
  bool has = false;  // no problem of the range has level lf: nothing to build or launch
  for (int p = p0; p < p1; ++p) has = has || lf < c->probs[p].nlev;
  if (!has) return MLSWE_OK;
  int rc;
  if ((rc = build_launch(c, lf))) return rc;
  LevelLaunch& LL = c->launch[lf];
  int first = -1, count = 0;
  for (int p = p0; p < p1 && p < (int)LL.rfx_first.size(); ++p) {
    if (LL.rfx_count[p] == 0) continue;
    if (first < 0) first = LL.rfx_first[p];
    count = LL.rfx_first[p] + LL.rfx_count[p] - first;
  }
  if (count == 0) return MLSWE_OK;
  auto blocks_of = [](long long threads) { return dim3((unsigned)((threads + 63) / 64)); };
  const dim3 block(64);
  if (which == 0) {
    hipLaunchKernelGGL(k_reflux_coarse, blocks_of(4LL * count), block, 0, c->stream, LL.rfx + first, count, parity);
  } else if (which == 1) {
    hipLaunchKernelGGL(k_reflux_fine, blocks_of(64LL * count), block, 0, c->stream, LL.rfx + first, count, parity);
    HIPCHK(c, hipGetLastError());
    hipLaunchKernelGGL(k_reflux_fsum, blocks_of(count), block, 0, c->stream, LL.rfx + first, count);
  } else {
    hipLaunchKernelGGL(k_reflux_apply, blocks_of(count), block, 0, c->stream, LL.rfx + first, count, parity,
                       c->probs[p0].rt[lf - 1]);
  }
  HIPCHK(c, hipGetLastError());
  return MLSWE_OK;
}

// One substep of level l for problems [p0, p1): fill, sweeps, buffer flip.
int substep(mlswe_ctx* c, int l, int p0, int p1, double theta, bool batched) {
  int rc;
  if ((rc = build_launch(c, l))) return rc;
  if (l > 0 && (rc = build_launch(c, l - 1))) return rc;
  LevelLaunch& LL = c->launch[l];
  if ((rc = timed(c, 2, [&] { return launch_fill(c, l, p0, p1, theta); }))) return rc;
  const int parity = c->probs[p0].L[l].cur;
  for (int p = p0; p < p1; ++p)
    if (l < c->probs[p].nlev && c->probs[p].L[l].cur != parity)
      return fail(c, MLSWE_ESTATE, "problems out of step on level %d", l);
  // patches of [p0, p1) are contiguous in the launch data
  int a = -1, b = -1;
  for (int k = 0; k < LL.nptch; ++k)
    if (LL.patch_prob[k] >= p0 && LL.patch_prob[k] < p1) {
      if (a < 0) a = k;
      b = k;
    }
  int runs = 0;
  if (a >= 0) {
    if (batched) {
      int xt0 = LL.xr[a].first, nxt = LL.xr[b].first + LL.xr[b].second - xt0;
      int yt0 = LL.yr[a].first, nyt = LL.yr[b].first + LL.yr[b].second - yt0;
      // levels with several patches per problem: one-wave run tiles over the union
      const bool rx = LL.use_runs && c->tune.sched_x == 0 && !c->sig_on;
      const bool ry = LL.use_runs && c->tune.sched_y == 0 && !c->sig_on;
      auto run_range = [&](const std::vector<std::pair<int, int>>& rr, int& t0, int& n) {
        int e = -1;
        t0 = -1;
        for (int p = p0; p < p1; ++p) {
          if (rr[p].second == 0) continue;
          if (t0 < 0) t0 = rr[p].first;
          e = rr[p].first + rr[p].second;
        }
        n = t0 < 0 ? 0 : e - t0;
        if (t0 < 0) t0 = 0;
      };
      if (rx) run_range(LL.xrun, xt0, nxt);
      if (ry) run_range(LL.yrun, yt0, nyt);
      runs = (rx ? 1 : 0) | (ry ? 2 : 0);
      if ((rc = launch_sweeps(c, l, parity, xt0, nxt, yt0, nyt, rx, ry))) return rc;
    } else {
      // plain: x then y of every patch, one launch each
      for (int k = a; k <= b; ++k)
        if ((rc = launch_sweeps(c, l, parity, LL.xr[k].first, LL.xr[k].second, LL.yr[k].first, LL.yr[k].second)))
          return rc;
    }
  }
  if (c->cfg.reflux) {
    // face fluxes from this substep's sweep inputs (still intact): as the coarse
    // side of the finer level's faces, and as the fine side of this level's
    if (l + 1 < MAXLEV && (rc = timed(c, 5, [&] { return launch_reflux(c, l + 1, p0, p1, 0, parity); }))) return rc;
    if (l >= 1 && (rc = timed(c, 5, [&] { return launch_reflux(c, l, p0, p1, 1, parity); }))) return rc;
  }
  for (int p = p0; p < p1; ++p) {
    ProblemH& P = c->probs[p];
    if (l >= P.nlev) continue;
    LevelH& L = P.L[l];
    L.cur = 1 - L.cur;
    for (const Box& bx : L.boxes) P.updates[l] += (long long)bx.nx * bx.ny;
  }
  return timed(c, 3, [&] { return launch_after(c, l, p0, p1, runs); });
}

// apply_reflux: the coarsening ends a coarse level's substep inside a coarse
// step, so the flux correction (if on) follows it.
int coarsen_level(mlswe_ctx* c, int lf, int p0, int p1, bool apply_reflux = false) {
  int rc;
  if ((rc = build_launch(c, lf))) return rc;
  LevelLaunch& LL = c->launch[lf];
  int first = -1, count = 0, maxc = 0;
  for (int p = p0; p < p1; ++p) {
    if (LL.crs_first[p] < 0 || LL.crs_count[p] == 0) continue;
    if (first < 0) first = LL.crs_first[p];
    count = LL.crs_first[p] + LL.crs_count[p] - first;
    const int r = c->probs[p].ratio[lf - 1];
    for (const Box& b : c->probs[p].L[lf].boxes) {
      const int cnx = b.nx / r, rows = std::max(1, 256 / std::max(1, cnx));
      maxc = std::max(maxc, cnx * std::min(rows, b.ny / r));
    }
  }
  if (count == 0) return MLSWE_OK;
  const int fpar = c->probs[p0].L[lf].cur, cpar = c->probs[p0].L[lf - 1].cur;
  rc = timed(c, 4, [&]() -> int {
    for (int k0 = 0; k0 < count; k0 += 65535)  // grid y is at most 65535
      hipLaunchKernelGGL(k_coarsen, dim3((maxc + 255) / 256, (unsigned)std::min(65535, count - k0)), dim3(256), 0,
                         c->stream, LL.cp[fpar * 2 + cpar] + first + k0);
    HIPCHK(c, hipGetLastError());
    return MLSWE_OK;
  });
  if (rc) return rc;
  return apply_reflux && c->cfg.reflux ? timed(c, 5, [&] { return launch_reflux(c, lf, p0, p1, 2, cpar); })
                                       : MLSWE_OK;
}

bool level_active(const mlswe_ctx* c, int l, int p0, int p1) {
  for (int p = p0; p < p1; ++p)
    if (l < c->probs[p].nlev && !c->probs[p].L[l].boxes.empty()) return true;
  return false;
}

int adv(mlswe_ctx* c, int l, int p0, int p1, double theta, bool batched) {
  int rc;
  if ((rc = substep(c, l, p0, p1, theta, batched))) return rc;
  const ProblemH& P0 = c->probs[p0];
  if (l + 1 < P0.nlev && level_active(c, l + 1, p0, p1)) {
    const int r = P0.rt[l];
    for (int k = 0; k < r; ++k)
      if ((rc = adv(c, l + 1, p0, p1, double(k) / double(r), batched))) return rc;
    if ((rc = coarsen_level(c, l + 1, p0, p1, true))) return rc;
  }
  return MLSWE_OK;
}

int next_dt(mlswe_ctx* c, int p0, int p1, bool initial) {
  int rc;
  if ((rc = build_pdt(c))) return rc;
  if (initial) {
    std::vector<SpeedLevel> sl;
    for (int p = p0; p < p1; ++p) {
      ProblemH& P = c->probs[p];
      for (int l = 0; l < P.nlev; ++l) {
        if (P.L[l].boxes.empty()) continue;
        LevelH& L = P.L[l];
        SpeedLevel s;
        s.q = L.q[L.cur]; s.mask = L.mask; s.ctl = c->ctl + P.ctl0 + l;
        s.pitch = L.pitch; s.plane = L.plane; s.nx = L.nx; s.ny = L.ny;
        s.g = P.P.g; s.hdry = P.P.hdry;
        sl.push_back(s);
      }
    }
    if ((rc = ensure(c, &c->spd, &c->spd_cap, (int)sl.size()))) return rc;
    hipLaunchKernelGGL(k_reset_acc, dim3((p1 - p0 + 63) / 64), dim3(64), 0, c->stream, c->ctl, c->pdt + p0, p1 - p0);
    HIPCHK(c, hipMemcpyAsync(c->spd, sl.data(), sizeof(SpeedLevel) * sl.size(), hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL(k_initial_speed, dim3(64, (unsigned)sl.size()), dim3(256), 0, c->stream, c->spd);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return timed(c, 6, [&]() -> int {
    hipLaunchKernelGGL(k_next_dt, dim3((p1 - p0 + 63) / 64), dim3(64), 0, c->stream, c->ctl, c->pdt + p0, p1 - p0,
                       c->cfg.cfl_desired, initial ? 1 : 0);
    HIPCHK(c, hipGetLastError());
    return MLSWE_OK;
  });
}

// Control blocks of problems [p0, p1) (contiguous, problem-major) in one copy.
int read_ctls(mlswe_ctx* c, int p0, int p1, std::vector<LevelCtl>& h) {
  const int a = c->probs[p0].ctl0, b = c->probs[p1 - 1].ctl0 + c->probs[p1 - 1].nlev;
  h.resize((size_t)(b - a));
  HIPCHK(c, hipMemcpyAsync(h.data(), c->ctl + a, sizeof(LevelCtl) * h.size(), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return MLSWE_OK;
}

int read_status(mlswe_ctx* c, int p0, int p1, int* status) {
  *status = 0;
  std::vector<LevelCtl> h;
  int rc = read_ctls(c, p0, p1, h);
  if (rc) return rc;
  for (const LevelCtl& x : h) *status |= x.status;
  return MLSWE_OK;
}

// ------------------------------------------------------------ patches
void host_mask(LevelH& L);
const std::vector<unsigned char>& host_cov(LevelH& L);

int upload_mask(mlswe_ctx* c, LevelH& L) {
  host_mask(L);
  HIPCHK(c, hipMemcpyAsync(L.mask, L.mask_h.data(), L.mask_h.size(), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return MLSWE_OK;
}

// Validates a patch list of level l of problem p (inside the level, aligned to
// the ratio, covered by the coarser level, no overlaps; level 0 covered).
int check_patches(mlswe_ctx* c, int p, int l, int n, const int32_t* bx, std::vector<Box>& nb_out) {
  ProblemH& P = c->probs[p];
  if (l < 0 || l >= P.nlev) return fail(c, MLSWE_EINVAL, "level %d out of range", l);
  if (n < 0 || (n > 0 && !bx)) return fail(c, MLSWE_EINVAL, "bad patch list");
  LevelH& L = P.L[l];
  std::vector<Box> nb(n);
  std::vector<unsigned char> cov((size_t)L.nx * L.ny, 0);
  for (int k = 0; k < n; ++k) {
    Box b{bx[4 * k], bx[4 * k + 1], bx[4 * k + 2], bx[4 * k + 3]};
    if (b.nx <= 0 || b.ny <= 0 || b.ilo < 0 || b.jlo < 0 || b.ilo + b.nx > L.nx || b.jlo + b.ny > L.ny)
      return fail(c, MLSWE_EINVAL, "patch %d outside level %d", k, l);
    if (l > 0) {
      const int r = P.ratio[l - 1];
      if (b.ilo % r || b.jlo % r || b.nx % r || b.ny % r)
        return fail(c, MLSWE_EINVAL, "patch %d not aligned to ratio %d", k, r);
      LevelH& C = P.L[l - 1];
      const std::vector<unsigned char>& cm = host_cov(C);
      for (int j = b.jlo / r; j < (b.jlo + b.ny) / r; ++j)
        for (int i = b.ilo / r; i < (b.ilo + b.nx) / r; ++i)
          if (!cm[idx(C, i, j)]) return fail(c, MLSWE_EINVAL, "patch %d not covered by level %d", k, l - 1);
    }
    for (int j = b.jlo; j < b.jlo + b.ny; ++j)
      for (int i = b.ilo; i < b.ilo + b.nx; ++i) {
        unsigned char& m = cov[(size_t)j * L.nx + i];
        if (m) return fail(c, MLSWE_EINVAL, "patches overlap on level %d", l);
        m = 1;
      }
    nb[k] = b;
  }
  if (l == 0) {
    for (unsigned char m : cov)
      if (!m) return fail(c, MLSWE_EINVAL, "level 0 patches must cover the domain");
  }
  nb_out = nb;
  return MLSWE_OK;
}

// Coverage bytes of a level: COV_IN on patch interiors, plus COV_COL0 / COV_ROW0
// on each patch's first column / row.
void host_mask(LevelH& L) {
  std::fill(L.mask_h.begin(), L.mask_h.end(), 0);
  for (const Box& b : L.boxes)
    for (int j = b.jlo; j < b.jlo + b.ny; ++j) {
      unsigned char* row = &L.mask_h[idx(L, b.ilo, j)];
      std::memset(row, j == b.jlo ? COV_IN | COV_ROW0 : COV_IN, b.nx);
      row[0] |= COV_COL0;
    }
  L.mask_h_ok = true;
}

// The host copy of a level's coverage, rebuilt from the boxes after a regrid
// left it stale (the regrid sets the device coverage directly).
const std::vector<unsigned char>& host_cov(LevelH& L) {
  if (!L.mask_h_ok) host_mask(L);
  return L.mask_h;
}

int set_patches_impl(mlswe_ctx* c, int p, int l, int n, const int32_t* bx) {
  std::vector<Box> nb;
  int rc0 = check_patches(c, p, l, n, bx, nb);
  if (rc0) return rc0;
  ProblemH& P = c->probs[p];
  LevelH& L = P.L[l];
  // keep the old coverage for the fill of new cells
  if (l > 0) {
    HIPCHK(c, hipMemcpyAsync(L.mask_old, L.mask, (size_t)L.plane, hipMemcpyDeviceToDevice, c->stream));
  }
  L.boxes = nb;
  int rc = upload_mask(c, L);
  if (rc) return rc;
  mark_dirty(c, l);
  if (l > 0 && n > 0) {
    std::vector<FillPatch> f;
    int maxn = 0;
    const LevelH& C = P.L[l - 1];
    for (const Box& b : L.boxes) {
      FillPatch x;
      std::memset(&x, 0, sizeof x);
      x.q = L.q[L.cur]; x.B = L.B; x.mask = L.mask; x.mask_old = L.mask_old;
      x.qco = C.q[C.cur]; x.qcn = C.q[C.cur]; x.Bc = C.B;
      x.cnt = c->cnt + P.cnt;
      x.pitch = L.pitch; x.plane = L.plane; x.cpitch = C.pitch; x.cplane = C.plane;
      x.nx = L.nx; x.ny = L.ny; x.ncx = C.nx; x.ncy = C.ny;
      x.ilo = b.ilo; x.jlo = b.jlo; x.bnx = b.nx; x.bny = b.ny;
      x.r = P.ratio[l - 1];
      x.P = P.P;
      f.push_back(x);
      maxn = std::max(maxn, b.nx * b.ny);
    }
    FillPatch* fd = nullptr;
    if ((rc = dalloc(c, (void**)&fd, sizeof(FillPatch) * f.size()))) return rc;
    HIPCHK(c, hipMemcpyAsync(fd, f.data(), sizeof(FillPatch) * f.size(), hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL(k_refine_new, dim3((maxn + 255) / 256, (unsigned)f.size()), dim3(256), 0, c->stream, fd);
    hipError_t e = hipGetLastError();
    hipError_t s = hipStreamSynchronize(c->stream);
    dfree(fd);
    c->bytes -= (long long)(sizeof(FillPatch) * f.size());
    if (e != hipSuccess || s != hipSuccess)
      return fail(c, MLSWE_EDEVICE, "refine launch: %s", hipGetErrorString(e != hipSuccess ? e : s));
  }
  return MLSWE_OK;
}

int flag_impl(mlswe_ctx* c, int p, int l, double tau, int nbuf, std::vector<unsigned char>& out) {
  ProblemH& P = c->probs[p];
  LevelH& L = P.L[l];
  int rc;
  if (!L.fraw) {
    if ((rc = dalloc(c, (void**)&L.fraw, (size_t)L.nx * L.ny))) return rc;
    if ((rc = dalloc(c, (void**)&L.fout, (size_t)L.nx * L.ny))) return rc;
  }
  FlagLevel F;
  F.q = L.q[L.cur]; F.B = L.B; F.mask = L.mask; F.raw = L.fraw; F.out = L.fout;
  F.pitch = L.pitch; F.plane = L.plane; F.nx = L.nx; F.ny = L.ny; F.nbuf = nbuf;
  F.dx = L.dx; F.dy = L.dy; F.tau = tau; F.hdry = P.P.hdry;
  if ((rc = ensure(c, &c->flv_d, &c->flv_cap, 1))) return rc;
  HIPCHK(c, hipMemcpyAsync(c->flv_d, &F, sizeof F, hipMemcpyHostToDevice, c->stream));
  hipLaunchKernelGGL(k_flag_raw, dim3((L.nx + 255) / 256, L.ny, 1), dim3(256), 0, c->stream, c->flv_d);
  hipLaunchKernelGGL(k_flag_dilate, dim3((L.nx + 255) / 256, L.ny, 1), dim3(256), 0, c->stream, c->flv_d);
  HIPCHK(c, hipGetLastError());
  out.resize((size_t)L.nx * L.ny);
  HIPCHK(c, hipMemcpyAsync(out.data(), L.fout, out.size(), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return MLSWE_OK;
}

int regrid_group(mlswe_ctx* c, int p0, int p1, const double* tau_all, int nbuf);

int regrid_impl(mlswe_ctx* c, int p, const double* tau, int nbuf) {
  std::vector<double> t((size_t)(p + 1) * MAXLEV, 0.0);
  for (int l = 0; l < MAXLEV; ++l) t[(size_t)p * MAXLEV + l] = tau[l];
  return regrid_group(c, p, p + 1, t.data(), nbuf);
}

// Regrid of problems [p0, p1) with one host wait per level: the flags of every
// problem are summarised per clustering tile on the device and come back in one
// pinned buffer, clustering runs on the host (its boxes are valid by
// construction: aligned, inside the covered region, disjoint), and the new
// coverage (old coverage kept for the fill), the masks and the refinement of
// newly covered cells are each one launch over all problems.
int regrid_group(mlswe_ctx* c, int p0, int p1, const double* tau_all, int nbuf) {
  int maxlev = 0;
  for (int p = p0; p < p1; ++p) maxlev = std::max(maxlev, c->probs[p].nlev);
  for (int l = 0; l + 1 < maxlev; ++l) {
    std::vector<int> who;
    std::vector<size_t> off;
    std::vector<FlagLevel> fl;
    std::vector<FlagTiles> ft;
    int mx = 0, my = 0, mt = 0;
    size_t total = 0;
    int rc;
    for (int p = p0; p < p1; ++p) {
      ProblemH& P = c->probs[p];
      if (l + 1 >= P.nlev) continue;
      LevelH& L = P.L[l];
      if (!L.fraw) {
        if ((rc = dalloc(c, (void**)&L.fraw, (size_t)L.nx * L.ny))) return rc;
        if ((rc = dalloc(c, (void**)&L.fout, (size_t)L.nx * L.ny))) return rc;
      }
      FlagLevel F;
      F.q = L.q[L.cur]; F.B = L.B; F.mask = L.mask; F.raw = L.fraw; F.out = L.fout;
      F.pitch = L.pitch; F.plane = L.plane; F.nx = L.nx; F.ny = L.ny; F.nbuf = nbuf;
      F.dx = L.dx; F.dy = L.dy; F.tau = tau_all[(size_t)p * MAXLEV + l]; F.hdry = P.P.hdry;
      fl.push_back(F);
      mx = std::max(mx, L.nx);
      my = std::max(my, L.ny);
      const int r = P.ratio[l];
      FlagTiles T;
      T.flags = L.fout; T.mask = L.mask; T.out = nullptr; T.pitch = L.pitch;
      T.nx = L.nx; T.ny = L.ny; T.r = r;
      T.tx = (L.nx * r + TILE - 1) / TILE; T.ty = (L.ny * r + TILE - 1) / TILE;
      ft.push_back(T);
      mt = std::max(mt, T.tx * T.ty);
      who.push_back(p);
      off.push_back(total);
      total += (size_t)T.tx * T.ty;
    }
    if (who.empty()) continue;
    if ((rc = ensure(c, &c->tbits_d, &c->tbits_cap, (int)total))) return rc;
    for (size_t k = 0; k < ft.size(); ++k) ft[k].out = c->tbits_d + off[k];
    if ((rc = ensure(c, &c->flv_d, &c->flv_cap, (int)fl.size()))) return rc;
    HIPCHK(c, hipMemcpyAsync(c->flv_d, fl.data(), sizeof(FlagLevel) * fl.size(), hipMemcpyHostToDevice, c->stream));
    for (size_t k0 = 0; k0 < fl.size(); k0 += 65535) {  // grid z is at most 65535
      const unsigned nz = (unsigned)std::min<size_t>(65535, fl.size() - k0);
      hipLaunchKernelGGL(k_flag_raw, dim3((mx + 255) / 256, my, nz), dim3(256), 0, c->stream, c->flv_d + k0);
    }
    for (size_t k0 = 0; k0 < fl.size(); k0 += 65535) {
      const unsigned nz = (unsigned)std::min<size_t>(65535, fl.size() - k0);
      hipLaunchKernelGGL(k_flag_dilate, dim3((mx + 255) / 256, my, nz), dim3(256), 0, c->stream, c->flv_d + k0);
    }
    if ((rc = ensure(c, &c->ftl_d, &c->ftl_cap, (int)ft.size()))) return rc;
    HIPCHK(c, hipMemcpyAsync(c->ftl_d, ft.data(), sizeof(FlagTiles) * ft.size(), hipMemcpyHostToDevice, c->stream));
    for (size_t k0 = 0; k0 < ft.size(); k0 += 65535) {
      const unsigned ny = (unsigned)std::min<size_t>(65535, ft.size() - k0);
      hipLaunchKernelGGL(k_flag_tiles, dim3((mt + 255) / 256, ny), dim3(256), 0, c->stream, c->ftl_d + k0);
    }
    HIPCHK(c, hipGetLastError());
    if (total > c->pin_cap) {
      HIPCHK(c, hipStreamSynchronize(c->stream));
      if (c->pin) (void)hipHostFree(c->pin);
      c->pin = nullptr;
      c->pin_cap = 0;
      HIPCHK(c, hipHostMalloc((void**)&c->pin, total, hipHostMallocDefault));
      c->pin_cap = total;
    }
    HIPCHK(c, hipMemcpyAsync(c->pin, c->tbits_d, total, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    // host: clusters, then the new layouts
    std::vector<std::vector<Box>> nbs(who.size());
    for (size_t k = 0; k < who.size(); ++k) {
      const LevelH& F = c->probs[who[k]].L[l + 1];
      nbs[k] = cluster_tiles(F.nx, F.ny, c->pin + off[k]);
    }
    std::vector<ByteSeg> keep, clear;
    std::vector<MaskBox> mb;
    std::vector<FillPatch> fills;
    int maxn = 0, maxbox = 0;
    for (size_t k = 0; k < who.size(); ++k) {
      ProblemH& P = c->probs[who[k]];
      LevelH& L = P.L[l + 1];
      const LevelH& C = P.L[l];
      keep.push_back(ByteSeg{L.mask, L.mask_old, L.plane, 0});
      clear.push_back(ByteSeg{nullptr, L.mask, L.plane, 0});
      L.boxes = nbs[k];
      L.mask_h_ok = false;
      mark_dirty(c, l + 1);
      for (const Box& b : L.boxes) {
        mb.push_back(MaskBox{L.mask, L.pitch, b.ilo, b.jlo, b.nx, b.ny});
        FillPatch x;
        std::memset(&x, 0, sizeof x);
        x.q = L.q[L.cur]; x.B = L.B; x.mask = L.mask; x.mask_old = L.mask_old;
        x.qco = C.q[C.cur]; x.qcn = C.q[C.cur]; x.Bc = C.B;
        x.cnt = c->cnt + P.cnt;
        x.pitch = L.pitch; x.plane = L.plane; x.cpitch = C.pitch; x.cplane = C.plane;
        x.nx = L.nx; x.ny = L.ny; x.ncx = C.nx; x.ncy = C.ny;
        x.ilo = b.ilo; x.jlo = b.jlo; x.bnx = b.nx; x.bny = b.ny;
        x.r = P.ratio[l];
        x.P = P.P;
        fills.push_back(x);
        maxn = std::max(maxn, b.nx * b.ny);
      }
      maxbox = std::max(maxbox, (int)L.plane);
    }
    // device: old coverage kept, masks cleared and set, new cells refined
    if ((rc = ensure(c, &c->bsegs_d, &c->bsegs_cap, (int)(2 * keep.size())))) return rc;
    std::vector<ByteSeg> both(keep);
    both.insert(both.end(), clear.begin(), clear.end());
    HIPCHK(c, hipMemcpyAsync(c->bsegs_d, both.data(), sizeof(ByteSeg) * both.size(), hipMemcpyHostToDevice, c->stream));
    const unsigned gb = (unsigned)std::min(64, (maxbox + 255) / 256);
    hipLaunchKernelGGL(k_byte_segs, dim3(gb, (unsigned)keep.size()), dim3(256), 0, c->stream, c->bsegs_d);
    hipLaunchKernelGGL(k_byte_segs, dim3(gb, (unsigned)clear.size()), dim3(256), 0, c->stream,
                       c->bsegs_d + keep.size());
    if (!mb.empty()) {
      if ((rc = ensure(c, &c->mboxes_d, &c->mboxes_cap, (int)mb.size()))) return rc;
      HIPCHK(c, hipMemcpyAsync(c->mboxes_d, mb.data(), sizeof(MaskBox) * mb.size(), hipMemcpyHostToDevice, c->stream));
      hipLaunchKernelGGL(k_mask_boxes, dim3((unsigned)std::min(64, (maxn + 255) / 256), (unsigned)mb.size()), dim3(256),
                         0, c->stream, c->mboxes_d);
      if ((rc = ensure(c, &c->rfills_d, &c->rfills_cap, (int)fills.size()))) return rc;
      HIPCHK(c, hipMemcpyAsync(c->rfills_d, fills.data(), sizeof(FillPatch) * fills.size(), hipMemcpyHostToDevice,
                               c->stream));
      hipLaunchKernelGGL(k_refine_new, dim3((maxn + 255) / 256, (unsigned)fills.size()), dim3(256), 0, c->stream,
                         c->rfills_d);
    }
    HIPCHK(c, hipGetLastError());
    // the descriptor lists above are host vectors read by the copies: wait
    // before they go out of scope (one wait per level of the regrid)
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return MLSWE_OK;
}

int copy_state(mlswe_ctx* c, LevelH& L, int buf, const double* src, int where, bool to_dev, double* dst) {
  if (where == MLSWE_DEVICE) {  // device to device: one kernel for the six fields
    hipLaunchKernelGGL(k_copy6, dim3(blocks((long long)L.nx * L.ny)), dim3(256), 0, c->stream, L.q[buf],
                       (long long)L.pitch, (long long)L.plane, to_dev ? const_cast<double*>(src) : dst, L.nx, L.ny,
                       to_dev ? 0 : 1);
    HIPCHK(c, hipGetLastError());
    return MLSWE_OK;
  }
  const hipMemcpyKind kind = to_dev ? hipMemcpyHostToDevice : hipMemcpyDeviceToHost;
  for (int f = 0; f < 6; ++f) {
    double* lv = L.q[buf] + f * L.plane + idx(L, 0, 0);
    const size_t hrow = (size_t)L.nx * sizeof(double);
    if (to_dev)
      HIPCHK(c, hipMemcpy2DAsync(lv, L.pitch * sizeof(double), src + (size_t)f * L.nx * L.ny, hrow, hrow, L.ny, kind,
                                 c->stream));
    else
      HIPCHK(c, hipMemcpy2DAsync(dst + (size_t)f * L.nx * L.ny, hrow, lv, L.pitch * sizeof(double), hrow, L.ny, kind,
                                 c->stream));
  }
  // device-to-device copies stay ordered on the stream; host memory is released
  // to the caller only once the copy is done
  if (where != MLSWE_DEVICE) HIPCHK(c, hipStreamSynchronize(c->stream));
  return MLSWE_OK;
}

}  // namespace

// ============================================================ C ABI
// ------------------------------------------------------------ allocation-free flagging
// mlswe_flag_noalloc stages a level's undilated flags in this file-scope device
// array instead of library allocations.  Each GPU holds its own copy at its own
// address until the process ends; in host code the name stands for no device
// address, so the copy's address is resolved per device (scratch_setup, from
// mlswe_create with the context's device current) and only that address is
// handed to kernels.
namespace {
constexpr long long NOALLOC_SCRATCH_BYTES = 16ll << 20;
static_assert(NOALLOC_SCRATCH_BYTES == (long long)MLSWE_NOALLOC_SCRATCH_BYTES, "header and library agree");
constexpr int NOALLOC_MAX_DEVICES = 64;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];
std::mutex scratch_mu;
unsigned char* scratch_dev[NOALLOC_MAX_DEVICES] = {};

int scratch_setup(mlswe_ctx* c) {
  if (c->device < 0 || c->device >= NOALLOC_MAX_DEVICES) return MLSWE_OK;  // the variant then refuses
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (scratch_dev[c->device]) return MLSWE_OK;
  void* a = nullptr;
  const hipError_t e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !a) return fail(c, MLSWE_EDEVICE, "scratch address: %s", hipGetErrorString(e));
  scratch_dev[c->device] = (unsigned char*)a;
  return MLSWE_OK;
}

unsigned char* scratch_of(int device) {
  if (device < 0 || device >= NOALLOC_MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(scratch_mu);
  return scratch_dev[device];
}
}  // namespace

extern "C" {

int mlswe_flag_noalloc(mlswe_ctx* c, int p, int level, double tau, int nbuf, uint8_t* flags_dev) {
  if (!c) return MLSWE_EINVAL;
  if (!valid_prob(c, p) || level < 0 || level >= c->probs[p].nlev || !flags_dev || nbuf < 0)
    return fail(c, MLSWE_EINVAL, "bad args");
  const ProblemH& P = c->probs[p];
  const LevelH& L = P.L[level];
  const long long cells = (long long)L.nx * L.ny;
  if (cells > NOALLOC_SCRATCH_BYTES)
    return fail(c, MLSWE_EINVAL, "level %d holds %lld cells, above the %lld bytes of the allocation-free scratch",
                level, cells, NOALLOC_SCRATCH_BYTES);
  unsigned char* raw = scratch_of(c->device);
  if (!raw) return fail(c, MLSWE_EDEVICE, "no allocation-free scratch on device %d", c->device);
  FlagLevel F;
  F.q = L.q[L.cur]; F.B = L.B; F.mask = L.mask; F.raw = raw; F.out = flags_dev;
  F.pitch = L.pitch; F.plane = L.plane; F.nx = L.nx; F.ny = L.ny; F.nbuf = nbuf;
  F.dx = L.dx; F.dy = L.dy; F.tau = tau; F.hdry = P.P.hdry;
  // every raw byte of the level is written before the dilation reads it, so
  // what an earlier call left in the scratch is never seen
  const unsigned nb = (unsigned)((cells + 255) / 256);
  hipLaunchKernelGGL(k_flag_raw_v, dim3(nb), dim3(256), 0, c->stream, F);
  hipLaunchKernelGGL(k_flag_dilate_v, dim3(nb), dim3(256), 0, c->stream, F);
  HIPCHK(c, hipGetLastError());
  return MLSWE_OK;
}

int mlswe_version(void) { return MLSWE_VERSION; }

const char* mlswe_last_error(const mlswe_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int mlswe_create(const mlswe_config* cfg, void* hip_stream, mlswe_ctx** out) {
  if (!out) return MLSWE_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return MLSWE_EDEVICE;
  mlswe_ctx* c = new (std::nothrow) mlswe_ctx;
  if (!c) return MLSWE_ENOMEM;
  mlswe_config d;
  std::memset(&d, 0, sizeof d);
  d.g = 9.81; d.hdry = 1e-3; d.kmin = 1e-6; d.cfl_desired = 0.9; d.cfl_max = 1.0;
  if (cfg) d = *cfg;
  if (d.max_retries == 0) d.max_retries = 8;
  if (!(d.g > 0) || !(d.hdry > 0) || !(d.kmin > 0) || !(d.cfl_desired > 0) || !(d.cfl_max >= d.cfl_desired) ||
      d.y_rows < 0 || d.x_rows < 0 || (d.reflux != 0 && d.reflux != 1) ||
      (d.dynamic_rt != 0 && d.dynamic_rt != 1)) {
    delete c;
    return MLSWE_EINVAL;
  }
  c->cfg = d;
  c->stream = (hipStream_t)hip_stream;
  if (hipGetDevice(&c->device) != hipSuccess) { delete c; return MLSWE_EDEVICE; }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, c->device) == hipSuccess && prop.multiProcessorCount > 0)
    c->ncu = prop.multiProcessorCount;
  std::memset(&c->tune, 0, sizeof c->tune);
  c->tune.x_rows = d.x_rows;  // 0: chosen per level when the tiles are built
  c->tune.y_rows = d.y_rows;
  c->tune.grid_x = 1;
  c->tune.grid_y = 1;
  if (dalloc(c, (void**)&c->tickets, 2 * sizeof(unsigned)) != MLSWE_OK) { delete c; return MLSWE_ENOMEM; }
  if (scratch_setup(c) != MLSWE_OK) {
    dfree(c->tickets);
    delete c;
    return MLSWE_EDEVICE;
  }
  *out = c;
  return MLSWE_OK;
}

int mlswe_destroy(mlswe_ctx* c) {
  if (!c) return MLSWE_EINVAL;
  (void)hipStreamSynchronize(c->stream);
  for (ProblemH& P : c->probs) {
    dfree(P.adj.lam1); dfree(P.adj.lamS); dfree(P.adj.lamG); dfree(P.adj.cL); dfree(P.adj.cR);
    dfree(P.adj.Bbx); dfree(P.adj.Bby); dfree(P.adj.status);
    if (P.adj.status_host) (void)hipHostFree(P.adj.status_host);
    if (P.adj.status_ev) (void)hipEventDestroy(P.adj.status_ev);
  }
  for (ProblemH& P : c->probs)
    for (int l = 0; l < P.nlev; ++l) {
      LevelH& L = P.L[l];
      dfree(L.q[0]); dfree(L.q[1]); dfree(L.qs); dfree(L.B); dfree(L.mask); dfree(L.mask_old);
      dfree(L.fraw); dfree(L.fout); dfree(L.bk);
    }
  for (LevelLaunch& LL : c->launch) {
    dfree(LL.pd[0]); dfree(LL.pd[1]); dfree(LL.xt); dfree(LL.yt); dfree(LL.li); dfree(LL.parts);
    for (int k = 0; k < 4; ++k) { dfree(LL.fp[k]); dfree(LL.cp[k]); }
    dfree(LL.rfx); dfree(LL.rfx_reg);
  }
  dfree(c->ctl); dfree(c->cnt); dfree(c->pdt); dfree(c->spd); dfree(c->dt_stage);
  dfree(c->tickets); dfree(c->ctl_bk); dfree(c->cnt_bk); dfree(c->dt0_d); dfree(c->boxes_d);
  dfree(c->bsegs_d); dfree(c->mboxes_d); dfree(c->rfills_d); dfree(c->flv_d);
  dfree(c->ftl_d); dfree(c->tbits_d); dfree(c->lrep_d);
  if (c->pin) (void)hipHostFree(c->pin);
  if (c->ctl_pin) (void)hipHostFree(c->ctl_pin);
  for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.exec);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  for (auto& u : c->ev_used) { (void)hipEventDestroy(u.second.first); (void)hipEventDestroy(u.second.second); }
  delete c;
  return MLSWE_OK;
}

int mlswe_problem_define(mlswe_ctx* c, int* p_out, double r, int nx0, int ny0, double dx0, double dy0, int nlevels,
                         const int* ratios) {
  if (!c || !p_out) return MLSWE_EINVAL;
  if (!(r > 0.0 && r < 1.0) || nx0 < 2 || ny0 < 2 || !(dx0 > 0) || !(dy0 > 0) || nlevels < 1 || nlevels > MAXLEV)
    return fail(c, MLSWE_EINVAL, "bad problem geometry");
  if (nlevels > 1 && !ratios) return fail(c, MLSWE_EINVAL, "ratios missing");
  for (int l = 0; l + 1 < nlevels; ++l)
    if (ratios[l] < 2 || ratios[l] > 16 || TILE % ratios[l])
      return fail(c, MLSWE_EINVAL, "ratio %d must divide %d", ratios[l], TILE);
  ProblemH P;
  P.P.g = c->cfg.g; P.P.r = r; P.P.hdry = c->cfg.hdry; P.P.kmin = c->cfg.kmin;
  P.P.gp = (1.0 - r) * c->cfg.g;
  P.P.inv_gp = 1.0 / ((1.0 - r) * c->cfg.g);
  P.nlev = nlevels;
  long long nx = nx0, ny = ny0;
  double dx = dx0, dy = dy0;
  for (int l = 0; l < nlevels; ++l) {
    if (l > 0) {
      P.ratio[l - 1] = ratios[l - 1];
      P.rt[l - 1] = ratios[l - 1];
      nx *= ratios[l - 1]; ny *= ratios[l - 1];
      dx = dx / ratios[l - 1]; dy = dy / ratios[l - 1];
    }
    if (nx > (1 << 20) || ny > (1 << 20)) return fail(c, MLSWE_EINVAL, "level %d too large", l);
    LevelH& L = P.L[l];
    L.nx = (int)nx; L.ny = (int)ny; L.dx = dx; L.dy = dy;
    L.pitch = ((XOFF + nx + 2) + 15) / 16 * 16;
    L.plane = L.pitch * (ny + 4);
    const size_t sb = sizeof(double) * 6 * (size_t)L.plane;
    int rc;
    if ((rc = dalloc(c, (void**)&L.q[0], sb)) || (rc = dalloc(c, (void**)&L.q[1], sb)) ||
        (rc = dalloc(c, (void**)&L.qs, sb)) || (rc = dalloc(c, (void**)&L.B, sizeof(double) * (size_t)L.plane)) ||
        (rc = dalloc(c, (void**)&L.mask, (size_t)L.plane)) || (rc = dalloc(c, (void**)&L.mask_old, (size_t)L.plane))) {
      for (int k = 0; k <= l; ++k) {
        dfree(P.L[k].q[0]); dfree(P.L[k].q[1]); dfree(P.L[k].qs); dfree(P.L[k].B); dfree(P.L[k].mask);
        dfree(P.L[k].mask_old);
      }
      return rc;
    }
    HIPCHK(c, hipMemsetAsync(L.q[0], 0, sb, c->stream));
    HIPCHK(c, hipMemsetAsync(L.q[1], 0, sb, c->stream));
    HIPCHK(c, hipMemsetAsync(L.qs, 0, sb, c->stream));
    HIPCHK(c, hipMemsetAsync(L.B, 0, sizeof(double) * (size_t)L.plane, c->stream));
    HIPCHK(c, hipMemsetAsync(L.mask, 0, (size_t)L.plane, c->stream));
    HIPCHK(c, hipMemsetAsync(L.mask_old, 0, (size_t)L.plane, c->stream));
    L.mask_h.assign((size_t)L.plane, 0);
  }
  const int pidx = (int)c->probs.size();
  // device control blocks: grow and copy
  int nctl = 0;
  for (const ProblemH& Q : c->probs) nctl += Q.nlev;
  P.ctl0 = nctl;
  P.cnt = pidx;
  if (nctl + nlevels > c->ctl_cap || pidx + 1 > c->cnt_cap) {
    int ncap = std::max(2 * (nctl + nlevels), 64);
    int ccap = std::max(2 * (pidx + 1), 64);
    LevelCtl* nc = nullptr;
    Counters* ncn = nullptr;
    int rc;
    if ((rc = dalloc(c, (void**)&nc, sizeof(LevelCtl) * ncap))) return rc;
    if ((rc = dalloc(c, (void**)&ncn, sizeof(Counters) * ccap))) return rc;
    HIPCHK(c, hipMemsetAsync(nc, 0, sizeof(LevelCtl) * ncap, c->stream));
    HIPCHK(c, hipMemsetAsync(ncn, 0, sizeof(Counters) * ccap, c->stream));
    if (c->ctl) HIPCHK(c, hipMemcpyAsync(nc, c->ctl, sizeof(LevelCtl) * nctl, hipMemcpyDeviceToDevice, c->stream));
    if (c->cnt) HIPCHK(c, hipMemcpyAsync(ncn, c->cnt, sizeof(Counters) * pidx, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    dfree(c->ctl); dfree(c->cnt);
    c->ctl = nc; c->cnt = ncn; c->ctl_cap = ncap; c->cnt_cap = ccap;
    for (int l = 0; l < MAXLEV; ++l) c->launch[l].dirty = true;  // descriptors hold ctl pointers
  }
  P.L[0].boxes.push_back(Box{0, 0, nx0, ny0});
  c->probs.push_back(P);
  int rc = upload_mask(c, c->probs.back().L[0]);
  if (rc) return rc;
  for (int l = 0; l < MAXLEV; ++l) c->launch[l].dirty = true;
  c->pdt_dirty = true;
  c->generation++;
  *p_out = pidx;
  return MLSWE_OK;
}

int mlswe_set_bathymetry(mlswe_ctx* c, int p, const double* Bf, int where) {
  if (!c) return MLSWE_EINVAL;
  if (!valid_prob(c, p) || !Bf) return fail(c, MLSWE_EINVAL, "bad problem or pointer");
  ProblemH& P = c->probs[p];
  const LevelH& F = P.L[P.nlev - 1];
  std::vector<double> fine((size_t)F.nx * F.ny);
  if (where == MLSWE_DEVICE) {
    HIPCHK(c, hipMemcpy(fine.data(), Bf, sizeof(double) * fine.size(), hipMemcpyDeviceToHost));
  } else {
    std::memcpy(fine.data(), Bf, sizeof(double) * fine.size());
  }
  std::vector<double> prev;
  for (int l = P.nlev - 1; l >= 0; --l) {
    LevelH& L = P.L[l];
    std::vector<double> a((size_t)L.plane, 0.0);
    if (l == P.nlev - 1) {
      for (int j = 0; j < L.ny; ++j)
        for (int i = 0; i < L.nx; ++i) a[idx(L, i, j)] = fine[(size_t)j * L.nx + i];
    } else {
      const LevelH& Fl = P.L[l + 1];
      const int r = P.ratio[l];
      const double inv = 1.0 / double(r * r);
      for (int J = 0; J < L.ny; ++J)
        for (int I = 0; I < L.nx; ++I) {
          double s = 0.0;
          for (int b = 0; b < r; ++b)
            for (int a2 = 0; a2 < r; ++a2) s = s + prev[idx(Fl, r * I + a2, r * J + b)];
          a[idx(L, I, J)] = s * inv;
        }
    }
    mirror_frame_host(L, a);
    HIPCHK(c, hipMemcpyAsync(L.B, a.data(), sizeof(double) * a.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    prev.swap(a);
  }
  P.bathy = true;
  return MLSWE_OK;
}

int mlswe_set_patches(mlswe_ctx* c, int p, int level, int n, const int32_t* boxes) {
  if (!c) return MLSWE_EINVAL;
  if (!valid_prob(c, p)) return fail(c, MLSWE_EINVAL, "bad problem %d", p);
  if (!c->probs[p].bathy) return fail(c, MLSWE_ESTATE, "set the bathymetry first");
  return set_patches_impl(c, p, level, n, boxes);
}

int mlswe_refine(mlswe_ctx* c, int p, int fine_level, int n, const int32_t* boxes) {
  if (!c) return MLSWE_EINVAL;
  if (fine_level < 1) return fail(c, MLSWE_EINVAL, "refine needs a level > 0");
  return mlswe_set_patches(c, p, fine_level, n, boxes);
}

int mlswe_get_patches(mlswe_ctx* c, int p, int level, int cap, int32_t* boxes, int* n_out) {
  if (!c) return MLSWE_EINVAL;
  if (!valid_prob(c, p) || level < 0 || level >= c->probs[p].nlev || !n_out) return fail(c, MLSWE_EINVAL, "bad args");
  const std::vector<Box>& B = c->probs[p].L[level].boxes;
  if ((int)B.size() > cap || (!boxes && !B.empty())) return fail(c, MLSWE_EINVAL, "capacity %d < %zu", cap, B.size());
  for (size_t k = 0; k < B.size(); ++k) {
    boxes[4 * k] = B[k].ilo; boxes[4 * k + 1] = B[k].jlo; boxes[4 * k + 2] = B[k].nx; boxes[4 * k + 3] = B[k].ny;
  }
  *n_out = (int)B.size();
  return MLSWE_OK;
}

int mlswe_set_state(mlswe_ctx* c, int p, int level, const double* q, int where) {
  if (!c) return MLSWE_EINVAL;
  if (!valid_prob(c, p) || !q || level < 0 || level >= c->probs[p].nlev) return fail(c, MLSWE_EINVAL, "bad args");
  ProblemH& P = c->probs[p];
  LevelH& L = P.L[level];
  int rc = copy_state(c, L, L.cur, q, where, true, nullptr);
  if (rc) return rc;
  if (level > 0) {
    const long long pu = (long long)L.nx * L.ny;
    hipLaunchKernelGGL(k_zero_uncovered, dim3((unsigned)((pu + 255) / 256)), dim3(256), 0, c->stream, L.q[L.cur],
                       L.mask, L.pitch, L.plane, L.nx, L.ny);
    HIPCHK(c, hipGetLastError());
  }
  P.state = true;
  return MLSWE_OK;
}

int mlswe_get_step_state(mlswe_ctx* c, int p, double* out) {
  if (!c) return MLSWE_EINVAL;
  if (!valid_prob(c, p) || !out) return fail(c, MLSWE_EINVAL, "bad args");
  const ProblemH& P = c->probs[p];
  std::vector<LevelCtl> h((size_t)P.nlev);
  HIPCHK(c, hipMemcpyAsync(h.data(), c->ctl + P.ctl0, sizeof(LevelCtl) * h.size(), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  out[0] = h[0].t;
  out[1] = P.have_dt ? 1.0 : 0.0;
  for (int l = 0; l < P.nlev; ++l) {
    out[2 + 2 * l] = __builtin_bit_cast(double, (long long)h[l].acc_smax[0]);
    out[3 + 2 * l] = __builtin_bit_cast(double, (long long)h[l].acc_smax[1]);
  }
  return MLSWE_OK;
}

int mlswe_get_time_ratios(mlswe_ctx* c, int p, int32_t* out) {
  if (!c) return MLSWE_EINVAL;
  if (!valid_prob(c, p) || !out) return fail(c, MLSWE_EINVAL, "bad args");
  for (int l = 0; l + 1 < c->probs[p].nlev; ++l) out[l] = c->probs[p].rt[l];
  return MLSWE_OK;
}

int mlswe_set_step_state(mlswe_ctx* c, int p, const double* in) {
  if (!c) return MLSWE_EINVAL;
  if (!valid_prob(c, p) || !in) return fail(c, MLSWE_EINVAL, "bad args");
  ProblemH& P = c->probs[p];
  if (!(in[0] == in[0]) || (in[1] != 0.0 && in[1] != 1.0)) return fail(c, MLSWE_EINVAL, "bad time or flag");
  for (int l = 0; l < 2 * P.nlev; ++l)
    if (!(in[2 + l] >= 0.0) || std::signbit(in[2 + l]) || in[2 + l] == std::numeric_limits<double>::infinity())
      return fail(c, MLSWE_EINVAL, "speed %g of level %d is not finite and non-negative", in[2 + l], l / 2);
  std::vector<LevelCtl> h((size_t)P.nlev);
  HIPCHK(c, hipMemcpyAsync(h.data(), c->ctl + P.ctl0, sizeof(LevelCtl) * h.size(), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  h[0].t = in[0];
  for (int l = 0; l < P.nlev; ++l) {
    h[l].acc_smax[0] = (unsigned long long)__builtin_bit_cast(long long, in[2 + 2 * l]);
    h[l].acc_smax[1] = (unsigned long long)__builtin_bit_cast(long long, in[3 + 2 * l]);
  }
  HIPCHK(c, hipMemcpyAsync(c->ctl + P.ctl0, h.data(), sizeof(LevelCtl) * h.size(), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  P.have_dt = in[1] != 0.0;
  P.acc_known = false;
  return MLSWE_OK;
}

int mlswe_get_state(mlswe_ctx* c, int p, int level, double* q, int where) {
  if (!c) return MLSWE_EINVAL;
  if (!valid_prob(c, p) || !q || level < 0 || level >= c->probs[p].nlev) return fail(c, MLSWE_EINVAL, "bad args");
  LevelH& L = c->probs[p].L[level];
  int rc = copy_state(c, L, L.cur, nullptr, where, false, q);
  if (rc) return rc;
  if (where == MLSWE_DEVICE) {
    const long long pu = (long long)L.nx * L.ny;
    hipLaunchKernelGGL(k_nan_uncovered, dim3((unsigned)((pu + 255) / 256)), dim3(256), 0, c->stream, q, L.mask,
                       L.pitch, L.nx, L.ny);
    HIPCHK(c, hipGetLastError());
    return MLSWE_OK;
  }
  const double nan = std::numeric_limits<double>::quiet_NaN();
  const std::vector<unsigned char>& cov = host_cov(L);
  for (int j = 0; j < L.ny; ++j)
    for (int i = 0; i < L.nx; ++i)
      if (!cov[idx(L, i, j)])
        for (int f = 0; f < 6; ++f) q[((size_t)f * L.ny + j) * L.nx + i] = nan;
  return MLSWE_OK;
}

int mlswe_step_level(mlswe_ctx* c, int level, const double* dt, double theta, double* smax_out) {
  if (!c) return MLSWE_EINVAL;
  if (c->probs.empty()) return fail(c, MLSWE_ESTATE, "no problem defined");
  for (ProblemH& P : c->probs) P.acc_known = false;  // the substep adds to the device speeds
  const int np = (int)c->probs.size();
  for (int p = 0; p < np; ++p) {
    const ProblemH& P = c->probs[p];
    if (!P.bathy || !P.state) return fail(c, MLSWE_ESTATE, "problem %d lacks bathymetry or state", p);
    if (level < 0 || level >= P.nlev) return fail(c, MLSWE_EINVAL, "level %d missing in problem %d", level, p);
  }
  int rc;
  if (dt) {
    for (int p = 0; p < np; ++p) {
      if (!(dt[p] > 0.0) || !std::isfinite(dt[p])) return fail(c, MLSWE_EINVAL, "dt[%d] must be positive", p);
      HIPCHK(c, hipMemcpyAsync(&c->ctl[c->probs[p].ctl0 + level].dt, &dt[p], sizeof(double), hipMemcpyHostToDevice,
                               c->stream));
    }
  }
  if ((rc = substep(c, level, 0, np, theta, true))) return rc;
  if (smax_out) {
    HIPCHK(c, hipStreamSynchronize(c->stream));
    int status = 0;
    for (int p = 0; p < np; ++p) {
      LevelCtl h;
      HIPCHK(c, hipMemcpy(&h, c->ctl + c->probs[p].ctl0 + level, sizeof h, hipMemcpyDeviceToHost));
      smax_out[2 * p] = __builtin_bit_cast(double, (long long)h.last_smax[0]);
      smax_out[2 * p + 1] = __builtin_bit_cast(double, (long long)h.last_smax[1]);
      status |= h.status;
    }
    if (status & STATUS_NAN) return fail(c, MLSWE_ENAN, "non-finite state");
    if (status & STATUS_CFL) return fail(c, MLSWE_ECFL, "Courant number above %g", c->cfg.cfl_max);
  }
  return MLSWE_OK;
}

int mlswe_coarsen(mlswe_ctx* c, int p, int fine_level) {
  if (!c) return MLSWE_EINVAL;
  if (!valid_prob(c, p) || fine_level < 1 || fine_level >= c->probs[p].nlev) return fail(c, MLSWE_EINVAL, "bad level");
  int rc = coarsen_level(c, fine_level, p, p + 1);
  if (rc) return rc;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return MLSWE_OK;
}

int mlswe_flag(mlswe_ctx* c, int p, int level, double tau, int nbuf, uint8_t* flags_out) {
  if (!c) return MLSWE_EINVAL;
  if (!valid_prob(c, p) || level < 0 || level >= c->probs[p].nlev || !flags_out || nbuf < 0)
    return fail(c, MLSWE_EINVAL, "bad args");
  std::vector<unsigned char> f;
  int rc = flag_impl(c, p, level, tau, nbuf, f);
  if (rc) return rc;
  std::memcpy(flags_out, f.data(), f.size());
  return MLSWE_OK;
}

int mlswe_regrid(mlswe_ctx* c, int p, const double* tau, int nbuf) {
  if (!c) return MLSWE_EINVAL;
  if (!valid_prob(c, p) || !tau || nbuf < 0) return fail(c, MLSWE_EINVAL, "bad args");
  return regrid_impl(c, p, tau, nbuf);
}

int mlswe_refine_layers(mlswe_ctx* c, int M, int r, const double* qc, const double* Bc, int nxc, int nyc, int fi0,
                        int fj0, int fnx, int fny, const double* Bf, double* qf, int64_t* repairs_out) {
  if (!c) return MLSWE_EINVAL;
  if (M < 1 || M > LAYERS_MAX) return fail(c, MLSWE_EINVAL, "layers %d outside 1..%d", M, LAYERS_MAX);
  if (r < 1 || r > 8) return fail(c, MLSWE_EINVAL, "ratio %d outside 1..8", r);
  if (nxc < 1 || nyc < 1 || fi0 < 0 || fj0 < 0 || fnx < 0 || fny < 0 ||
      (long long)fi0 + fnx > (long long)r * nxc || (long long)fj0 + fny > (long long)r * nyc)
    return fail(c, MLSWE_EINVAL, "fine box (%d, %d, %d, %d) outside the %d x %d coarse grid at ratio %d", fi0, fj0,
                fnx, fny, nxc, nyc, r);
  if ((long long)nxc * nyc * 3 * M > (1ll << 40) || (long long)fnx * fny * 3 * M > (1ll << 40))
    return fail(c, MLSWE_EINVAL, "grid too large");
  const long long nI = fnx ? (fi0 + fnx - 1) / r - fi0 / r + 1 : 0;
  const long long nJ = fny ? (fj0 + fny - 1) / r - fj0 / r + 1 : 0;
  if ((nJ + 3) / 4 > 65535) return fail(c, MLSWE_EINVAL, "more than 262140 coarse rows");
  if (repairs_out) *repairs_out = 0;
  if (nI == 0 || nJ == 0) return MLSWE_OK;
  if (!qc || !Bc || !Bf || !qf) return fail(c, MLSWE_EINVAL, "null array");
  LayersRefine A;
  A.qc = qc; A.Bc = Bc; A.Bf = Bf; A.qf = qf;
  A.repairs = nullptr;
  A.cplane = (long long)nxc * nyc;
  A.fplane = (long long)fnx * fny;
  A.nxc = nxc; A.nyc = nyc; A.r = r;
  A.fi0 = fi0; A.fj0 = fj0; A.fnx = fnx; A.fny = fny;
  A.I0 = fi0 / r; A.J0 = fj0 / r; A.nI = (int)nI; A.nJ = (int)nJ;
  A.hdry = c->cfg.hdry;
  if (repairs_out) {
    int rc = ensure(c, &c->lrep_d, &c->lrep_cap, 1);
    if (rc) return rc;
    HIPCHK(c, hipMemsetAsync(c->lrep_d, 0, sizeof(unsigned long long), c->stream));
    A.repairs = c->lrep_d;
  }
  HIPCHK(c, launch_refine_layers(M, A, c->stream));
  if (repairs_out) {
    unsigned long long n = 0;
    HIPCHK(c, hipMemcpyAsync(&n, c->lrep_d, sizeof n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *repairs_out = (int64_t)n;
  }
  return MLSWE_OK;
}

int mlswe_coarsen_layers(mlswe_ctx* c, int M, int r, const double* qf, int ci0, int cj0, int cnx, int cny, double* qc,
                         int nxc, int nyc) {
  if (!c) return MLSWE_EINVAL;
  if (M < 1 || M > LAYERS_MAX) return fail(c, MLSWE_EINVAL, "layers %d outside 1..%d", M, LAYERS_MAX);
  if (r < 1 || r > 8) return fail(c, MLSWE_EINVAL, "ratio %d outside 1..8", r);
  if (nxc < 1 || nyc < 1 || ci0 < 0 || cj0 < 0 || cnx < 0 || cny < 0 || (long long)ci0 + cnx > nxc ||
      (long long)cj0 + cny > nyc)
    return fail(c, MLSWE_EINVAL, "coarse box (%d, %d, %d, %d) outside the %d x %d grid", ci0, cj0, cnx, cny, nxc, nyc);
  if ((long long)nxc * nyc * 3 * M > (1ll << 40) || (long long)cnx * cny * r * r * 3 * M > (1ll << 40))
    return fail(c, MLSWE_EINVAL, "grid too large");
  if ((cny + 3) / 4 > 65535) return fail(c, MLSWE_EINVAL, "more than 262140 coarse rows");
  if (cnx == 0 || cny == 0) return MLSWE_OK;
  if (!qf || !qc) return fail(c, MLSWE_EINVAL, "null array");
  LayersCoarsen A;
  A.qf = qf; A.qc = qc;
  A.cplane = (long long)nxc * nyc;
  A.fplane = (long long)cnx * cny * r * r;
  A.nxc = nxc; A.r = r; A.ci0 = ci0; A.cj0 = cj0; A.cnx = cnx; A.cny = cny;
  A.hdry = c->cfg.hdry;
  HIPCHK(c, launch_coarsen_layers(M, A, c->stream));
  return MLSWE_OK;
}

}  // extern "C"

namespace {

// Time ratios of the coming coarse step from the largest speeds of the last one
// (reading of Sec. 2, text after Eq. 2): per problem, with a_l = cfl * min(dx /
// sx, dy / sy) (infinite without speeds), A_l = min(a_l, r_l A_{l+1}) from the
// finest level up and dt0 the coming coarse step (the dt rule's value), level
// l takes ceil(dt_{l-1} / A_l) substeps, clipped to [1, r]; a problem without
// speeds, or with a populated level that has none (new since the last step),
// takes the space ratios.  Each level then takes the largest number any
// problem takes (clipped to each problem's ratio).
int choose_time_ratios(mlswe_ctx* c) {
  const int np = (int)c->probs.size();
  std::vector<LevelCtl> h;
  int rc;
  bool cached = true;  // speeds already read back after the last step's Courant check
  for (int p = 0; p < np; ++p) cached = cached && c->probs[p].acc_known;
  if (!cached && (rc = read_ctls(c, 0, np, h))) return rc;
  const int base = c->probs[0].ctl0;
  const double inf = std::numeric_limits<double>::infinity();
  int RT[MAXLEV] = {0};
  for (int p = 0; p < np; ++p) {
    const ProblemH& P = c->probs[p];
    int k[MAXLEV];
    for (int l = 0; l + 1 < P.nlev; ++l) k[l] = P.ratio[l];
    // a level with patches but no speeds of the last coarse step (just
    // populated by a regrid) has no Courant bound of its own: the problem then
    // keeps its space ratios, as on its first step
    bool fresh = false;
    for (int l = 1; l < P.nlev && P.have_dt; ++l) {
      const unsigned long long bx = cached ? P.last_acc[l][0] : h[(size_t)(P.ctl0 - base + l)].acc_smax[0];
      const unsigned long long by = cached ? P.last_acc[l][1] : h[(size_t)(P.ctl0 - base + l)].acc_smax[1];
      const double sx = __builtin_bit_cast(double, (long long)bx);
      const double sy = __builtin_bit_cast(double, (long long)by);
      if (!P.L[l].boxes.empty() && !(sx > 0.0) && !(sy > 0.0)) fresh = true;
    }
    if (P.have_dt && !fresh) {
      double a[MAXLEV], A[MAXLEV];
      double best = inf, fac = 1.0;
      for (int l = 0; l < P.nlev; ++l) {
        const unsigned long long bx = cached ? P.last_acc[l][0] : h[(size_t)(P.ctl0 - base + l)].acc_smax[0];
        const unsigned long long by = cached ? P.last_acc[l][1] : h[(size_t)(P.ctl0 - base + l)].acc_smax[1];
        if (l > 0) fac *= (double)P.ratio[l - 1];
        const double sx = __builtin_bit_cast(double, (long long)bx);
        const double sy = __builtin_bit_cast(double, (long long)by);
        const double ax = sx > 0.0 ? P.L[l].dx / sx : inf;
        const double ay = sy > 0.0 ? P.L[l].dy / sy : inf;
        const double m = ax < ay ? ax : ay;
        a[l] = m < inf ? c->cfg.cfl_desired * m : inf;
        if (m < inf) { const double v = fac * (c->cfg.cfl_desired * m); best = v < best ? v : best; }
      }
      for (int l = P.nlev - 1; l >= 0; --l)
        A[l] = l + 1 < P.nlev ? std::min(a[l], (double)P.ratio[l] * A[l + 1]) : a[l];
      double dtp = best;
      for (int l = 1; l < P.nlev; ++l) {
        const double q = dtp / A[l];
        int kk = P.ratio[l - 1];
        if (q < (double)kk) {
          const double cq = std::ceil(q);
          kk = cq < 1.0 ? 1 : (int)cq;
        }
        k[l - 1] = kk;
        dtp = dtp / (double)kk;
      }
    }
    for (int l = 0; l + 1 < P.nlev; ++l) RT[l] = std::max(RT[l], k[l]);
  }
  for (int p = 0; p < np; ++p) {
    ProblemH& P = c->probs[p];
    P.acc_known = false;  // consumed: the coming step replaces the speeds
    for (int l = 0; l + 1 < P.nlev; ++l) {
      const int v = std::min(RT[l], P.ratio[l]);
      if (v != P.rt[l]) { P.rt[l] = v; c->pdt_dirty = true; }
    }
  }
  return MLSWE_OK;
}

int build_all(mlswe_ctx* c) {
  int nl = 0;
  for (const ProblemH& P : c->probs) nl = std::max(nl, P.nlev);
  int rc;
  for (int l = 0; l < nl; ++l)
    if ((rc = build_launch(c, l))) return rc;
  return build_pdt(c);
}

// One coarse step of problems [p0, p1): dt rule, then the subcycled recursion.
int coarse_step(mlswe_ctx* c, int p0, int p1, bool batched) {
  int rc;
  // the dt comes from the state for every problem of the range if one of them
  // has no speeds of a last step (a fresh or re-initialised problem)
  bool initial = false;
  for (int p = p0; p < p1; ++p) initial = initial || !c->probs[p].have_dt;
  if ((rc = next_dt(c, p0, p1, initial))) return rc;
  for (int p = p0; p < p1; ++p) c->probs[p].have_dt = true;
  return adv(c, 0, p0, p1, 0.0, batched);
}

// A coarse step of all problems replayed from a captured hipGraph.  The graph of
// a step depends only on the launch data and on the buffer parity of every
// level at its start; it is captured on first use (the capture also advances the
// host-side bookkeeping, and the graph is then launched once) and replayed while
// the launch data is unchanged.
int graph_step(mlswe_ctx* c, int p0, int p1) {
  int rc;
  const ProblemH& P0 = c->probs[p0];
  // buffer parities, then the time ratios (the substep structure)
  unsigned long long key = 0;
  for (int l = 0; l < P0.nlev; ++l) key |= (unsigned long long)P0.L[l].cur << l;
  for (int l = 0; l + 1 < P0.nlev; ++l) key |= (unsigned long long)(P0.rt[l] & 31) << (8 + 5 * l);
  for (auto it = c->graphs.begin(); it != c->graphs.end();) {
    if (it->gen != c->generation) {
      (void)hipGraphExecDestroy(it->exec);
      it = c->graphs.erase(it);
    } else {
      ++it;
    }
  }
  for (auto& g : c->graphs) {
    if (g.key != key || g.p0 != p0 || g.p1 != p1) continue;
    HIPCHK(c, hipGraphLaunch(g.exec, c->stream));
    c->graph_launches++;
    size_t k = 0;
    for (int p = p0; p < p1; ++p) {
      ProblemH& P = c->probs[p];
      for (int l = 0; l < P.nlev; ++l, ++k) {
        P.updates[l] += g.upd[k];
        if (g.flips[k]) P.L[l].cur = 1 - P.L[l].cur;
      }
    }
    return MLSWE_OK;
  }
  if ((rc = build_all(c))) return rc;
  std::vector<long long> upd0;
  std::vector<int> cur0;
  for (int p = p0; p < p1; ++p)
    for (int l = 0; l < c->probs[p].nlev; ++l) {
      upd0.push_back(c->probs[p].updates[l]);
      cur0.push_back(c->probs[p].L[l].cur);
    }
  if (!c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  hipStream_t saved = c->stream;
  const bool saved_timing = c->timing;
  c->stream = c->cap_stream;
  c->timing = false;
  hipGraph_t graph = nullptr;
  hipError_t eb = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
  if (eb == hipSuccess) rc = coarse_step(c, p0, p1, true);
  hipError_t ee = eb == hipSuccess ? hipStreamEndCapture(c->cap_stream, &graph) : eb;
  c->stream = saved;
  c->timing = saved_timing;
  auto restore = [&]() {
    size_t k = 0;
    for (int p = p0; p < p1; ++p)
      for (int l = 0; l < c->probs[p].nlev; ++l, ++k) {
        c->probs[p].updates[l] = upd0[k];
        c->probs[p].L[l].cur = cur0[k];
      }
  };
  if (rc || eb != hipSuccess || ee != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    restore();
    return rc ? rc : fail(c, MLSWE_EDEVICE, "graph capture: %s", hipGetErrorString(eb != hipSuccess ? eb : ee));
  }
  mlswe_ctx::GraphRec g;
  g.key = key; g.gen = c->generation; g.p0 = p0; g.p1 = p1;
  hipError_t ei = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ei != hipSuccess) {
    restore();
    return fail(c, MLSWE_EDEVICE, "graph instantiate: %s", hipGetErrorString(ei));
  }
  size_t k = 0;
  for (int p = p0; p < p1; ++p)
    for (int l = 0; l < c->probs[p].nlev; ++l, ++k) {
      g.upd.push_back(c->probs[p].updates[l] - upd0[k]);
      g.flips.push_back(c->probs[p].L[l].cur != cur0[k] ? 1 : 0);
    }
  HIPCHK(c, hipGraphLaunch(g.exec, c->stream));
  c->graphs.push_back(g);
  c->graph_captures++;
  c->graph_launches++;
  return MLSWE_OK;
}

// Backup (to_bk) or restore of a group's coarse-step start: the patch interiors
// of its finer levels and the control blocks and counters of every problem,
// in one launch.
int copy_step_start(mlswe_ctx* c, int p0, int p1, bool to_bk, int nctl, int ncnt) {
  std::vector<CopyBox> boxes;
  long long longest = 0;
  auto add = [&](const double* from, double* to, long long pitch, long long plane, int nx, int ny, int nf) {
    boxes.push_back(CopyBox{from, to, pitch, plane, nx, ny, nf, 0});
    longest = std::max(longest, (long long)nx * ny * nf);
  };
  auto run = [&](double* live, double* saved, long long n) {
    if (n > 0) add(to_bk ? live : saved, to_bk ? saved : live, 0, 0, (int)n, 1, 1);
  };
  static_assert(sizeof(LevelCtl) % sizeof(double) == 0 && sizeof(Counters) % sizeof(double) == 0, "copied as doubles");
  run((double*)c->ctl, (double*)c->ctl_bk, (long long)nctl * (long long)(sizeof(LevelCtl) / sizeof(double)));
  run((double*)c->cnt, (double*)c->cnt_bk, (long long)ncnt * (long long)(sizeof(Counters) / sizeof(double)));
  for (int p = p0; p < p1; ++p) {
    ProblemH& P = c->probs[p];
    for (int l = 1; l < P.nlev; ++l) {
      LevelH& L = P.L[l];
      for (const Box& b : L.boxes) {
        // pieces of whole rows, about 4096 doubles each over the six fields
        const int rows = std::max(1, 4096 / (6 * b.nx));
        for (int j = b.jlo; j < b.jlo + b.ny; j += rows) {
          const long long off = idx(L, b.ilo, j);
          double* q = L.q[L.cur] + off;
          double* k = L.bk + off;
          add(to_bk ? q : k, to_bk ? k : q, L.pitch, L.plane, b.nx, std::min(rows, b.jlo + b.ny - j), 6);
        }
      }
    }
  }
  int rc;
  if ((rc = ensure(c, &c->boxes_d, &c->boxes_cap, (int)boxes.size()))) return rc;
  HIPCHK(c, hipMemcpyAsync(c->boxes_d, boxes.data(), sizeof(CopyBox) * boxes.size(), hipMemcpyHostToDevice, c->stream));
  // a block per piece of up to 4096 doubles (sixteen per thread)
  const unsigned gx = (unsigned)std::min<long long>(64, (longest + 4095) / 4096);
  for (size_t k0 = 0; k0 < boxes.size(); k0 += 65535)  // grid y is at most 65535
    hipLaunchKernelGGL(k_copy_boxes, dim3(gx, (unsigned)std::min<size_t>(65535, boxes.size() - k0)), dim3(256), 0,
                       c->stream, c->boxes_d + k0);
  HIPCHK(c, hipGetLastError());
  return MLSWE_OK;
}

// A coarse step of problems [p0, p1) with rejection: when the largest substep
// Courant number of a problem exceeds cfl_max, every problem of the group is
// put back (fine-level patch interiors, controls, counters, host bookkeeping;
// level 0 keeps its input buffer through a step) and the step is retaken, the
// failing problems with dt scaled by cfl_desired / that number, the others
// unchanged.  Frames and uncovered cells of the finer levels are refilled or
// unused before they are read again, so the backup leaves them out.
int step_with_retry(mlswe_ctx* c, int p0, int p1, int mode) {
  int rc;
  // one launch per level substep over the group's patches, or one per patch
  const bool together = mode == MLSWE_BATCHED || mode == MLSWE_GRAPH;
  const bool retry = c->cfg.max_retries > 0;
  int nctl = 0;
  for (const ProblemH& P : c->probs) nctl += P.nlev;
  const int ncnt = (int)c->probs.size();
  std::vector<int> cur0;
  std::vector<long long> upd0;
  if (retry) {
    if ((rc = ensure(c, &c->ctl_bk, &c->bk_cap, nctl))) return rc;
    if ((rc = ensure(c, &c->cnt_bk, &c->cbk_cap, ncnt))) return rc;
    for (int p = p0; p < p1; ++p) {
      ProblemH& P = c->probs[p];
      for (int l = 0; l < P.nlev; ++l) {
        LevelH& L = P.L[l];
        cur0.push_back(L.cur);
        upd0.push_back(P.updates[l]);
        if (l == 0 || L.boxes.empty()) continue;
        const size_t sb = sizeof(double) * 6 * (size_t)L.plane;
        if (!L.bk && (rc = dalloc(c, (void**)&L.bk, sb))) return rc;
      }
    }
    if ((rc = copy_step_start(c, p0, p1, true, nctl, ncnt))) return rc;
  }
  bool all_dt = true;
  for (int p = p0; p < p1; ++p) all_dt = all_dt && c->probs[p].have_dt;
  if (mode == MLSWE_GRAPH && all_dt && !c->timing)
    rc = graph_step(c, p0, p1);
  else
    rc = coarse_step(c, p0, p1, together);
  if (rc || !retry) return rc;
  const int np = p1 - p0;
  std::vector<double> dt0(np);
  for (int attempt = 0;; ++attempt) {
    if ((size_t)nctl * sizeof(LevelCtl) > c->ctl_pin_cap) {
      if (c->ctl_pin) (void)hipHostFree(c->ctl_pin);
      c->ctl_pin = nullptr;
      c->ctl_pin_cap = 0;
      HIPCHK(c, hipHostMalloc((void**)&c->ctl_pin, 2 * (size_t)nctl * sizeof(LevelCtl), hipHostMallocDefault));
      c->ctl_pin_cap = 2 * (size_t)nctl * sizeof(LevelCtl);
    }
    const LevelCtl* h = c->ctl_pin;  // pinned: the readback is one short DMA
    HIPCHK(c, hipMemcpyAsync(c->ctl_pin, c->ctl, sizeof(LevelCtl) * nctl, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    bool any = false;
    for (int p = p0; p < p1; ++p) {
      const ProblemH& P = c->probs[p];
      double cm = 0.0;
      bool nan = false;
      for (int l = 0; l < P.nlev; ++l) {
        const double v = h[P.ctl0 + l].cmax;
        if (v != v || (h[P.ctl0 + l].status & STATUS_NAN)) nan = true;
        else if (v > cm) cm = v;
      }
      const double dtp = h[P.ctl0].dt;
      if (nan || cm > c->cfg.cfl_max) {
        if (nan) return fail(c, MLSWE_ENAN, "non-finite state or Courant number in problem %d", p);
        any = true;
        dt0[p - p0] = dtp * (c->cfg.cfl_desired / cm);
      } else {
        dt0[p - p0] = dtp;
      }
    }
    if (!any) {
      for (int p = p0; p < p1; ++p) {
        ProblemH& P = c->probs[p];
        for (int l = 0; l < P.nlev; ++l) {
          P.last_acc[l][0] = h[P.ctl0 + l].acc_smax[0];
          P.last_acc[l][1] = h[P.ctl0 + l].acc_smax[1];
        }
        P.acc_known = true;
      }
      return MLSWE_OK;
    }
    if (attempt + 1 > c->cfg.max_retries) return fail(c, MLSWE_ECFL, "Courant number above %g", c->cfg.cfl_max);
    // put the group back
    size_t k = 0;
    for (int p = p0; p < p1; ++p) {
      ProblemH& P = c->probs[p];
      P.rejected++;
      for (int l = 0; l < P.nlev; ++l, ++k) {
        LevelH& L = P.L[l];
        L.cur = cur0[k];
        P.updates[l] = upd0[k];
      }
    }
    if ((rc = copy_step_start(c, p0, p1, false, nctl, ncnt))) return rc;
    if ((rc = ensure(c, &c->dt0_d, &c->dt0_cap, np))) return rc;
    HIPCHK(c, hipMemcpyAsync(c->dt0_d, dt0.data(), sizeof(double) * np, hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL(k_set_dt0, dim3((np + 63) / 64), dim3(64), 0, c->stream, c->ctl, c->pdt + p0, c->dt0_d, np);
    HIPCHK(c, hipGetLastError());
    if ((rc = adv(c, 0, p0, p1, 0.0, together))) return rc;
  }
}

}  // namespace

extern "C" {

int mlswe_advance(mlswe_ctx* c, int nsteps, int regrid_every, const double* tau, int nbuf, int mode, double* dts_out) {
  if (!c) return MLSWE_EINVAL;
  const int np = (int)c->probs.size();
  if (np == 0) return fail(c, MLSWE_ESTATE, "no problem defined");
  if (nsteps < 0 || regrid_every < 0 || (regrid_every > 0 && !tau) || nbuf < 0 ||
      (mode != MLSWE_PLAIN && mode != MLSWE_BATCHED && mode != MLSWE_GRAPH && mode != MLSWE_PER_PATCH))
    return fail(c, MLSWE_EINVAL, "bad advance arguments");
  for (int p = 0; p < np; ++p)
    if (!c->probs[p].bathy || !c->probs[p].state) return fail(c, MLSWE_ESTATE, "problem %d not initialised", p);
  const bool together = mode != MLSWE_PLAIN;
  if (together)
    for (int p = 1; p < np; ++p) {
      if (c->probs[p].nlev != c->probs[0].nlev) return fail(c, MLSWE_EINVAL, "batched problems need equal levels");
      for (int l = 0; l + 1 < c->probs[p].nlev; ++l)
        if (c->probs[p].ratio[l] != c->probs[0].ratio[l]) return fail(c, MLSWE_EINVAL, "batched ratios differ");
    }
  // every coarse step: the regrid of all problems (one pass, the problems are
  // independent), then the step of the problems together (batched, graph: one
  // launch per level substep; per-patch: one launch per patch) or one problem
  // at a time with one launch per patch (plain)
  const int ngroups = together ? 1 : np;
  for (int n = 0; n < nsteps; ++n) {
    int rc;
    if (regrid_every > 0 && n % regrid_every == 0) {
      const auto t0 = std::chrono::steady_clock::now();
      if ((rc = regrid_group(c, 0, np, tau, nbuf))) return rc;
      if (c->timing) {
        c->kms[7] += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        c->klaunch[7] += 1;
      }
    }
    if (c->cfg.dynamic_rt && (rc = choose_time_ratios(c))) return rc;
    if ((rc = build_pdt(c))) return rc;
    for (int gi = 0; gi < ngroups; ++gi) {
      const int p0 = together ? 0 : gi, p1 = together ? np : gi + 1;
      if ((rc = step_with_retry(c, p0, p1, mode))) return rc;
    }
    if (dts_out || c->timing) {
      if ((rc = collect_events(c))) return rc;
    }
    if (dts_out) {
      std::vector<LevelCtl> h;
      if ((rc = read_ctls(c, 0, np, h))) return rc;
      for (int p = 0; p < np; ++p) dts_out[(size_t)p * nsteps + n] = h[c->probs[p].ctl0].dt;
    }
  }
  int status = 0;
  int rc = read_status(c, 0, np, &status);
  if (rc) return rc;
  if (status & STATUS_NAN) return fail(c, MLSWE_ENAN, "non-finite state");
  if (status & STATUS_CFL) return fail(c, MLSWE_ECFL, "Courant number above %g", c->cfg.cfl_max);
  return MLSWE_OK;
}

int mlswe_get_counters(mlswe_ctx* c, int p, mlswe_counters* out) {
  if (!c) return MLSWE_EINVAL;
  if (!valid_prob(c, p) || !out) return fail(c, MLSWE_EINVAL, "bad args");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  Counters h;
  HIPCHK(c, hipMemcpy(&h, c->cnt + c->probs[p].cnt, sizeof h, hipMemcpyDeviceToHost));
  mlswe_counters o;
  std::memset(&o, 0, sizeof o);
  const ProblemH& P = c->probs[p];
  for (int l = 0; l < P.nlev; ++l) o.cell_updates[l] = P.updates[l];
  o.hyp = (int64_t)h.hyp; o.nclip = (int64_t)h.nclip; o.repair = (int64_t)h.repair;
  o.clip1 = h.clip1; o.clip2 = h.clip2;
  o.rejected = P.rejected;
  LevelCtl lc;
  HIPCHK(c, hipMemcpy(&lc, c->ctl + P.ctl0, sizeof lc, hipMemcpyDeviceToHost));
  o.t = lc.t;
  int status = 0;
  int rc = read_status(c, p, p + 1, &status);
  if (rc) return rc;
  o.status = status;
  *out = o;
  return MLSWE_OK;
}

int mlswe_synchronize(mlswe_ctx* c) {
  if (!c) return MLSWE_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return MLSWE_OK;
}

int mlswe_set_kernel_timing(mlswe_ctx* c, int enable) {
  if (!c) return MLSWE_EINVAL;
  int rc = collect_events(c);
  if (rc) return rc;
  c->timing = enable != 0;
  for (int k = 0; k < 8; ++k) { c->kms[k] = 0.0; c->klaunch[k] = 0; }
  return MLSWE_OK;
}

int mlswe_phase_times(mlswe_ctx* c, double* ms_out, int64_t* counts_out, int cap) {
  if (!c || cap < 0 || (cap > 0 && (!ms_out || !counts_out))) return MLSWE_EINVAL;
  int rc = collect_events(c);
  if (rc) return rc;
  for (int k = 0; k < 8 && k < cap; ++k) { ms_out[k] = c->kms[k]; counts_out[k] = c->klaunch[k]; }
  return 8;
}

int mlswe_kernel_times(mlswe_ctx* c, double* ms_out, int64_t* launches_out) {
  if (!c || !ms_out || !launches_out) return MLSWE_EINVAL;
  int rc = collect_events(c);
  if (rc) return rc;
  ms_out[0] = c->kms[0]; ms_out[1] = c->kms[1];
  launches_out[0] = c->klaunch[0]; launches_out[1] = c->klaunch[1];
  return MLSWE_OK;
}

// ------------------------------------------------------------ adjoint
static int ensure_adj(mlswe_ctx* c, ProblemH& P) {
  AdjBuf& A = P.adj;
  if (A.lam1) return MLSWE_OK;
  const LevelH& L = P.L[0];
  const size_t pb = sizeof(double) * (size_t)L.plane;
  int rc;
  if ((rc = dalloc(c, (void**)&A.lam1, 6 * pb)) || (rc = dalloc(c, (void**)&A.lamS, 6 * pb)) ||
      (rc = dalloc(c, (void**)&A.lamG, 6 * pb)) || (rc = dalloc(c, (void**)&A.cL, 7 * pb)) ||
      (rc = dalloc(c, (void**)&A.cR, 7 * pb)) || (rc = dalloc(c, (void**)&A.Bbx, pb)) ||
      (rc = dalloc(c, (void**)&A.Bby, pb)) || (rc = dalloc(c, (void**)&A.status, sizeof(int))))
    return rc;
  HIPCHK(c, hipMemsetAsync(A.lam1, 0, 6 * pb, c->stream));
  HIPCHK(c, hipMemsetAsync(A.lamS, 0, 6 * pb, c->stream));
  HIPCHK(c, hipMemsetAsync(A.lamG, 0, 6 * pb, c->stream));
  HIPCHK(c, hipMemsetAsync(A.cL, 0, 7 * pb, c->stream));
  HIPCHK(c, hipMemsetAsync(A.cR, 0, 7 * pb, c->stream));
  HIPCHK(c, hipMemsetAsync(A.Bbx, 0, pb, c->stream));
  HIPCHK(c, hipMemsetAsync(A.Bby, 0, pb, c->stream));
  HIPCHK(c, hipMemsetAsync(A.status, 0, sizeof(int), c->stream));
  HIPCHK(c, hipHostMalloc((void**)&A.status_host, sizeof(int), hipHostMallocDefault));
  *A.status_host = 0;
  HIPCHK(c, hipEventCreateWithFlags(&A.status_ev, hipEventDisableTiming));
  return MLSWE_OK;
}

static int check_single(mlswe_ctx* c, int p) {
  if (!valid_prob(c, p)) return fail(c, MLSWE_EINVAL, "bad problem %d", p);
  const ProblemH& P = c->probs[p];
  if (!P.bathy) return fail(c, MLSWE_ESTATE, "set the bathymetry first");
  const LevelH& L = P.L[0];
  if (L.boxes.size() != 1 || L.boxes[0].nx != L.nx || L.boxes[0].ny != L.ny)
    return fail(c, MLSWE_EINVAL, "level 0 must be a single patch over the domain");
  return MLSWE_OK;
}


extern "C" int mlswe_run_fixed(mlswe_ctx* c, int p, int n, const double* dts) {
  if (!c) return MLSWE_EINVAL;
  int rc = check_single(c, p);
  if (rc) return rc;
  if (n < 0 || (n > 0 && !dts)) return fail(c, MLSWE_EINVAL, "bad step list");
  ProblemH& P = c->probs[p];
  if (!P.state) return fail(c, MLSWE_ESTATE, "set the state first");
  for (int k = 0; k < n; ++k)
    if (!(dts[k] > 0.0) || !std::isfinite(dts[k])) return fail(c, MLSWE_EINVAL, "dt[%d] must be positive", k);
  // each step's dt travels as a kernel argument: no copy, no host wait
  for (int k = 0; k < n; ++k) {
    hipLaunchKernelGGL(k_set_dt, dim3(1), dim3(1), 0, c->stream, c->ctl + P.ctl0, dts[k]);
    if ((rc = substep(c, 0, p, p + 1, 0.0, false))) return rc;
  }
  return MLSWE_OK;
}

extern "C" int mlswe_adjoint_step(mlswe_ctx* c, int p, const double* q_n, const double* lam_np1, double* lam_n,
                                  double* B_bar, double dt) {
  if (!c) return MLSWE_EINVAL;
  int rc = check_single(c, p);
  if (rc) return rc;
  if (!q_n || !lam_np1 || !lam_n || !B_bar || !(dt > 0.0)) return fail(c, MLSWE_EINVAL, "bad adjoint arguments");
  ProblemH& P = c->probs[p];
  LevelH& L = P.L[0];
  if ((rc = ensure_adj(c, P))) return rc;
  AdjBuf& A = P.adj;
  // a non-wet edge met by an earlier step (its status copy has landed)
  if (hipEventQuery(A.status_ev) == hipSuccess && *A.status_host) {
    *A.status_host = 0;
    HIPCHK(c, hipMemsetAsync(A.status, 0, sizeof(int), c->stream));
    return fail(c, MLSWE_ESTATE, "adjoint needs both layers wet at every edge");
  }
  // forward recomputation: state, walls, x-sweep
  if ((rc = copy_state(c, L, L.cur, q_n, MLSWE_DEVICE, true, nullptr))) return rc;
  hipLaunchKernelGGL(k_set_dt, dim3(1), dim3(1), 0, c->stream, c->ctl + P.ctl0, dt);
  if ((rc = build_launch(c, 0))) return rc;
  if ((rc = launch_fill(c, 0, p, p + 1, 0.0))) return rc;
  LevelLaunch& LL = c->launch[0];
  int k0 = -1;
  for (int k = 0; k < LL.nptch; ++k)
    if (LL.patch_prob[k] == p) { k0 = k; break; }
  if (k0 < 0) return fail(c, MLSWE_ESTATE, "problem %d has no patch", p);
  if ((rc = launch_sweeps(c, 0, L.cur, LL.xr[k0].first, LL.xr[k0].second, 0, 0))) return rc;
  // adjoint of the step's output into the level layout
  hipLaunchKernelGGL(k_copy6, dim3(blocks((long long)L.nx * L.ny)), dim3(256), 0, c->stream, A.lam1, (long long)L.pitch,
                     (long long)L.plane, const_cast<double*>(lam_np1), L.nx, L.ny, 0);
  AdjView V;
  std::memset(&V, 0, sizeof V);
  V.B = L.B; V.cL = A.cL; V.cR = A.cR; V.plane = L.plane; V.P = P.P; V.status = A.status;
  // y-sweep lines: columns, cells along rows
  V.q = L.qs; V.lam = A.lam1;
  V.lstride = 1; V.kstride = L.pitch; V.base = idx(L, 0, 0);
  V.nlines = L.nx; V.n = L.ny; V.orient = 1; V.nu = dt / L.dy;
  hipLaunchKernelGGL(k_adj_edges, dim3(blocks((long long)L.nx * (L.ny + 3))), dim3(256), 0, c->stream, V);
  hipLaunchKernelGGL(k_adj_gather, dim3(blocks((long long)L.nx * (L.ny + 4))), dim3(256), 0, c->stream, V, A.lamS,
                     A.Bby);
  // x-sweep lines: rows -2..ny+1 of the wall-filled state, cells along x
  V.q = L.q[L.cur]; V.lam = A.lamS;
  V.lstride = L.pitch; V.kstride = 1; V.base = idx(L, 0, -2);
  V.nlines = L.ny + 4; V.n = L.nx; V.orient = 0; V.nu = dt / L.dx;
  hipLaunchKernelGGL(k_adj_edges, dim3(blocks((long long)(L.ny + 4) * (L.nx + 3))), dim3(256), 0, c->stream, V);
  hipLaunchKernelGGL(k_adj_gather, dim3(blocks((long long)(L.ny + 4) * (L.nx + 4))), dim3(256), 0, c->stream, V,
                     A.lamG, A.Bbx);
  AdjFold F;
  F.lam_g = A.lamG; F.Bbx = A.Bbx; F.Bby = A.Bby; F.lam_out = lam_n; F.Bbar = B_bar;
  F.pitch = L.pitch; F.plane = L.plane; F.nx = L.nx; F.ny = L.ny;
  hipLaunchKernelGGL(k_adj_fold, dim3(blocks((long long)L.nx * L.ny)), dim3(256), 0, c->stream, F);
  HIPCHK(c, hipGetLastError());
  // the status travels back without a host wait; a later adjoint call or
  // mlswe_param_map_adjoint reports it
  HIPCHK(c, hipMemcpyAsync(A.status_host, A.status, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipEventRecord(A.status_ev, c->stream));
  return MLSWE_OK;
}

extern "C" int mlswe_run_tiles(int nx, int ny, int nbox, const int32_t* boxes, int axis, int rows, int32_t* out,
                               int cap) {
  if (nx <= 0 || ny <= 0 || nbox < 0 || (nbox > 0 && !boxes) || (axis != 0 && axis != 1) || rows <= 0 || cap < 0 ||
      (cap > 0 && !out))
    return MLSWE_EINVAL;
  LevelH L;
  L.nx = nx;
  L.ny = ny;
  for (int k = 0; k < nbox; ++k) {
    Box b{boxes[4 * k], boxes[4 * k + 1], boxes[4 * k + 2], boxes[4 * k + 3]};
    if (b.nx <= 0 || b.ny <= 0 || b.ilo < 0 || b.jlo < 0 || b.ilo + b.nx > nx || b.jlo + b.ny > ny) return MLSWE_EINVAL;
    L.boxes.push_back(b);
  }
  std::vector<XTile> xt;
  std::vector<YTile> yt;
  run_blocks(L, axis, rows, 0, axis == 0 ? &xt : nullptr, axis == 1 ? &yt : nullptr);
  const size_t n = axis == 0 ? xt.size() : yt.size();
  for (size_t k = 0; k < n && k < (size_t)cap; ++k) {
    int32_t* o = out + 5 * k;
    if (axis == 0) { o[0] = xt[k].i0; o[1] = xt[k].ncols; o[2] = xt[k].j0; o[3] = xt[k].nrows; o[4] = xt[k].flags; }
    else { o[0] = yt[k].i0; o[1] = yt[k].ncols; o[2] = yt[k].j0; o[3] = yt[k].nrows; o[4] = yt[k].last; }
  }
  return (int)n;
}

extern "C" int mlswe_branch_signature(mlswe_ctx* c, int enable, int p, uint64_t* sig_out) {
  if (!c) return MLSWE_EINVAL;
  if (enable >= 0 && (enable ? 1 : 0) != c->sig_on) {
    c->sig_on = enable ? 1 : 0;
    c->generation++;
    for (int l = 0; l < MAXLEV; ++l) c->launch[l].dirty = true;
  }
  if (sig_out) {
    if (!valid_prob(c, p)) return fail(c, MLSWE_EINVAL, "bad problem %d", p);
    Counters h;
    HIPCHK(c, hipMemcpyAsync(&h, c->cnt + c->probs[p].cnt, sizeof h, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *sig_out = h.sig;
    h.sig = 0;
    HIPCHK(c, hipMemcpyAsync(c->cnt + c->probs[p].cnt, &h, sizeof h, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return MLSWE_OK;
}

extern "C" int mlswe_param_map(mlswe_ctx* c, int p, const double* eta1_0, double eta2_0, double* q_out) {
  if (!c) return MLSWE_EINVAL;
  int rc = check_single(c, p);
  if (rc) return rc;
  if (!eta1_0 || !q_out) return fail(c, MLSWE_EINVAL, "null pointer");
  const LevelH& L = c->probs[p].L[0];
  ParamMap M;
  M.eta1 = eta1_0; M.B = L.B; M.q = q_out; M.pitch = L.pitch; M.nx = L.nx; M.ny = L.ny;
  M.eta2 = eta2_0; M.hdry = c->probs[p].P.hdry;
  hipLaunchKernelGGL(k_param_map, dim3(blocks((long long)L.nx * L.ny)), dim3(256), 0, c->stream, M);
  HIPCHK(c, hipGetLastError());
  return MLSWE_OK;
}

extern "C" int mlswe_param_map_adjoint(mlswe_ctx* c, int p, const double* eta1_0, double eta2_0, const double* lam0,
                                       double* eta1_bar, double* B_bar) {
  if (!c) return MLSWE_EINVAL;
  int rc = check_single(c, p);
  if (rc) return rc;
  if (!eta1_0 || !lam0 || !eta1_bar || !B_bar) return fail(c, MLSWE_EINVAL, "null pointer");
  const LevelH& L = c->probs[p].L[0];
  AdjBuf& A = c->probs[p].adj;
  if (A.status) {  // the adjoint steps so far: any non-wet edge fails the chain
    HIPCHK(c, hipStreamSynchronize(c->stream));
    int st = 0;
    HIPCHK(c, hipMemcpy(&st, A.status, sizeof(int), hipMemcpyDeviceToHost));
    if (st) {
      *A.status_host = 0;
      HIPCHK(c, hipMemset(A.status, 0, sizeof(int)));
      return fail(c, MLSWE_ESTATE, "adjoint needs both layers wet at every edge");
    }
  }
  ParamMap M;
  M.eta1 = eta1_0; M.B = L.B; M.q = nullptr; M.pitch = L.pitch; M.nx = L.nx; M.ny = L.ny;
  M.eta2 = eta2_0; M.hdry = c->probs[p].P.hdry;
  hipLaunchKernelGGL(k_param_map_adj, dim3(blocks((long long)L.nx * L.ny)), dim3(256), 0, c->stream, M, lam0,
                     eta1_bar, B_bar);
  HIPCHK(c, hipGetLastError());
  return MLSWE_OK;
}

extern "C" int mlswe_gauge_misfit(mlswe_ctx* c, int p, const double* q, int i0, int j0, int gn, const double* target,
                                  double* loss, double* lam, double* B_bar) {
  if (!c) return MLSWE_EINVAL;
  int rc = check_single(c, p);
  if (rc) return rc;
  const LevelH& L = c->probs[p].L[0];
  if (!target || gn <= 0 || i0 < 0 || j0 < 0 || i0 + gn > L.nx || j0 + gn > L.ny)
    return fail(c, MLSWE_EINVAL, "gauge region outside the domain");
  Gauge G;
  G.q = q ? q : L.q[L.cur]; G.qlevel = q ? 0 : 1;
  G.qplane = q ? (long long)L.nx * L.ny : L.plane;
  G.B = L.B; G.target = target; G.loss = loss; G.lam = lam; G.B_bar = B_bar;
  G.pitch = L.pitch; G.nx = L.nx; G.ny = L.ny; G.i0 = i0; G.j0 = j0; G.gn = gn;
  hipLaunchKernelGGL(k_gauge, dim3(1), dim3(256), 0, c->stream, G);
  HIPCHK(c, hipGetLastError());
  return MLSWE_OK;
}


// ------------------------------------------------------------ tuning
extern "C" int mlswe_get_tuning(mlswe_ctx* c, mlswe_tuning* out) {
  if (!c || !out) return MLSWE_EINVAL;
  *out = c->tune;
  return MLSWE_OK;
}

extern "C" int mlswe_set_tuning(mlswe_ctx* c, const mlswe_tuning* t) {
  if (!c || !t) return MLSWE_EINVAL;
  if (t->x_rows < 0 || t->x_rows > 4096 || t->y_rows < 0 || t->y_rows > 4096 || t->sched_x < 0 || t->sched_x > 2 ||
      t->sched_y < 0 || t->sched_y > 2 || t->grid_x < 0 || t->grid_x > 64 || t->grid_y < 0 || t->grid_y > 64 ||
      t->fast < 0 || t->fast > 1)
    return fail(c, MLSWE_EINVAL, "bad tuning");
  c->tune = *t;
  c->generation++;
  for (int l = 0; l < MAXLEV; ++l) c->launch[l].dirty = true;
  return MLSWE_OK;
}

static std::string layout_key(const mlswe_ctx* c) {
  std::string k = "np=" + std::to_string(c->probs.size());
  int nl = 0;
  for (const ProblemH& P : c->probs) nl = std::max(nl, P.nlev);
  for (int l = 0; l < nl; ++l) {
    long long cells = 0, npatch = 0;
    for (const ProblemH& P : c->probs)
      if (l < P.nlev)
        for (const Box& b : P.L[l].boxes) { cells += (long long)b.nx * b.ny; ++npatch; }
    k += ";L" + std::to_string(l) + "=" + std::to_string(npatch) + "/" + std::to_string(cells);
  }
  return k;
}

// Milliseconds of reps launches of one sweep (axis 0: x, 1: y) over the patches
// of every level of every problem.
static int time_sweeps(mlswe_ctx* c, int axis, int reps, double* ms) {
  int rc;
  if ((rc = build_all(c))) return rc;
  hipEvent_t a, b;
  HIPCHK(c, hipEventCreate(&a));
  HIPCHK(c, hipEventCreate(&b));
  int nl = 0;
  for (const ProblemH& P : c->probs) nl = std::max(nl, P.nlev);
  auto launch_all = [&]() -> int {
    for (int l = 0; l < nl; ++l) {
      LevelLaunch& LL = c->launch[l];
      if (LL.nptch == 0) continue;
      const int par = c->probs[LL.patch_prob[0]].L[l].cur;
      // the tiles a batched substep would launch: run tiles for one-wave
      // schedules on levels with several patches per problem
      const bool run = LL.use_runs && (axis == 0 ? c->tune.sched_x : c->tune.sched_y) == 0 && !c->sig_on;
      const int t0 = axis == 0 ? (run ? LL.nxt_p : 0) : (run ? LL.nyt_p : 0);
      const int n = axis == 0 ? (run ? LL.nxt - LL.nxt_p : LL.nxt_p) : (run ? LL.nyt - LL.nyt_p : LL.nyt_p);
      int r2 = axis == 0 ? launch_sweeps(c, l, par, t0, n, 0, 0, run, false)
                         : launch_sweeps(c, l, par, 0, 0, t0, n, false, run);
      if (r2) return r2;
    }
    return MLSWE_OK;
  };
  if ((rc = launch_all())) return rc;  // warm-up
  HIPCHK(c, hipEventRecord(a, c->stream));
  for (int k = 0; k < reps; ++k)
    if ((rc = launch_all())) return rc;
  HIPCHK(c, hipEventRecord(b, c->stream));
  HIPCHK(c, hipEventSynchronize(b));
  float f = 0.f;
  HIPCHK(c, hipEventElapsedTime(&f, a, b));
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  *ms = f / reps;
  return MLSWE_OK;
}

extern "C" int mlswe_autotune(mlswe_ctx* c, const char* cache_path, int reps) {
  if (!c) return MLSWE_EINVAL;
  if (c->probs.empty()) return fail(c, MLSWE_ESTATE, "no problem defined");
  for (const ProblemH& P : c->probs)
    if (!P.bathy || !P.state) return fail(c, MLSWE_ESTATE, "problems must be initialised before tuning");
  if (reps <= 0) reps = 3;
  for (ProblemH& P : c->probs) P.acc_known = false;  // timed sweeps run on the device copies
  const std::string key = layout_key(c);
  if (cache_path) {
    FILE* f = std::fopen(cache_path, "r");
    if (f) {
      char line[1024];
      while (std::fgets(line, sizeof line, f)) {
        char k[900];
        mlswe_tuning t;
        if (std::sscanf(line, "%899s %d %d %d %d %d %d", k, &t.x_rows, &t.y_rows, &t.sched_x, &t.sched_y, &t.grid_x,
                        &t.grid_y) == 7 &&
            key == k) {
          std::fclose(f);
          t.fast = c->tune.fast;
          return mlswe_set_tuning(c, &t);
        }
      }
      std::fclose(f);
    }
  }
  const bool saved_timing = c->timing;
  c->timing = false;
  int nctl = 0;
  for (const ProblemH& P : c->probs) nctl += P.nlev;
  const int ncnt = (int)c->probs.size();
  std::vector<LevelCtl> ctl_save(nctl);
  std::vector<Counters> cnt_save(ncnt);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(ctl_save.data(), c->ctl, sizeof(LevelCtl) * nctl, hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(cnt_save.data(), c->cnt, sizeof(Counters) * ncnt, hipMemcpyDeviceToHost));
  const int scheds[5][2] = {{0, 0}, {1, 1}, {1, 2}, {2, 1}, {2, 2}};
  mlswe_tuning best = c->tune;
  int rc = MLSWE_OK;
  for (int axis = 0; axis < 2 && !rc; ++axis) {
    // 0: the per-level choice made when the tiles are built
    const int rows_x[5] = {0, 4, 8, 16, 32};
    const int rows_y[6] = {0, 16, 32, 64, 128, 256};
    const int nrows = axis == 0 ? 5 : 6;
    double best_ms = 1e300;
    for (int ri = 0; ri < nrows && !rc; ++ri)
      for (int si = 0; si < 5 && !rc; ++si) {
        mlswe_tuning t = best;
        if (axis == 0) { t.x_rows = rows_x[ri]; t.sched_x = scheds[si][0]; t.grid_x = scheds[si][1]; }
        else { t.y_rows = rows_y[ri]; t.sched_y = scheds[si][0]; t.grid_y = scheds[si][1]; }
        if ((rc = mlswe_set_tuning(c, &t))) break;
        double ms = 0;
        if ((rc = time_sweeps(c, axis, reps, &ms))) break;
        if (ms < best_ms) {
          best_ms = ms;
          if (axis == 0) { best.x_rows = t.x_rows; best.sched_x = t.sched_x; best.grid_x = t.grid_x; }
          else { best.y_rows = t.y_rows; best.sched_y = t.sched_y; best.grid_y = t.grid_y; }
        }
      }
  }
  c->timing = saved_timing;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(c->ctl, ctl_save.data(), sizeof(LevelCtl) * nctl, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->cnt, cnt_save.data(), sizeof(Counters) * ncnt, hipMemcpyHostToDevice));
  if (rc) return rc;
  if ((rc = mlswe_set_tuning(c, &best))) return rc;
  if (cache_path) {
    FILE* f = std::fopen(cache_path, "a");
    if (f) {
      std::fprintf(f, "%s %d %d %d %d %d %d\n", key.c_str(), best.x_rows, best.y_rows, best.sched_x, best.sched_y,
                   best.grid_x, best.grid_y);
      std::fclose(f);
    }
  }
  return MLSWE_OK;
}

}  // extern "C"
