// Host-side internals of libmlswe.so shared by its source files: the
// context with its problems, levels and launch data, and the helpers the
// files call across (contexts and state: mlswe_lib.cpp; launch data and
// launches: mlswe_launch.cpp; patches, flags and regrids: mlswe_regrid.cpp;
// coarse steps, graphs and retakes: mlswe_advance.cpp; adjoint entry
// points: mlswe_adjoint_host.cpp; tuning: mlswe_tuning.cpp).
#pragma once
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

#include "mlswe.h"
#include "mlswe_kernels.hpp"
#include "mlswe_layers.hpp"

using namespace mlswe;

namespace mlswe_host {

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
  double* lamS = nullptr;  // adjoint of the x-swept state
  double* lamG = nullptr;  // adjoint of the wall-filled state
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
  SliceRed* red = nullptr;                   // slice results of the partial reduction
  int cap_red = 0;
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

}  // namespace mlswe_host

using namespace mlswe_host;


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
  unsigned* halt = nullptr;     // [HALT_WORDS] halt words of deferred Courant checks
  bool armed = false;           // a deferred window is open (halt words armed)
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
  long long host_waits = 0;  // waits of the host on the context's stream
  unsigned* skip = nullptr;  // per problem: set while a retake leaves it alone
  int skip_cap = 0;
  unsigned char* fail_d = nullptr;  // per problem: taken again by a retake
  int fail_cap = 0;
  LevelCtl* dt_ctl = nullptr;  // a time step for the next fill launch to store (fixed-grid calls)
  double dt_value = 0.0;
  LevelCtl* ctl_bk = nullptr;
  Counters* cnt_bk = nullptr;
  int bk_cap = 0, cbk_cap = 0;
  double* dt0_d = nullptr;
  int dt0_cap = 0;
  // copy lists uploaded for the current launch data, by (direction, buffer
  // parities of the group's levels): a backup is one launch with no upload
  struct BoxList {
    bool to_bk;
    std::vector<char> cur;  // buffer parity of every level above 0 of the group
    long long gen;
    int p0, p1;
    CopyBox* d;
    int n;
    long long longest;
  };
  std::vector<BoxList> box_lists;
  LevelCtl* ctl_pin = nullptr;  // pinned readback of the control blocks
  size_t ctl_pin_cap = 0;
  unsigned char* pin = nullptr;  // pinned staging of the regrid flags
  size_t pin_cap = 0;
  ByteSeg* bsegs_d = nullptr;    // regrid descriptor lists
  int bsegs_cap = 0;
  // host sides of the regrid's descriptor copies: kept until the next regrid
  // level, whose flag readback waits for the stream before they are rebuilt
  std::vector<ByteSeg> rg_segs;
  std::vector<MaskBox> rg_boxes;
  std::vector<FillPatch> rg_fills;
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

namespace mlswe_host {

#define HIPCHK(c, call)                                                                      \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess) return fail((c), MLSWE_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

inline long long idx(const LevelH& L, int i, int j) { return (long long)(j + 2) * L.pitch + (i + XOFF); }
// The host waits for the context's stream (every such wait is counted).
inline hipError_t host_wait(mlswe_ctx* c) {
  c->host_waits++;
  return hipStreamSynchronize(c->stream);
}
inline unsigned blocks(long long n) { return (unsigned)((n + 255) / 256); }
inline bool valid_prob(mlswe_ctx* c, int p) { return p >= 0 && p < (int)c->probs.size(); }

int fail(mlswe_ctx* c, int code, const char* fmt, ...);
int dalloc(mlswe_ctx* c, void** p, size_t bytes);
void dfree(void* p);
void mirror_frame_host(const LevelH& L, std::vector<double>& a);
std::vector<Box> cluster_tiles(int fnx, int fny, const unsigned char* bits);
long long run_blocks(const LevelH& L, int axis, int rows, int pdi, std::vector<XTile>* xo, std::vector<YTile>* yo,
                     std::vector<int>* rows_out = nullptr);
long long tile_makespan(const std::vector<int>& rows, int extra, long long slots);
int build_reflux(mlswe_ctx* c, int l, std::vector<RefluxCell>& out);
int build_launch(mlswe_ctx* c, int l);
void mark_dirty(mlswe_ctx* c, int l);
int build_pdt(mlswe_ctx* c);
int ev_begin(mlswe_ctx* c, hipEvent_t* e);
int collect_events(mlswe_ctx* c);
int launch_sweeps(mlswe_ctx* c, int l, int parity, int xt0, int nxt, int yt0, int nyt, bool rx = false,
                  bool ry = false);
int launch_fill(mlswe_ctx* c, int l, int p0, int p1, double theta);
int launch_after(mlswe_ctx* c, int l, int p0, int p1, int runs);
int launch_reflux(mlswe_ctx* c, int lf, int p0, int p1, int which, int parity);
int substep(mlswe_ctx* c, int l, int p0, int p1, double theta, bool batched);
int coarsen_level(mlswe_ctx* c, int lf, int p0, int p1, bool apply_reflux = false);
bool level_active(const mlswe_ctx* c, int l, int p0, int p1);
int adv(mlswe_ctx* c, int l, int p0, int p1, double theta, bool batched);
int next_dt(mlswe_ctx* c, int p0, int p1, bool initial);
int read_ctls(mlswe_ctx* c, int p0, int p1, std::vector<LevelCtl>& h);
int read_status(mlswe_ctx* c, int p0, int p1, int* status);
void host_mask(LevelH& L);
const std::vector<unsigned char>& host_cov(LevelH& L);
int upload_mask(mlswe_ctx* c, LevelH& L);
int check_patches(mlswe_ctx* c, int p, int l, int n, const int32_t* bx, std::vector<Box>& nb_out);
int set_patches_impl(mlswe_ctx* c, int p, int l, int n, const int32_t* bx);
int flag_impl(mlswe_ctx* c, int p, int l, double tau, int nbuf, std::vector<unsigned char>& out);
int regrid_group(mlswe_ctx* c, int p0, int p1, const double* tau_all, int nbuf);
int regrid_impl(mlswe_ctx* c, int p, const double* tau, int nbuf);
int copy_state(mlswe_ctx* c, LevelH& L, int buf, const double* src, int where, bool to_dev, double* dst);
int choose_time_ratios(mlswe_ctx* c);
int build_all(mlswe_ctx* c);
int coarse_step(mlswe_ctx* c, int p0, int p1, bool batched);
int graph_step(mlswe_ctx* c, int p0, int p1);
int copy_step_start(mlswe_ctx* c, int p0, int p1, bool to_bk, bool mark);
int step_with_retry(mlswe_ctx* c, int p0, int p1, int mode, bool* retaken = nullptr);

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

}  // namespace mlswe_host
