// Launch descriptors shared by the HIP kernels and the host library.
#pragma once
#include "mlswe_device.hpp"

namespace mlswe {

constexpr int XOFF = 8;         // column offset of interior column 0 within a row
constexpr int XTILE_COLS = 60;  // interior columns per x-sweep wave (64 lanes - 4 halo)
// Waves per block of the one-wave-per-tile sweep kernels.  The waves share
// nothing, and a block's LDS is released only when all its waves are done, so
// smaller blocks let a finished tile's slot take the next tile at once.
constexpr int LEAN_WAVES = 1;
constexpr int STATUS_CFL = 1;
constexpr int STATUS_NAN = 2;

// Halt words of a context (device memory), for coarse steps whose Courant
// check is deferred: while HALT_ARMED is set, the first substep reduction that
// finds a Courant number above the limit (or a non-finite state) sets
// HALT_SET, and from then on the kernels that would change what a retake
// needs (y-sweep outputs, coarsening, the dt rule, the step-start backups and
// the substep reductions' results) do nothing, so the backup still holds the
// failing step's start.  HALT_MARKS counts the backups taken while armed and
// not halted: the failing step's index in the window plus one.
constexpr int HALT_SET = 0, HALT_MARKS = 1, HALT_ARMED = 2, HALT_WORDS = 4;

struct Counters {
  unsigned long long hyp, nclip, repair;
  double clip1, clip2;
  unsigned long long sig;  // branch signature (sum of position-hashed limiter branches)
  unsigned long long pad[2];
};

// Device-resident time-step control of one (problem, level).
struct LevelCtl {
  double dt;                        // substep of this level
  unsigned long long acc_smax[2];   // largest speeds over the current coarse step
  unsigned long long last_smax[2];  // largest speeds of the last finished substep
  double t;                         // simulated time (level 0 entry of a problem)
  double cmax;                      // largest substep Courant number of the coarse step
  int status;
  int pad;
};

// One patch of one level of one problem as seen by the sweep kernels.
struct PatchDev {
  const double* q;   // input state (field 0 plane; field f at + f * plane)
  double* qo;        // output state
  double* qs;        // x-swept intermediate state
  const double* B;
  LevelCtl* ctl;
  Counters* cnt;
  long long pitch, plane;
  int ilo, jlo, nx, ny;
  double dx, dy;
  PhysParams P;
  int sig_on;        // accumulate the branch signature into cnt->sig
  const unsigned char* mask;  // coverage of the level (bits below)
  const unsigned* halt;       // the context's halt words (HALT_*)
  const unsigned* skip;       // the problem's skip flag (set: a retake of other problems)
};

// Coverage byte of a level cell: interior of some patch, and whether the cell
// is the first column / first row of that patch.  A cell's neighbour to the
// left (below) lies in the same patch iff both are interior and the cell is
// not a first column (row).
constexpr unsigned char COV_IN = 1, COV_COL0 = 2, COV_ROW0 = 4;

// Sweep tiles.  Patch tiles cover one patch (its rows and two frame rows on
// each side for x, its interior for y).  Run tiles cover fixed blocks of the
// union of a level's patches (60 or 64 columns by a row chunk): `patch` is then
// the level's descriptor, cells and edges are told apart through the coverage
// bytes, and flags bit 0 says the tile owns the edge after its last column (x)
// or row (y) because no tile of the union follows it.
struct XTile { int patch, i0, ncols, j0, nrows, flags; };
struct YTile { int patch, i0, ncols, j0, nrows, last; };

// Ghost fill / regrid refine of one fine patch.
struct FillPatch {
  double* q;                  // fine level buffer written
  const double* B;            // fine bathymetry
  const unsigned char* mask;  // fine coverage
  const unsigned char* mask_old;  // coverage before a regrid (new-cell fill only)
  const double* qco;          // coarse state at the start of its step
  const double* qcn;          // coarse state at the end of its step
  const double* Bc;
  Counters* cnt;
  long long pitch, plane, cpitch, cplane;
  int nx, ny, ncx, ncy;
  int ilo, jlo, bnx, bny;
  int r;
  int coarse_none;            // level 0: walls only
  PhysParams P;
  const unsigned* skip;       // the problem's skip flag (null: never skipped)
};

struct CoarsenPatch {
  const double* qf;
  double* qc;
  long long fpitch, fplane, cpitch, cplane;
  int ilo, jlo, bnx, bny, r;
  PhysParams P;
  const unsigned* halt;
  const unsigned* skip;
};

struct FlagLevel {
  const double* q;            // current state (field 0 = h1)
  const double* B;
  const unsigned char* mask;
  unsigned char* raw;         // nx * ny scratch
  unsigned char* out;         // nx * ny flags
  long long pitch, plane;
  int nx, ny, nbuf;
  double dx, dy, tau, hdry;
};

// Clustering works on tiles of CLUSTER_TILE x CLUSTER_TILE fine cells.  The
// tile summary of one level of one problem: per tile of the finer level, bit 0
// = a flagged coarse cell under it, bit 1 = the coarse cells under it and two
// around it (clipped to the level) are all covered.
constexpr int CLUSTER_TILE = 16;
struct FlagTiles {
  const unsigned char* flags;  // nx * ny dilated flags of the coarse level
  const unsigned char* mask;   // coverage of the coarse level
  unsigned char* out;          // tx * ty tile bits, row-major
  long long pitch;
  int nx, ny, r, tx, ty;
};

// Partial results of one sweep tile (largest edge speed, fix-up and clamp
// counts), written by the tile's wave and reduced per problem and level after
// the substep, so no two waves update the same word.
struct TilePart {
  double smax, clip1, clip2;
  unsigned hyp, nclip, repair, nonfinite;
};

// One problem on one level: its control block and counters, spacings, and the
// ranges of its x- and y-tile partials in the level's partial array.
struct LevelInfo {
  int ctl, cnt, prob;
  double dx, dy;
  int x0, nx, y0, ny;
};

struct SpeedLevel {
  const double* q;
  const unsigned char* mask;
  LevelCtl* ctl;
  long long pitch, plane;
  int nx, ny;
  double g, hdry;
};

struct ProbDt {
  int ctl0, nlev;
  int ratio[8];   // space ratios (the dt limit)
  int rt[8];      // time ratios of the coming coarse step (the levels' substeps)
  int active[8];
  double dx[8], dy[8];
  double* dt_out;
};

// Lines of one sweep for the adjoint: cell (line, k) at base + line * lstride
// + k * kstride, field f at + f * plane.  orient 0: normal momentum hu (x-sweep),
// 1: hv (y-sweep).  Cells -2..n+1 exist, cells 0..n-1 are updated.
struct AdjView {
  const double* q;
  const double* B;
  const double* lam;   // adjoint of the sweep's outputs (read at cells 0..n-1)
  long long lplane, lbase, llstride, lkstride;  // its own indexing (level or dense layout)
  long long plane, lstride, kstride, base;
  int nlines, n, orient;
  double nu;
  PhysParams P;
  int* status;
};

struct AdjFold {
  const double* lam_g;   // adjoint of the wall-filled state (level layout)
  const double* Bbx;     // bathymetry adjoint from the x-sweep (level layout)
  const double* Bby;     // from the y-sweep (level layout, interior columns)
  double* lam_out;       // [6][ny][nx]
  double* Bbar;          // [ny][nx], accumulated
  long long pitch, plane;
  int nx, ny;
};

struct ParamMap {
  const double* eta1;  // [ny][nx]
  const double* B;     // level array
  double* q;           // [6][ny][nx]
  long long pitch;
  int nx, ny;
  double eta2, hdry;
};

struct Gauge {
  const double* q;       // state: level layout (qlevel = 1) or [6][ny][nx]
  const double* B;       // level array
  const double* target;  // [gn][gn]
  double* loss;          // device scalar (accumulated) or null
  double* lam;           // [6][ny][nx] accumulated source or null
  double* B_bar;         // [ny][nx] accumulated or null
  long long pitch, qplane;
  int nx, ny, i0, j0, gn, qlevel;
};

__global__ void k_adj_edges_row(AdjView V, double* lam_in, double* Bbar);
__global__ void k_adj_edges_col(AdjView V, double* lam_in, double* Bbar);
__global__ void k_adj_fold(AdjFold F);
__global__ void k_param_map(ParamMap M);
__global__ void k_param_map_adj(ParamMap M, const double* __restrict__ lam0, double* eta1_bar, double* B_bar);
__global__ void k_gauge(Gauge G);
__global__ void k_set_dt(LevelCtl* ctl, double dt);

__global__ void k_sweep_x(const PatchDev* __restrict__ patches, const XTile* __restrict__ tiles, int ntiles, int sched,
                          unsigned* ticket, TilePart* parts);
__global__ void k_sweep_y(const PatchDev* __restrict__ patches, const YTile* __restrict__ tiles, int ntiles, int sched,
                          unsigned* ticket, TilePart* parts);
__global__ void k_sweep_xr(const PatchDev* __restrict__ patches, const XTile* __restrict__ tiles, int ntiles,
                           TilePart* parts);
__global__ void k_sweep_yr(const PatchDev* __restrict__ patches, const YTile* __restrict__ tiles, int ntiles,
                           TilePart* parts);
__global__ void k_sweep_xr_fast(const PatchDev* __restrict__ patches, const XTile* __restrict__ tiles, int ntiles,
                                TilePart* parts);
__global__ void k_sweep_yr_fast(const PatchDev* __restrict__ patches, const YTile* __restrict__ tiles, int ntiles,
                                TilePart* parts);
__global__ void k_sweep_x1(const PatchDev* __restrict__ patches, const XTile* __restrict__ tiles, int ntiles,
                           TilePart* parts);
__global__ void k_sweep_y1(const PatchDev* __restrict__ patches, const YTile* __restrict__ tiles, int ntiles,
                           TilePart* parts);
__global__ void k_sweep_x1_fast(const PatchDev* __restrict__ patches, const XTile* __restrict__ tiles, int ntiles,
                                TilePart* parts);
__global__ void k_sweep_y1_fast(const PatchDev* __restrict__ patches, const YTile* __restrict__ tiles, int ntiles,
                                TilePart* parts);
__global__ void k_sweep_x_fast(const PatchDev* __restrict__ patches, const XTile* __restrict__ tiles, int ntiles,
                               int sched, unsigned* ticket, TilePart* parts);
__global__ void k_sweep_y_fast(const PatchDev* __restrict__ patches, const YTile* __restrict__ tiles, int ntiles,
                               int sched, unsigned* ticket, TilePart* parts);
__global__ void k_zero_u32(unsigned* p, int n);
__global__ void k_ghost_fill(const FillPatch* __restrict__ fills, int pass, double theta, LevelCtl* dt_ctl,
                             double dt);
__global__ void k_refine_new(const FillPatch* __restrict__ fills);
__global__ void k_coarsen(const CoarsenPatch* __restrict__ cps);

// Mass flux correction at coarse-fine edges: one record per coarse cell O
// (level l, outside level l + 1) with face neighbours covered by level l + 1.
// dirs bit d: the neighbour in direction d (+x, -x, +y, -y) is covered.  reg
// holds, per direction and layer, the coarse face flux (gc) and the running
// sum over fine substeps of the fine face fluxes along the face (acc).
struct RefluxCell {
  double* cq[2];          // level l buffers by parity
  const double* cqs;      // level l x-swept state
  const double* cB;
  const double* fq[2];    // level l + 1 buffers by parity
  const double* fqs;
  const double* fB;
  const LevelCtl* cctl;
  const LevelCtl* fctl;
  double* reg;            // [4][2] gc, [4][2] acc, then [4][16][2] fine face fluxes of a substep
  long long cpitch, cplane, fpitch, fplane;
  int i, j, dirs, r;
  double cdx, cdy, fdx, fdy;
  PhysParams P;
  const unsigned* skip;
};
__global__ void k_reflux_coarse(const RefluxCell* __restrict__ rc, int n, int parity);
__global__ void k_reflux_fine(const RefluxCell* __restrict__ rc, int n, int parity);
__global__ void k_reflux_fsum(const RefluxCell* __restrict__ rc, int n);
constexpr int REFLUX_REG = 16 + 128;  // doubles of registers per record (ratios up to 16)
__global__ void k_reflux_apply(const RefluxCell* __restrict__ rc, int n, int parity, int rt);
__global__ void k_flag_raw(const FlagLevel* __restrict__ Fs);
__global__ void k_flag_dilate(const FlagLevel* __restrict__ Fs);
__global__ void k_flag_raw_v(FlagLevel F);
__global__ void k_flag_dilate_v(FlagLevel F);
__global__ void k_flag_tiles(const FlagTiles* __restrict__ Ts);
// Reduction of one slice of a (problem, level)'s tile partials when several
// blocks share the reduction.
struct SliceRed {
  double sx, sy, c1, c2;
  unsigned long long h, nc, rp, nf;
};
constexpr int AFTER_MAX_SLICES = 32;
__global__ void k_after_substep(LevelCtl* ctls, Counters* cnts, const LevelInfo* infos, const TilePart* parts,
                                double cflmax, SliceRed* red, unsigned* halt, const unsigned* skip);
__global__ void k_after_combine(LevelCtl* ctls, Counters* cnts, const LevelInfo* infos, int n, int ns,
                                const SliceRed* __restrict__ red, double cflmax, unsigned* halt,
                                const unsigned* skip);
__global__ void k_initial_speed(const SpeedLevel* __restrict__ sl);
__global__ void k_next_dt(LevelCtl* ctls, const ProbDt* __restrict__ pd, int nprob, double cfl, int initial,
                          const unsigned* halt);
__global__ void k_nan_uncovered(double* q, const unsigned char* __restrict__ mask, long long pitch, int nx, int ny);
__global__ void k_zero_uncovered(double* q, const unsigned char* __restrict__ mask, long long pitch, long long plane,
                                 int nx, int ny);
// A contiguous run of doubles to copy (one row range of one field plane).
// A box of nf fields copied between two arrays of the same layout: element
// (f, a, b) at f * plane + b * pitch + a from the box origins src / dst.  A
// plain run of n doubles is nf = 1, ny = 1, nx = n.
struct CopyBox {
  const double* src;
  double* dst;
  long long pitch, plane;
  int nx, ny, nf, pad;
  const unsigned* skip;  // the owning problem's skip flag (null: always copied)
};
__global__ void k_copy_boxes(const CopyBox* __restrict__ boxes, unsigned* halt, int mark);
__global__ void k_set_halt(unsigned* halt, unsigned armed);
// Byte runs: copied (src set) or filled with a value (src null).
struct ByteSeg {
  const unsigned char* src;
  unsigned char* dst;
  long long n;
  int value;
};
__global__ void k_byte_segs(const ByteSeg* __restrict__ segs);
// One patch box of a level's coverage mask, to be set.
struct MaskBox {
  unsigned char* mask;
  long long pitch;
  int ilo, jlo, nx, ny;
};
__global__ void k_mask_boxes(const MaskBox* __restrict__ boxes);
__global__ void k_copy6(double* lv, long long pitch, long long plane, double* cq, int nx, int ny, int dir);
__global__ void k_reset_acc(LevelCtl* ctls, const ProbDt* __restrict__ pd, int nprob);
__global__ void k_set_dt0(LevelCtl* ctls, const ProbDt* __restrict__ pd, const double* __restrict__ dt0, int nprob,
                          const unsigned* skip);
// Skip flags of problems 0..n-1: set where fail[p] is 0 (the problems a retake
// leaves alone), cleared where it is 1; fail null clears them all.
__global__ void k_set_skip(unsigned* skip, const unsigned char* __restrict__ fail, int n);

}  // namespace mlswe
