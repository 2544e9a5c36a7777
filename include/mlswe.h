/*
 * mlswe.h -- C ABI of the MI355X two-layer shallow-water AMR hot path.
 *
 * Paper: A. Schwarzschild, K. Mandli, "An Implementation of Adaptive Mesh
 * Refinement for Shallow Water Equations" (arXiv 1803.01450).
 *
 * Conventions for every entry point:
 *  - Returns 0 on success or a negative MLSWE_E* code; mlswe_last_error(ctx)
 *    then holds a message.  No C++ exception crosses this boundary.
 *  - Out-parameters are written only on success.
 *  - State arrays are structure-of-arrays FP64, field-major, rows with x
 *    fastest: q[f][j][i] for the fields f = h1, h1*u1, h1*v1, h2, h2*u2, h2*v2
 *    (layer 1 on top), over a whole level's index space (nx_l x ny_l).
 *  - `where` says whether a pointer is host memory (MLSWE_HOST) or device memory
 *    of the context's GPU (MLSWE_DEVICE).  Pointers are borrowed for the call
 *    only; device pointers are read or written in the order of the context's
 *    stream.  The library owns all of its internal device memory.
 *  - A context is used by one host thread at a time.
 *  - Time-stepping calls are asynchronous on the context's stream; calls that
 *    return host data (get_*, flag, counters, step smax) synchronise it.
 */
#ifndef MLSWE_H
#define MLSWE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MLSWE_VERSION 1

enum {
  MLSWE_OK = 0,
  MLSWE_EINVAL = -1,  /* bad argument (shape, box, level, ratio, pointer) */
  MLSWE_ENOMEM = -2,  /* device allocation failed or exceeds the configured cap */
  MLSWE_EDEVICE = -3, /* no usable GPU, or a HIP call failed */
  MLSWE_ECFL = -4,    /* observed Courant number above cfl_max in a substep */
  MLSWE_ENAN = -5,    /* non-finite state detected */
  MLSWE_ESTATE = -6   /* call order violated (e.g. stepping before set_state) */
};

enum { MLSWE_HOST = 0, MLSWE_DEVICE = 1 };
enum { MLSWE_PLAIN = 0, MLSWE_BATCHED = 1, MLSWE_GRAPH = 2, MLSWE_PER_PATCH = 3 };

typedef struct mlswe_ctx mlswe_ctx;

typedef struct mlswe_config {
  double g;           /* gravity (9.81) */
  double hdry;        /* dry tolerance: a layer is wet where its depth >= hdry */
  double kmin;        /* floor of the internal-wave hyperbolicity factor */
  double cfl_desired; /* Courant number aimed at by the dt rule (0.9) */
  double cfl_max;     /* Courant number above which a substep fails (1.0) */
  int y_rows;         /* rows per y-sweep wave (0 = chosen per level, see mlswe_tuning) */
  int x_rows;         /* rows per x-sweep wave (0 = chosen per level) */
  int64_t max_device_bytes; /* cap on the library's device memory (0 = none) */
  int max_retries;    /* a coarse step whose largest substep Courant number exceeds
                         cfl_max is undone and retaken with dt scaled by
                         cfl_desired / that number, at most this often; -1 = never
                         (the step then fails with MLSWE_ECFL), 0 = the default 8.
                         Only the problems that failed are retaken: the other
                         problems of a batched group keep their step (their
                         launches in the retake do nothing).
                         mlswe_advance in MLSWE_BATCHED, MLSWE_GRAPH and
                         MLSWE_PER_PATCH checks once per window of up to 32
                         coarse steps (and before each regrid) with no host
                         wait in between: the first failing substep halts the
                         window on the device, and the run resumes from that
                         step's retake (of every problem, as the halt stopped
                         all of them part way), with results identical to a
                         check after every step (which plain mode, dts_out,
                         kernel timing, reflux and dynamic_rt keep); after a
                         retake the windows restart from single checked steps
                         and double with each clean window */
  int reflux;         /* 1: mass flux correction at coarse-fine edges (the paper has
                         none), within mlswe_advance (mlswe_step_level and
                         mlswe_coarsen called on their own leave it out): after a
                         level's fine substeps and coarsening, each
                         coarse cell beside a fine patch has the coarse mass flux
                         through the shared face replaced by the fine fluxes summed
                         over the face's r fine faces and the fine substeps (divided
                         by r times the number of substeps),
                         so each layer's mass on the composite grid changes only by
                         clipping; 0 (default): off */
  int dynamic_rt;     /* 1: time-refinement ratios chosen per coarse step (Sec. 2,
                         text after Eq. 2) from the largest speeds of the last one:
                         level l takes the fewest substeps per substep of level
                         l - 1, at most the space ratio, that keep its substep
                         within cfl_desired of its own speeds and leave every finer
                         level able to meet its own with full ratios; in a context
                         of several problems each level takes the largest number
                         any problem needs (so all launch modes agree); the first
                         step of a problem uses the space ratios, and so does a
                         step in which a level holds patches but has no speeds of
                         the last one (a level a regrid has just populated).  0 (default):
                         time ratio = space ratio */
  int pad_;
} mlswe_config;

/* Launch shape of the two sweep kernels.  rows: rows per x-sweep wave / per
 * y-sweep wave (a y wave marches its rows with the last edge in registers);
 * 0 chooses them per level and sweep among 4-32 (x) and 8-128 (y) by a model
 * of the level's tiles finishing on the device's wave slots.  Batched launches
 * with sched 0 on levels where a problem has several patches sweep the union
 * of each problem's patches in fixed blocks; other launches sweep each patch's
 * own tiles (the results are the same bit for bit).  sched: 0 one wave per
 * tile, 1 persistent waves striding over the tile list, 2 persistent waves
 * taking tiles from an atomic ticket.
 * grid: persistent blocks of four waves per compute unit.  fast: 1 selects the
 * build of the sweeps with Newton-refined hardware reciprocals and reciprocal
 * square roots and fused multiply-adds (FP64 throughout, a few ulps per
 * operation from the default build, which reproduces the same arithmetic bit
 * for bit in every launch shape). */
typedef struct mlswe_tuning {
  int x_rows, y_rows;
  int sched_x, sched_y;
  int grid_x, grid_y;
  int fast;
} mlswe_tuning;

typedef struct mlswe_counters {
  int64_t cell_updates[8]; /* interior cells stepped, per level, summed over substeps */
  int64_t hyp;             /* edges whose internal-wave factor was clamped */
  int64_t nclip;           /* cells whose nonzero depth fell below hdry */
  int64_t repair;          /* wet-ordering repairs (top layer dry over a wet bottom layer) */
  double clip1, clip2;     /* mass removed from layers 1 and 2 by clipping */
  double t;                /* simulated time of the problem */
  int status;              /* sticky device status bits (1: Courant above cfl_max, 2: non-finite state) */
  int64_t rejected;        /* coarse steps undone and retaken (Courant above cfl_max) */
} mlswe_counters;

/* Library version (MLSWE_VERSION). */
int mlswe_version(void);

/* Message of the last error on ctx (never NULL; empty string if none). */
const char* mlswe_last_error(const mlswe_ctx* ctx);

/* Creates a context on the current HIP device using stream `hip_stream`
 * (a hipStream_t; NULL = the default stream).  cfg may be NULL for defaults.
 * Errors: MLSWE_EDEVICE if no GPU is usable, MLSWE_EINVAL for bad settings. */
int mlswe_create(const mlswe_config* cfg, void* hip_stream, mlswe_ctx** out);

/* Frees every device allocation of ctx and ctx itself. */
int mlswe_destroy(mlswe_ctx* ctx);

/* Defines a new problem (index returned in *p_out): level 0 of nx0 x ny0 cells
 * of size dx0 x dy0 with reflecting walls, nlevels levels whose spatial ratios
 * ratios[0..nlevels-2] give dx_{l+1} = dx_l / r_l and dy_{l+1} = dy_l / r_l
 * (Sec. 2, Eqs. 1-2), time ratio equal to the space ratio (Sec. 2), density
 * ratio r = rho1 / rho2 in (0, 1).  Level 0 starts as one patch over the
 * domain.  Allocates the problem's level arrays (two state buffers, an
 * intermediate buffer, bathymetry and coverage per level).
 * Errors: MLSWE_EINVAL (sizes below 2 cells -- the two mirrored ghost cells of
 * a wall need two cells --, ratios not in 2..16 or not dividing 16),
 * MLSWE_ENOMEM. */
int mlswe_problem_define(mlswe_ctx* ctx, int* p_out, double r, int nx0, int ny0, double dx0,
                         double dy0, int nlevels, const int* ratios);

/* Bathymetry samples at the cell centres of the finest level (ny_f x nx_f);
 * coarser levels hold block means, so refining the bathymetry (Sec. 2.1) is a
 * lookup.  Errors: MLSWE_EINVAL. */
int mlswe_set_bathymetry(mlswe_ctx* ctx, int p, const double* B_finest, int where);

/* Replaces the patch set of a level: n boxes {ilo, jlo, nx, ny} in the level's
 * index space, non-overlapping; on levels > 0 aligned to the level's ratio and
 * covered by the coarser level.  Level 0 must be covered completely.  New cells
 * of a level > 0 keep the value of an old patch that covered them, all others
 * are refined from the coarser level (surfaces interpolated bottom layer
 * first with minmod-limited slopes, depths recovered through the effective
 * bathymetry, wet ordering enforced: Sec. 2.1, Eqs. 3-10).
 * Errors: MLSWE_EINVAL. */
int mlswe_set_patches(mlswe_ctx* ctx, int p, int level, int n, const int32_t* boxes);

/* Copies up to cap boxes of a level into boxes (4 ints each); *n_out = count. */
int mlswe_get_patches(mlswe_ctx* ctx, int p, int level, int cap, int32_t* boxes, int* n_out);

/* Level-wide state q[6][ny_l][nx_l] into / out of the level's current buffer.
 * get_state writes NaN where no patch covers a cell (for a device destination
 * the copy is queued on the context's stream; for a host one it synchronises);
 * set_state zeroes such cells of levels > 0 (their values are never used, so a
 * get_state result can be handed back as it is).
 * Errors: MLSWE_EINVAL. */
int mlswe_set_state(mlswe_ctx* ctx, int p, int level, const double* q, int where);
int mlswe_get_state(mlswe_ctx* ctx, int p, int level, double* q, int where);

/* One substep of every patch of `level` of every problem: ghost cells (coarse
 * data at time fraction theta of the coarser level's last step, refined;
 * sibling values; walls), x-sweep, y-sweep, dry-state fix-ups, largest wave
 * speeds.  dt: host array [n_problems] of substeps, or NULL to use the
 * device-resident dt.  smax_out (nullable, host) receives [n_problems][2]
 * largest x / y speeds and synchronises.  Errors: MLSWE_EINVAL, MLSWE_ESTATE,
 * MLSWE_ENAN (a non-finite state after the x-sweep) and MLSWE_ECFL, both
 * checked only when smax_out is given. */
int mlswe_step_level(mlswe_ctx* ctx, int level, const double* dt, double theta, double* smax_out);

/* Averages the fine level onto the coarser one for all six fields (Sec. 2.2,
 * Eq. 11, divided by r_x r_y in two dimensions), then applies the dry-state
 * fix-up.  Errors: MLSWE_EINVAL. */
int mlswe_coarsen(mlswe_ctx* ctx, int p, int fine_level);

/* Refinement flags of a level (ny_l x nx_l bytes, host): cell flagged iff the top
 * layer is wet in it and its four neighbours and the centred |grad eta1| exceeds
 * tau, dilated by nbuf cells within the level's coverage.  Synchronises. */
int mlswe_flag(mlswe_ctx* ctx, int p, int level, double tau, int nbuf, uint8_t* flags_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the flags of
 * mlswe_flag, written to flags_dev (device memory of the context's GPU, ny_l x
 * nx_l bytes, caller-owned) in the order of the context's stream, without
 * synchronising and without allocating.  The undilated flags are staged in a
 * device array of MLSWE_NOALLOC_SCRATCH_BYTES that the library holds once per
 * GPU until the process ends (its address resolved by mlswe_create); every
 * call on one GPU shares it, so calls that overlap on one GPU (two streams or
 * two threads) race.  Errors: MLSWE_EINVAL (bad problem or level, nbuf < 0,
 * null flags_dev, a level of more than MLSWE_NOALLOC_SCRATCH_BYTES cells),
 * MLSWE_EDEVICE. */
#define MLSWE_NOALLOC_SCRATCH_BYTES (16ll << 20)
int mlswe_flag_noalloc(mlswe_ctx* ctx, int p, int level, double tau, int nbuf, uint8_t* flags_dev);

/* Sets the patches of fine_level (> 0) and fills them: same as set_patches. */
int mlswe_refine(mlswe_ctx* ctx, int p, int fine_level, int n, const int32_t* boxes);

/* Flag, cluster (16x16 fine tiles, kept if their coarse footprint grown by two
 * cells lies in the coarser coverage, merged row-major into rectangles of at
 * most 4x4 tiles) and refine, for levels 0..L-2 in order.  tau[l] per level. */
int mlswe_regrid(mlswe_ctx* ctx, int p, const double* tau, int nbuf);

/* n_coarse_steps subcycled coarse steps of every problem: regrid every
 * regrid_every steps (0 = never; tau is [n_problems][8]), dt from the previous
 * step's largest speeds (first step: from the state), each level l > 0 takes
 * r_{l-1} substeps per step of level l-1 and is then averaged onto it (Sec. 2).
 * The regrid treats all problems in one pass in every mode.  mode MLSWE_PLAIN
 * then steps one problem at a time and launches the sweeps per patch;
 * MLSWE_BATCHED launches one x-sweep and one y-sweep per level substep over the
 * patches of all problems;
 * MLSWE_GRAPH does the same and replays each coarse step from a captured
 * hipGraph (captured on first use, again after a regrid; the first step of a
 * run, which derives dt from the state, runs uncaptured);
 * MLSWE_PER_PATCH steps all problems together like MLSWE_BATCHED (one Courant
 * check and retake decision per coarse step for the whole group) but launches
 * the sweeps per patch, as MLSWE_PLAIN does.
 * dts_out (nullable, host [n_problems][n_coarse_steps]) receives the coarse
 * steps.  Errors: MLSWE_EINVAL, MLSWE_ESTATE, MLSWE_ECFL (Courant number above
 * cfl_max after the allowed retakes), MLSWE_ENAN (a non-finite Courant
 * number). */
int mlswe_advance(mlswe_ctx* ctx, int n_coarse_steps, int regrid_every, const double* tau, int nbuf,
                  int mode, double* dts_out);

/* Time-stepping state of problem p, for checkpoint and resume: out / in
 * [2 + 2 n_levels] holds t, 1 if the next coarse step takes its dt from the
 * largest speeds of the last one (0: from the state, as for a fresh problem),
 * and each level's largest x and y speeds over the last coarse step.  With
 * every level's patches (mlswe_set_patches, coarsest first) and state
 * (mlswe_set_state) restored into a new context, setting it continues the run
 * bit for bit (regrids fall on the same steps if the restart step is a
 * multiple of regrid_every).  In a batched advance, a problem without speeds
 * makes every problem of the batch take the next dt from its state.  Both
 * synchronise.  Errors: MLSWE_EINVAL (flag other than 0 or 1, t NaN, a speed
 * negative or not finite). */
int mlswe_get_step_state(mlswe_ctx* ctx, int p, double* out);

/* Time-refinement ratios of problem p's current (last) coarse step: out
 * [n_levels - 1], level l + 1's substeps per substep of level l (the space
 * ratios unless mlswe_config.dynamic_rt chose fewer).  Errors: MLSWE_EINVAL. */
int mlswe_get_time_ratios(mlswe_ctx* ctx, int p, int32_t* out);
int mlswe_set_step_state(mlswe_ctx* ctx, int p, const double* in);

/* Reads / sets the sweeps' launch shape (setting rebuilds the launch data). */
int mlswe_get_tuning(mlswe_ctx* ctx, mlswe_tuning* out);
int mlswe_set_tuning(mlswe_ctx* ctx, const mlswe_tuning* t);

/* Times candidate launch shapes of the x- and y-sweeps on the current patches
 * of every problem (the states are left unchanged: the sweeps write only the
 * intermediate and the spare buffer, and counters and speeds are restored),
 * keeps the fastest, and records it in the text file cache_path under a key of
 * the patch layout (nullable); a matching cache entry is applied without
 * timing.  reps: launches per candidate (0 = 3).  Synchronises. */
int mlswe_autotune(mlswe_ctx* ctx, const char* cache_path, int reps);

/* Counters of problem p (synchronises). */
int mlswe_get_counters(mlswe_ctx* ctx, int p, mlswe_counters* out);

/* Waits for all work queued on the context's stream. */
int mlswe_synchronize(mlswe_ctx* ctx);

/* Host-side synchronisation counts since the context was created: the waits
 * of the library's calls for the context's stream (advance, regrid, readbacks,
 * launch-data uploads), and the coarse-step graphs captured and replayed.  A
 * batched advance with retakes waits once per window of up to 32 coarse steps
 * and once per regrid; the Courant check of paper Sec. 2 needs no other wait.
 * Does not synchronise.  Errors: MLSWE_EINVAL (null argument). */
int mlswe_sync_counts(mlswe_ctx* ctx, int64_t* host_waits, int64_t* graph_captures, int64_t* graph_launches);

/* Kernel timing: when enabled, HIP events bracket every sweep launch on the
 * context's stream; mlswe_kernel_times returns, per kernel class (0: x-sweep,
 * 1: y-sweep), the summed milliseconds and launch counts since enabling.
 * Synchronises. */
int mlswe_set_kernel_timing(mlswe_ctx* ctx, int enable);
int mlswe_kernel_times(mlswe_ctx* ctx, double* ms_out /*[2]*/, int64_t* launches_out /*[2]*/);

/* Phase times since timing was enabled (mlswe_set_kernel_timing), per class:
 * 0 x-sweep, 1 y-sweep, 2 ghost fill, 3 substep reduction (speeds, Courant
 * check, counters), 4 coarsening, 5 flux correction, 6 dt rule (HIP events on
 * the context's stream around each launch group), 7 regrid (host wall time of
 * the regrid of all problems, its kernels and readbacks included).  Writes up
 * to cap classes of summed milliseconds and counts and returns the number of
 * classes (8).  Timing runs graph-mode advances eagerly.  Synchronises.
 * Errors: MLSWE_EINVAL. */
int mlswe_phase_times(mlswe_ctx* ctx, double* ms_out, int64_t* counts_out, int cap);

/* ---------------------------------------------------------------- adjoint
 * Differentiation of a fixed-grid run with a frozen dt sequence, for problems
 * with one level whose states keep both layers wet (the solve's reverse is the
 * transpose of its coupled branch).  A dry layer met by an adjoint step is
 * reported, without a host wait in the step itself, as MLSWE_ESTATE by a later
 * mlswe_adjoint_step of the problem or, at the latest, by
 * mlswe_param_map_adjoint, which closes the chain.  All arrays are device
 * pointers of the context's GPU in the layout of mlswe_set_state; the caller
 * owns them. */

/* n steps of problem p's level 0 with the given substeps (host array [n], read
 * before the call returns), without any host round trip. */
int mlswe_run_fixed(mlswe_ctx* ctx, int p, int n, const double* dts);

/* lam_n = (dQ_{n+1}/dQ_n)^T lam_np1 and B_bar += (dQ_{n+1}/dB)^T lam_np1 for the
 * step Q_{n+1} = S(Q_n; B, dt) of problem p (walls, x-sweep, y-sweep; the
 * dry-state fix-ups are the identity on wet states).  q_n, lam_np1, lam_n:
 * [6][ny][nx]; B_bar: [ny][nx]. */
int mlswe_adjoint_step(mlswe_ctx* ctx, int p, const double* q_n, const double* lam_np1, double* lam_n,
                       double* B_bar, double dt);

/* Initial state q [6][ny][nx] from the top surface eta1_0 [ny][nx], the
 * problem's bathymetry and a flat interface eta2_0: h2 = eta2_0 - B,
 * h1 = eta1_0 - eta2_0, at rest, thin layers dry.  And its adjoint:
 * eta1_bar = dh1 part of lam0 (written), B_bar -= dh2 part of lam0 (accumulated). */
int mlswe_param_map(mlswe_ctx* ctx, int p, const double* eta1_0, double eta2_0, double* q_out);
int mlswe_param_map_adjoint(mlswe_ctx* ctx, int p, const double* eta1_0, double eta2_0, const double* lam0,
                            double* eta1_bar, double* B_bar);

/* Gauge misfit: *loss += sum over the gn x gn cells at (i0, j0) of
 * (eta1 - target)^2 with eta1 = B + h2 + h1, from q [6][ny][nx] or, if q is
 * NULL, from the problem's current level-0 state.  If lam is not NULL its h1
 * and h2 parts get 2 (eta1 - target) added (and B_bar too if not NULL). */
int mlswe_gauge_misfit(mlswe_ctx* ctx, int p, const double* q, int i0, int j0, int gn, const double* target,
                       double* loss, double* lam, double* B_bar);

/* Branch signature for derivative checks: with enable = 1 the sweeps add, per
 * problem, a position-hashed code of every limiter branch and wave direction
 * to a 64-bit sum (enable = 0 stops, -1 leaves the setting); with sig_out not
 * NULL the sum of problem p is returned and cleared.  Two runs with equal sums
 * took the same branches (with overwhelming probability), so a finite
 * difference between them sees a smooth map.  Synchronises when reading. */
int mlswe_branch_signature(mlswe_ctx* ctx, int enable, int p, uint64_t* sig_out);

/* ---------------------------------------------------------------- M layers
 * The general multilayer refine and coarsen for M = 1..8 layers of one grid
 * (the solver itself is two-layer).  Arrays are device pointers of the
 * context's GPU, owned by the caller, field-major FP64 [3M][rows][cols] with
 * x fastest: h_m, h_m u_m, h_m v_m for layer m = 1 (top) .. M, so M = 2 is the
 * layout of mlswe_set_state.  The dry tolerance is the context's hdry.  Both
 * calls are asynchronous on the context's stream unless stated. */

/* Refine (Sec. 2.1: surfaces eta_m = B + h_M + ... + h_m, Eq. 4; effective
 * bathymetry B-hat_m = B + h_M + ... + h_{m+1}, Eq. 5; minmod slopes, Eq. 10;
 * bottom layer first, then up through B-hat; wet ordering).  Writes the fine
 * cells of the box (fi0, fj0, fnx, fny) of the fine index space of ratio r over
 * the coarse grid qc [3M][nyc][nxc] with bathymetry Bc [nyc][nxc]: qf
 * [3M][fny][fnx] from the box's fine bathymetry Bf [fny][fnx].  Each child
 * (a, b) of coarse cell (I, J) takes (eta + sx fa) + sy fb with fa = (2a + 1 -
 * r) / (2r); slopes are zero at the domain edge and for a layer dry in one of
 * the three cells of a direction; depths below hdry are dry and every layer
 * below a dry one is dry (a repair); momenta use the same interpolant and are
 * zero where the fine layer is dry.  repairs_out (nullable, host) receives the
 * number of repairs; the call then synchronises.  A box of zero cells does
 * nothing.  Errors: MLSWE_EINVAL (M or r outside 1..8, the box outside the
 * fine grid, more than 262140 coarse rows, a null array), MLSWE_EDEVICE. */
int mlswe_refine_layers(mlswe_ctx* ctx, int M, int r, const double* qc, const double* Bc, int nxc, int nyc, int fi0,
                        int fj0, int fnx, int fny, const double* Bf, double* qf, int64_t* repairs_out);

/* Coarsen (Sec. 2.2, Eq. 11 over r x r children): the coarse cells of the box
 * (ci0, cj0, cnx, cny) of the coarse grid qc [3M][nyc][nxc] become the
 * row-major sum of their children times 1/r^2 for every field, from qf
 * [3M][r cny][r cnx] (the children of the box, child (a, b) of box cell
 * (I, J) at column r I + a and row r J + b), then thin layers are dried and
 * every layer below a dry one too.  Cells of qc outside the box are left
 * as they are.  Errors: MLSWE_EINVAL (M or r outside 1..8, the box outside the
 * grid, more than 262140 rows, a null array), MLSWE_EDEVICE. */
int mlswe_coarsen_layers(mlswe_ctx* ctx, int M, int r, const double* qf, int ci0, int cj0, int cnx, int cny, double* qc,
                         int nxc, int nyc);

/* The union ("run") tiles a batched substep sweeps for one level of one
 * problem (host only, no GPU needed; for inspection and tests).  The level is
 * nx x ny cells with nbox patch boxes (ilo, jlo, nx, ny; int32, host memory,
 * as for mlswe_set_patches, unchecked beyond lying inside the level).  axis 0:
 * x-sweep blocks of 60 columns by `rows` rows counted from row -2 over the
 * patches' rows and two frame rows on each side; axis 1: y-sweep blocks of 64
 * columns by `rows` interior rows.  Writes up to cap tiles of five int32 each
 * to out: i0, ncols, j0, nrows, flags (bit 0: the tile owns the edge after its
 * last column (x) or row (y)), in launch order, and returns the number of
 * tiles (which may exceed cap), or MLSWE_EINVAL. */
int mlswe_run_tiles(int nx, int ny, int nbox, const int32_t* boxes, int axis, int rows, int32_t* out, int cap);

#ifdef __cplusplus
}
#endif
#endif /* MLSWE_H */
