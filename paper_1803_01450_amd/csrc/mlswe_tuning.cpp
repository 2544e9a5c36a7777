// Launch-shape tuning: get, set and the autotuner with its cache.
#include "mlswe_host.hpp"

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
  HIPCHK(c, host_wait(c));
  HIPCHK(c, hipMemcpy(ctl_save.data(), c->ctl, sizeof(LevelCtl) * nctl, hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(cnt_save.data(), c->cnt, sizeof(Counters) * ncnt, hipMemcpyDeviceToHost));
  const int scheds[5][2] = {{0, 0}, {1, 1}, {1, 2}, {2, 1}, {2, 2}};
  mlswe_tuning best = c->tune;
  int rc = MLSWE_OK;
  for (int axis = 0; axis < 2 && !rc; ++axis) {
    // 0: the per-level choice made when the tiles are built
    const int rows_x[6] = {0, 2, 4, 8, 16, 32};
    const int rows_y[8] = {0, 4, 8, 16, 32, 64, 128, 256};
    const int nrows = axis == 0 ? 6 : 8;
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
  HIPCHK(c, host_wait(c));
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
