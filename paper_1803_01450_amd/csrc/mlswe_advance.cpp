// Coarse steps: the dt rule and time ratios, the subcycled recursion, graph
// capture and replay, backups and retakes, and mlswe_advance with the
// counters and timing entry points.
#include "mlswe_host.hpp"

namespace mlswe_host {

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
// of its finer levels and the control blocks and counters of its problems, in
// one launch (a problem whose skip flag is set is left as it is).
int copy_step_start(mlswe_ctx* c, int p0, int p1, bool to_bk, bool mark) {
  // the list depends on the launch data (generation), the direction and the
  // buffer parity of every level: built and uploaded once per combination
  std::vector<char> cur;
  for (int p = p0; p < p1; ++p)
    for (int l = 1; l < c->probs[p].nlev; ++l) cur.push_back((char)c->probs[p].L[l].cur);
  for (auto it = c->box_lists.begin(); it != c->box_lists.end();) {
    if (it->gen != c->generation) {
      dfree(it->d);
      it = c->box_lists.erase(it);
    } else {
      ++it;
    }
  }
  mlswe_ctx::BoxList* hit = nullptr;
  for (auto& b : c->box_lists)
    if (b.to_bk == to_bk && b.p0 == p0 && b.p1 == p1 && b.cur == cur) hit = &b;
  if (!hit) {
    std::vector<CopyBox> boxes;
    long long longest = 0;
    // every box carries its problem's skip flag: a retake restores only the
    // problems it takes again
    const unsigned* sk = nullptr;
    auto add = [&](const double* from, double* to, long long pitch, long long plane, int nx, int ny, int nf) {
      boxes.push_back(CopyBox{from, to, pitch, plane, nx, ny, nf, 0, sk});
      longest = std::max(longest, (long long)nx * ny * nf);
    };
    auto run = [&](double* live, double* saved, long long n) {
      if (n > 0) add(to_bk ? live : saved, to_bk ? saved : live, 0, 0, (int)n, 1, 1);
    };
    static_assert(sizeof(LevelCtl) % sizeof(double) == 0 && sizeof(Counters) % sizeof(double) == 0,
                  "copied as doubles");
    for (int p = p0; p < p1; ++p) {
      ProblemH& P = c->probs[p];
      sk = c->skip + p;
      constexpr long long wc = (long long)(sizeof(LevelCtl) / sizeof(double));
      constexpr long long wn = (long long)(sizeof(Counters) / sizeof(double));
      run((double*)(c->ctl + P.ctl0), (double*)(c->ctl_bk + P.ctl0), P.nlev * wc);
      run((double*)(c->cnt + P.cnt), (double*)(c->cnt_bk + P.cnt), wn);
    }
    for (int p = p0; p < p1; ++p) {
      ProblemH& P = c->probs[p];
      sk = c->skip + p;
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
    if (c->box_lists.size() >= 32) {  // a bound on the cache: drop the oldest
      HIPCHK(c, host_wait(c));
      dfree(c->box_lists.front().d);
      c->box_lists.erase(c->box_lists.begin());
    }
    mlswe_ctx::BoxList bl;
    bl.to_bk = to_bk; bl.cur = cur; bl.gen = c->generation; bl.p0 = p0; bl.p1 = p1; bl.d = nullptr;
    bl.n = (int)boxes.size(); bl.longest = longest;
    int rc;
    if ((rc = dalloc(c, (void**)&bl.d, sizeof(CopyBox) * boxes.size()))) return rc;
    HIPCHK(c, hipMemcpyAsync(bl.d, boxes.data(), sizeof(CopyBox) * boxes.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, host_wait(c));  // the host vector goes out of scope
    c->box_lists.push_back(bl);
    hit = &c->box_lists.back();
  }
  const unsigned gx = (unsigned)std::min<long long>(64, (hit->longest + 4095) / 4096);
  const int nboxes = hit->n;
  CopyBox* boxes_d = hit->d;
  // backups skip once a deferred window has halted (and the first launch counts
  // the backup); restores always run
  for (int k0 = 0; k0 < nboxes; k0 += 65535)  // grid y is at most 65535
    hipLaunchKernelGGL(k_copy_boxes, dim3(gx, (unsigned)std::min(65535, nboxes - k0)), dim3(256), 0, c->stream,
                       boxes_d + k0, to_bk ? c->halt : nullptr, (mark && k0 == 0) ? 1 : 0);
  HIPCHK(c, hipGetLastError());
  return MLSWE_OK;
}

// Host bookkeeping of a coarse step's start: buffer parity and update count of
// every level of every problem of a group, problem-major.
struct StepMark {
  std::vector<int> cur;
  std::vector<long long> upd;
};

// Records the group's step start and makes sure its backup arrays exist.
int mark_step(mlswe_ctx* c, int p0, int p1, int nctl, int ncnt, StepMark& m) {
  int rc;
  if ((rc = ensure(c, &c->ctl_bk, &c->bk_cap, nctl))) return rc;
  if ((rc = ensure(c, &c->cnt_bk, &c->cbk_cap, ncnt))) return rc;
  m.cur.clear();
  m.upd.clear();
  for (int p = p0; p < p1; ++p) {
    ProblemH& P = c->probs[p];
    for (int l = 0; l < P.nlev; ++l) {
      LevelH& L = P.L[l];
      m.cur.push_back(L.cur);
      m.upd.push_back(P.updates[l]);
      if (l == 0 || L.boxes.empty()) continue;
      const size_t sb = sizeof(double) * 6 * (size_t)L.plane;
      if (!L.bk && (rc = dalloc(c, (void**)&L.bk, sb))) return rc;
    }
  }
  return MLSWE_OK;
}

// The group's coarse step itself: replayed from a graph, or launched.
int run_step(mlswe_ctx* c, int p0, int p1, int mode) {
  const bool together = mode == MLSWE_BATCHED || mode == MLSWE_GRAPH;
  bool all_dt = true;
  for (int p = p0; p < p1; ++p) all_dt = all_dt && c->probs[p].have_dt;
  if (mode == MLSWE_GRAPH && all_dt && !c->timing) return graph_step(c, p0, p1);
  return coarse_step(c, p0, p1, together);
}

// The control blocks of every problem in pinned memory, and (want_halt) the
// halt words after them, in one synchronised copy each.
int read_controls(mlswe_ctx* c, int nctl, bool want_halt, const LevelCtl** h, const unsigned** hw) {
  const size_t need = (size_t)nctl * sizeof(LevelCtl) + 64;
  if (need > c->ctl_pin_cap) {
    if (c->ctl_pin) (void)hipHostFree(c->ctl_pin);
    c->ctl_pin = nullptr;
    c->ctl_pin_cap = 0;
    HIPCHK(c, hipHostMalloc((void**)&c->ctl_pin, 2 * need, hipHostMallocDefault));
    c->ctl_pin_cap = 2 * need;
  }
  unsigned* words = (unsigned*)((char*)c->ctl_pin + (size_t)nctl * sizeof(LevelCtl));
  HIPCHK(c, hipMemcpyAsync(c->ctl_pin, c->ctl, sizeof(LevelCtl) * nctl, hipMemcpyDeviceToHost, c->stream));
  if (want_halt)
    HIPCHK(c, hipMemcpyAsync(words, c->halt, HALT_WORDS * sizeof(unsigned), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, host_wait(c));
  *h = c->ctl_pin;
  if (hw) *hw = words;
  return MLSWE_OK;
}

// From the control blocks after a step: each problem's largest substep Courant
// number; a problem above cfl_max gets dt scaled by cfl_desired / that number
// for its retake, the others keep theirs.  MLSWE_ENAN on a non-finite state.
int judge(mlswe_ctx* c, int p0, int p1, const LevelCtl* h, std::vector<double>& dt0, bool* any,
          std::vector<unsigned char>* failing) {
  *any = false;
  dt0.assign((size_t)(p1 - p0), 0.0);
  if (failing) failing->assign((size_t)(p1 - p0), 0);
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
    if (nan) return fail(c, MLSWE_ENAN, "non-finite state or Courant number in problem %d", p);
    if (cm > c->cfg.cfl_max) {
      *any = true;
      if (failing) (*failing)[p - p0] = 1;
      dt0[p - p0] = dtp * (c->cfg.cfl_desired / cm);
    } else {
      dt0[p - p0] = dtp;
    }
  }
  return MLSWE_OK;
}

void accept_step(mlswe_ctx* c, int p0, int p1, const LevelCtl* h) {
  for (int p = p0; p < p1; ++p) {
    ProblemH& P = c->probs[p];
    for (int l = 0; l < P.nlev; ++l) {
      P.last_acc[l][0] = h[P.ctl0 + l].acc_smax[0];
      P.last_acc[l][1] = h[P.ctl0 + l].acc_smax[1];
    }
    P.acc_known = true;
  }
}

// Retakes a rejected coarse step: the problems marked in rerun (those whose
// Courant number exceeded cfl_max, or the whole group when a deferred window
// stopped its step part way) are put back to the step's start m (patch
// interiors, controls and counters from the backup) and stepped again with
// dt0, while every other problem of the group is left alone through its skip
// flag (its launches do nothing, its buffers keep the accepted step, and the
// host bookkeeping replays the same parity flips and counts); failing marks
// the problems whose step is counted as rejected.  Checked after each attempt
// until it passes or max_retries retakes are spent.
int retake(mlswe_ctx* c, int p0, int p1, bool together, const StepMark& m, std::vector<double> dt0, int nctl,
           int ncnt, std::vector<unsigned char> rerun, std::vector<unsigned char> failing) {
  int rc;
  const int np = p1 - p0;
  // the skip flags are cleared whatever the outcome
  struct Clear {
    mlswe_ctx* c;
    int p0, np;
    ~Clear() { hipLaunchKernelGGL(k_set_skip, dim3((np + 63) / 64), dim3(64), 0, c->stream, c->skip + p0, nullptr, np); }
  } clear{c, p0, np};
  for (int attempt = 1;; ++attempt) {
    if (attempt > c->cfg.max_retries) return fail(c, MLSWE_ECFL, "Courant number above %g", c->cfg.cfl_max);
    size_t k = 0;
    for (int p = p0; p < p1; ++p) {
      ProblemH& P = c->probs[p];
      if (failing[p - p0]) P.rejected++;
      for (int l = 0; l < P.nlev; ++l, ++k) {
        P.L[l].cur = m.cur[k];
        P.updates[l] = m.upd[k];
      }
    }
    if ((rc = ensure(c, &c->fail_d, &c->fail_cap, np))) return rc;
    HIPCHK(c, hipMemcpyAsync(c->fail_d, rerun.data(), (size_t)np, hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL(k_set_skip, dim3((np + 63) / 64), dim3(64), 0, c->stream, c->skip + p0, c->fail_d, np);
    if ((rc = copy_step_start(c, p0, p1, false, false))) return rc;
    if ((rc = ensure(c, &c->dt0_d, &c->dt0_cap, np))) return rc;
    HIPCHK(c, hipMemcpyAsync(c->dt0_d, dt0.data(), sizeof(double) * np, hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL(k_set_dt0, dim3((np + 63) / 64), dim3(64), 0, c->stream, c->ctl, c->pdt + p0, c->dt0_d, np,
                       c->skip + p0);
    HIPCHK(c, hipGetLastError());
    if ((rc = adv(c, 0, p0, p1, 0.0, together))) return rc;
    const LevelCtl* h = nullptr;
    if ((rc = read_controls(c, nctl, false, &h, nullptr))) return rc;
    bool any = false;
    std::vector<unsigned char> again;
    if ((rc = judge(c, p0, p1, h, dt0, &any, &again))) return rc;
    if (!any) {
      accept_step(c, p0, p1, h);
      return MLSWE_OK;
    }
    failing = again;
    rerun = again;
  }
}

void counts(const mlswe_ctx* c, int* nctl, int* ncnt) {
  *nctl = 0;
  for (const ProblemH& P : c->probs) *nctl += P.nlev;
  *ncnt = (int)c->probs.size();
}

// A coarse step of problems [p0, p1) with rejection: when the largest substep
// Courant number of a problem exceeds cfl_max, that problem is put back
// (fine-level patch interiors, controls, counters; level 0 keeps its input
// buffer through a step) and retaken with dt scaled by cfl_desired / that
// number, while the group's other problems keep their step (retake).  Frames
// and uncovered cells of the finer levels are refilled or unused before they
// are read again, so the backup leaves them out.  The check waits for the step
// (one host round trip per coarse step); retaken reports whether a retake ran.
int step_with_retry(mlswe_ctx* c, int p0, int p1, int mode, bool* retaken) {
  int rc;
  if (retaken) *retaken = false;
  const bool together = mode == MLSWE_BATCHED || mode == MLSWE_GRAPH;
  if (c->cfg.max_retries <= 0) return run_step(c, p0, p1, mode);
  int nctl, ncnt;
  counts(c, &nctl, &ncnt);
  StepMark m;
  if ((rc = mark_step(c, p0, p1, nctl, ncnt, m))) return rc;
  if ((rc = copy_step_start(c, p0, p1, true, false))) return rc;
  if ((rc = run_step(c, p0, p1, mode))) return rc;
  const LevelCtl* h = nullptr;
  if ((rc = read_controls(c, nctl, false, &h, nullptr))) return rc;
  std::vector<double> dt0;
  std::vector<unsigned char> failing;
  bool any = false;
  if ((rc = judge(c, p0, p1, h, dt0, &any, &failing))) return rc;
  if (!any) {
    accept_step(c, p0, p1, h);
    return MLSWE_OK;
  }
  if (retaken) *retaken = true;
  return retake(c, p0, p1, together, m, dt0, nctl, ncnt, failing, failing);
}

// Deferred checks: the steps of a window run back to back with no host wait.
// Each takes its backup and counts it; the substep reduction that first finds
// a Courant number above the limit halts the window, after which the backups,
// outputs, coarsening, dt rule and reductions of the following kernels do
// nothing.  One readback at the window's end either accepts every step or
// finds the first failing one (the backup holds its start), puts the group
// back there and retakes it as step_with_retry does; the steps after it are
// then run again.  Results are those of step_with_retry bit for bit.
int deferred_step(mlswe_ctx* c, int mode, std::vector<StepMark>& win) {
  int rc;
  const int np = (int)c->probs.size();
  int nctl, ncnt;
  counts(c, &nctl, &ncnt);
  if (win.empty()) {
    hipLaunchKernelGGL(k_set_halt, dim3(1), dim3(64), 0, c->stream, c->halt, 1u);
    HIPCHK(c, hipGetLastError());
    c->armed = true;
  }
  win.emplace_back();
  if ((rc = mark_step(c, 0, np, nctl, ncnt, win.back()))) return rc;
  if ((rc = copy_step_start(c, 0, np, true, true))) return rc;
  return run_step(c, 0, np, mode);
}

int disarm(mlswe_ctx* c) {
  if (!c->armed) return MLSWE_OK;
  c->armed = false;
  hipLaunchKernelGGL(k_set_halt, dim3(1), dim3(64), 0, c->stream, c->halt, 0u);
  HIPCHK(c, hipGetLastError());
  return MLSWE_OK;
}

// kept: how many of the window's steps stand once it is checked (all, or up to
// and including the retaken first failure).
int verify_window(mlswe_ctx* c, int mode, std::vector<StepMark>& win, int* kept, bool* retook) {
  int rc;
  const int np = (int)c->probs.size();
  const bool together = mode == MLSWE_BATCHED || mode == MLSWE_GRAPH;
  int nctl, ncnt;
  counts(c, &nctl, &ncnt);
  const LevelCtl* h = nullptr;
  const unsigned* hw = nullptr;
  if ((rc = read_controls(c, nctl, true, &h, &hw))) return rc;
  const bool halted = hw[HALT_SET] != 0;
  const int f = (int)hw[HALT_MARKS] - 1;
  if ((rc = disarm(c))) return rc;
  std::vector<double> dt0;
  bool any = false;
  std::vector<unsigned char> failing;
  if ((rc = judge(c, 0, np, h, dt0, &any, &failing))) return rc;
  *retook = halted;
  if (!halted) {
    if (any) return fail(c, MLSWE_ESTATE, "deferred check: a failing step did not halt its window");
    accept_step(c, 0, np, h);
    *kept = (int)win.size();
    return MLSWE_OK;
  }
  if (!any || f < 0 || f >= (int)win.size())
    return fail(c, MLSWE_ESTATE, "deferred check: halted window without a failing step");
  // the halt stopped every problem's step part way: all of them are taken again
  std::vector<unsigned char> all((size_t)np, 1);
  if ((rc = retake(c, 0, np, together, win[f], dt0, nctl, ncnt, all, failing))) return rc;
  *kept = f + 1;
  return MLSWE_OK;
}

}  // namespace mlswe_host

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
  // batched, graph and per-patch steps with retakes check the Courant number
  // once per window of up to 32 coarse steps (and before every regrid) instead
  // of after every step; per-step readbacks (dts_out, timing, the dynamic time
  // ratio's speeds) and the flux correction keep the per-step check
  const bool defer = together && c->cfg.max_retries > 0 && !dts_out && !c->timing && !c->cfg.reflux &&
                     !c->cfg.dynamic_rt;
  // window length: 32 coarse steps, down to single checked steps after a
  // retake (a halted window takes every problem again, a checked step only
  // the failing ones), then doubling after each clean window
  constexpr int WINDOW = 32;
  int W = WINDOW;
  std::vector<StepMark> win;
  struct Guard {
    mlswe_ctx* c;
    ~Guard() { (void)disarm(c); }
  } guard{c};
  int n = 0;
  while (n < nsteps) {
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
    if (defer && (W > 1 || !win.empty())) {
      if ((rc = deferred_step(c, mode, win))) return rc;
      ++n;
      if ((int)win.size() >= W || n == nsteps || (regrid_every > 0 && n % regrid_every == 0)) {
        int kept = 0;
        bool retook = false;
        if ((rc = verify_window(c, mode, win, &kept, &retook))) return rc;
        const bool clean = !retook;
        n -= (int)win.size() - kept;
        win.clear();
        W = clean ? std::min(WINDOW, 2 * W) : 1;
      }
      continue;
    }
    bool retaken = false;
    for (int gi = 0; gi < ngroups; ++gi) {
      const int p0 = together ? 0 : gi, p1 = together ? np : gi + 1;
      bool r = false;
      if ((rc = step_with_retry(c, p0, p1, mode, &r))) return rc;
      retaken = retaken || r;
    }
    if (defer) W = retaken ? 1 : 2;
    if (dts_out || c->timing) {
      if ((rc = collect_events(c))) return rc;
    }
    if (dts_out) {
      std::vector<LevelCtl> h;
      if ((rc = read_ctls(c, 0, np, h))) return rc;
      for (int p = 0; p < np; ++p) dts_out[(size_t)p * nsteps + n] = h[c->probs[p].ctl0].dt;
    }
    ++n;
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
  HIPCHK(c, host_wait(c));
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
  HIPCHK(c, host_wait(c));
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

int mlswe_sync_counts(mlswe_ctx* c, int64_t* host_waits, int64_t* graph_captures, int64_t* graph_launches) {
  if (!c || !host_waits || !graph_captures || !graph_launches) return MLSWE_EINVAL;
  *host_waits = c->host_waits;
  *graph_captures = c->graph_captures;
  *graph_launches = c->graph_launches;
  return MLSWE_OK;
}

}  // extern "C"
