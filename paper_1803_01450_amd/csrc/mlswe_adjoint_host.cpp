// Entry points of the fixed-grid adjoint: stepping with given substeps, the
// adjoint step, the parameter map and the gauge misfit.
#include "mlswe_host.hpp"

// ------------------------------------------------------------ adjoint
static int ensure_adj(mlswe_ctx* c, ProblemH& P) {
  AdjBuf& A = P.adj;
  if (A.lamS) return MLSWE_OK;
  const LevelH& L = P.L[0];
  const size_t pb = sizeof(double) * (size_t)L.plane;
  int rc;
  if ((rc = dalloc(c, (void**)&A.lamS, 6 * pb)) ||
      (rc = dalloc(c, (void**)&A.lamG, 6 * pb)) || (rc = dalloc(c, (void**)&A.Bbx, pb)) ||
      (rc = dalloc(c, (void**)&A.Bby, pb)) || (rc = dalloc(c, (void**)&A.status, sizeof(int))))
    return rc;
  HIPCHK(c, hipMemsetAsync(A.lamS, 0, 6 * pb, c->stream));
  HIPCHK(c, hipMemsetAsync(A.lamG, 0, 6 * pb, c->stream));
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
    c->dt_ctl = c->ctl + P.ctl0;  // stored by the step's fill launch
    c->dt_value = dts[k];
    rc = substep(c, 0, p, p + 1, 0.0, false);
    c->dt_ctl = nullptr;
    if (rc) return rc;
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
  if ((rc = build_launch(c, 0))) return rc;
  c->dt_ctl = c->ctl + P.ctl0;  // stored by the fill launch
  c->dt_value = dt;
  rc = launch_fill(c, 0, p, p + 1, 0.0);
  c->dt_ctl = nullptr;
  if (rc) return rc;
  LevelLaunch& LL = c->launch[0];
  int k0 = -1;
  for (int k = 0; k < LL.nptch; ++k)
    if (LL.patch_prob[k] == p) { k0 = k; break; }
  if (k0 < 0) return fail(c, MLSWE_ESTATE, "problem %d has no patch", p);
  if ((rc = launch_sweeps(c, 0, L.cur, LL.xr[k0].first, LL.xr[k0].second, 0, 0))) return rc;
  AdjView V;
  std::memset(&V, 0, sizeof V);
  V.B = L.B; V.plane = L.plane; V.P = P.P; V.status = A.status;
  // y-sweep lines: columns, cells along rows
  // (the adjoint of the step's output is read where the caller holds it, [6][ny][nx])
  V.q = L.qs; V.lam = lam_np1;
  V.lstride = 1; V.kstride = L.pitch; V.base = idx(L, 0, 0);
  V.lplane = (long long)L.nx * L.ny; V.lbase = 0; V.llstride = 1; V.lkstride = L.nx;
  V.nlines = L.nx; V.n = L.ny; V.orient = 1; V.nu = dt / L.dy;
  {
    // a block per 4 columns and 61 cells (k_adj_edges_col), in eight XCD bands
    const long long tiles = ((L.nx + 3) / 4) * (long long)((L.ny + 4 + 60) / 61);
    hipLaunchKernelGGL(k_adj_edges_col, dim3((unsigned)(8 * ((tiles + 7) / 8))), dim3(256), 0, c->stream, V, A.lamS,
                       A.Bby);
  }
  // x-sweep lines: rows -2..ny+1 of the wall-filled state, cells along x
  V.q = L.q[L.cur]; V.lam = A.lamS;
  V.lstride = L.pitch; V.kstride = 1; V.base = idx(L, 0, -2);
  V.lplane = L.plane; V.lbase = V.base; V.llstride = V.lstride; V.lkstride = V.kstride;
  V.nlines = L.ny + 4; V.n = L.nx; V.orient = 0; V.nu = dt / L.dx;
  {
    // one wave per 61 cells of a row (k_adj_edges_row), four waves a block
    const long long waves = (long long)(L.ny + 4) * ((L.nx + 4 + 60) / 61);
    hipLaunchKernelGGL(k_adj_edges_row, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, c->stream, V, A.lamG,
                       A.Bbx);
  }
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
    HIPCHK(c, host_wait(c));
    *sig_out = h.sig;
    h.sig = 0;
    HIPCHK(c, hipMemcpyAsync(c->cnt + c->probs[p].cnt, &h, sizeof h, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, host_wait(c));
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
    HIPCHK(c, host_wait(c));
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
