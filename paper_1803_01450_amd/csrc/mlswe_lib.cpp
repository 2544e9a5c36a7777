// Host side of the MI355X two-layer shallow-water AMR library: contexts,
// problems, dense per-level device arrays and their state, behind the C
// ABI of include/mlswe.h.
#include "mlswe_host.hpp"

namespace mlswe_host {

int fail(mlswe_ctx* c, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return code;
}

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
  if (where != MLSWE_DEVICE) HIPCHK(c, host_wait(c));
  return MLSWE_OK;
}

}  // namespace mlswe_host

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
  if (dalloc(c, (void**)&c->halt, HALT_WORDS * sizeof(unsigned)) != MLSWE_OK ||
      hipMemsetAsync(c->halt, 0, HALT_WORDS * sizeof(unsigned), c->stream) != hipSuccess) {
    dfree(c->tickets);
    dfree(c->halt);
    delete c;
    return MLSWE_ENOMEM;
  }
  if (scratch_setup(c) != MLSWE_OK) {
    dfree(c->tickets);
    dfree(c->halt);
    delete c;
    return MLSWE_EDEVICE;
  }
  *out = c;
  return MLSWE_OK;
}

int mlswe_destroy(mlswe_ctx* c) {
  if (!c) return MLSWE_EINVAL;
  (void)host_wait(c);
  for (ProblemH& P : c->probs) {
    dfree(P.adj.lamS); dfree(P.adj.lamG);
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
    dfree(LL.red);
    for (int k = 0; k < 4; ++k) { dfree(LL.fp[k]); dfree(LL.cp[k]); }
    dfree(LL.rfx); dfree(LL.rfx_reg);
  }
  dfree(c->ctl); dfree(c->cnt); dfree(c->pdt); dfree(c->spd); dfree(c->dt_stage);
  dfree(c->tickets); dfree(c->halt); dfree(c->skip); dfree(c->fail_d); dfree(c->ctl_bk); dfree(c->cnt_bk); dfree(c->dt0_d);
  dfree(c->bsegs_d); dfree(c->mboxes_d); dfree(c->rfills_d); dfree(c->flv_d);
  for (auto& bl : c->box_lists) dfree(bl.d);
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
    if (ccap > c->skip_cap) {
      unsigned* ns = nullptr;
      if ((rc = dalloc(c, (void**)&ns, sizeof(unsigned) * ccap))) return rc;
      HIPCHK(c, hipMemsetAsync(ns, 0, sizeof(unsigned) * ccap, c->stream));
      dfree(c->skip);
      c->skip = ns;
      c->skip_cap = ccap;
    }
    HIPCHK(c, hipMemsetAsync(nc, 0, sizeof(LevelCtl) * ncap, c->stream));
    HIPCHK(c, hipMemsetAsync(ncn, 0, sizeof(Counters) * ccap, c->stream));
    if (c->ctl) HIPCHK(c, hipMemcpyAsync(nc, c->ctl, sizeof(LevelCtl) * nctl, hipMemcpyDeviceToDevice, c->stream));
    if (c->cnt) HIPCHK(c, hipMemcpyAsync(ncn, c->cnt, sizeof(Counters) * pidx, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, host_wait(c));
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
    HIPCHK(c, host_wait(c));
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
  HIPCHK(c, host_wait(c));
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
  HIPCHK(c, host_wait(c));
  h[0].t = in[0];
  for (int l = 0; l < P.nlev; ++l) {
    h[l].acc_smax[0] = (unsigned long long)__builtin_bit_cast(long long, in[2 + 2 * l]);
    h[l].acc_smax[1] = (unsigned long long)__builtin_bit_cast(long long, in[3 + 2 * l]);
  }
  HIPCHK(c, hipMemcpyAsync(c->ctl + P.ctl0, h.data(), sizeof(LevelCtl) * h.size(), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, host_wait(c));
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
    HIPCHK(c, host_wait(c));
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
  HIPCHK(c, host_wait(c));
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
    HIPCHK(c, host_wait(c));
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
