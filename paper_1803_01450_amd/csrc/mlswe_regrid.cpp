// Patches, coverage masks, flags, clustering and regridding.
#include "mlswe_host.hpp"

namespace mlswe_host {

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

// ------------------------------------------------------------ patches
int upload_mask(mlswe_ctx* c, LevelH& L) {
  host_mask(L);
  HIPCHK(c, hipMemcpyAsync(L.mask, L.mask_h.data(), L.mask_h.size(), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, host_wait(c));
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
    hipError_t s = host_wait(c);
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
  HIPCHK(c, host_wait(c));
  return MLSWE_OK;
}

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
      HIPCHK(c, host_wait(c));
      if (c->pin) (void)hipHostFree(c->pin);
      c->pin = nullptr;
      c->pin_cap = 0;
      HIPCHK(c, hipHostMalloc((void**)&c->pin, total, hipHostMallocDefault));
      c->pin_cap = total;
    }
    HIPCHK(c, hipMemcpyAsync(c->pin, c->tbits_d, total, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, host_wait(c));
    // host: clusters, then the new layouts
    std::vector<std::vector<Box>> nbs(who.size());
    for (size_t k = 0; k < who.size(); ++k) {
      const LevelH& F = c->probs[who[k]].L[l + 1];
      nbs[k] = cluster_tiles(F.nx, F.ny, c->pin + off[k]);
    }
    std::vector<ByteSeg> keep, clear;
    std::vector<MaskBox>& mb = c->rg_boxes;
    std::vector<FillPatch>& fills = c->rg_fills;
    mb.clear();
    fills.clear();
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
    std::vector<ByteSeg>& both = c->rg_segs;
    both.assign(keep.begin(), keep.end());
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
    // no wait here: the copies' host sides live in the context until the next
    // level's flag readback has drained the stream
  }
  return MLSWE_OK;
}

}  // namespace mlswe_host
