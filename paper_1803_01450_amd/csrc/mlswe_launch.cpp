// Launch data of a level (tiles of patches and unions, fill, coarsen and
// reduction descriptors, tile heights), kernel timing, and the launches of
// a level substep, coarsening and the dt rule.
#include "mlswe_host.hpp"

namespace mlswe_host {

// ------------------------------------------------------------ launch data
// Run tiles of one level of one problem: fixed blocks over the union of its
// patches, x blocks of XTILE_COLS columns by `rows` rows counted from row -2
// (the patches' rows and two frame rows on each side), y blocks of 64 columns
// by `rows` interior rows.  A block is kept where a patch region meets it; bit
// 0 of flags (x) / last (y) marks a block whose successor to the right (x) or
// above (y) is not kept, so that it owns the edge after its last column / row.
// Returns the number of blocks kept; appends tiles when the vectors are given.
long long run_blocks(const LevelH& L, int axis, int rows, int pdi, std::vector<XTile>* xo, std::vector<YTile>* yo,
                     std::vector<int>* rows_out) {
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
            R.skip = c->skip + p;
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
  // The last candidate (2 rows for x, 4 for y) serves small levels only: it
  // is weighed when the one before it leaves some SIMD without a tile, so
  // that a few waves do not each run a long serial chain of rows on an idle
  // chip (on fuller levels its extra halo and start work would cost more).
  const int xc[5] = {32, 16, 8, 4, 2}, yc[6] = {128, 64, 32, 16, 8, 4};
  auto pick = [&](int axis, int tuned, const std::function<void(int, std::vector<int>&)>& rows_of) {
    if (tuned > 0) return tuned;
    const int* cand = axis == 0 ? xc : yc;
    const int nc = axis == 0 ? 5 : 6;
    const long long slots = (axis == 0 ? 24LL : 16LL) * c->ncu;
    long long best = -1;
    int br = cand[0];
    std::vector<int> d;
    size_t prev_tiles = 0;
    for (int k = 0; k < nc; ++k) {
      d.clear();
      rows_of(cand[k], d);
      if (k == nc - 1 && (long long)prev_tiles >= 4LL * c->ncu) break;
      prev_tiles = d.size();
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
    info.ctl = P.ctl0 + l; info.cnt = P.cnt; info.prob = (int)pi; info.dx = L.dx; info.dy = L.dy;
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
        d.halt = c->halt;
        d.skip = c->skip + pi;
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
      f.skip = c->skip + pi;
      CoarsenPatch cc;
      std::memset(&cc, 0, sizeof cc);
      cc.skip = c->skip + pi;
      const LevelH* Cl = l > 0 ? &P.L[l - 1] : nullptr;
      if (Cl) {
        f.Bc = Cl->B;
        f.cpitch = Cl->pitch; f.cplane = Cl->plane; f.ncx = Cl->nx; f.ncy = Cl->ny;
        f.r = P.ratio[l - 1];
        f.coarse_none = 0;
        cc.fpitch = L.pitch; cc.fplane = L.plane; cc.cpitch = Cl->pitch; cc.cplane = Cl->plane;
        cc.ilo = b.ilo; cc.jlo = b.jlo; cc.bnx = b.nx; cc.bny = b.ny; cc.r = P.ratio[l - 1];
        cc.P = P.P;
        cc.halt = c->halt;
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
  // slice results of the partial reduction (one block per problem, or up to 32
  // per problem when a problem has many tiles)
  if ((rc = ensure(c, &LL.red, &LL.cap_red, AFTER_MAX_SLICES * std::max(1, LL.nli)))) return rc;
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
  HIPCHK(c, host_wait(c));
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
  HIPCHK(c, host_wait(c));
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
  HIPCHK(c, host_wait(c));
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

// ------------------------------------------------------------ launches
// Sweeps over tile ranges of level l; rx / ry: the ranges are run tiles.
int launch_sweeps(mlswe_ctx* c, int l, int parity, int xt0, int nxt, int yt0, int nyt, bool rx,
                  bool ry) {
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
  // the lean kernels: LEAN_WAVES waves (tiles) per block
  const dim3 lean_block(64 * LEAN_WAVES);
  auto lean_grid = [&](int ntiles) { return dim3((unsigned)(((ntiles + LEAN_WAVES - 1) / LEAN_WAVES + 7) / 8 * 8)); };
  if ((sx == 2 && nxt > 0) || (sy == 2 && nyt > 0))
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, c->stream, c->tickets, 2);
  if (nxt > 0) {
    if (c->timing && (rc = ev_begin(c, &e0))) return rc;
    if (rx)
      hipLaunchKernelGGL(c->tune.fast ? k_sweep_xr_fast : k_sweep_xr, lean_grid(nxt), lean_block, 0,
                         c->stream, LL.pd[parity], LL.xt + xt0, nxt, LL.parts + xt0);
    else if (sx == 0 && !c->sig_on)  // one wave per tile, no signature: the lean kernels
      hipLaunchKernelGGL(c->tune.fast ? k_sweep_x1_fast : k_sweep_x1, lean_grid(nxt), lean_block, 0,
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
      hipLaunchKernelGGL(c->tune.fast ? k_sweep_yr_fast : k_sweep_yr, lean_grid(nyt), lean_block, 0,
                         c->stream, LL.pd[parity], LL.yt + yt0, nyt, LL.parts + LL.nxt + yt0);
    else if (sy == 0 && !c->sig_on)
      hipLaunchKernelGGL(c->tune.fast ? k_sweep_y1_fast : k_sweep_y1, lean_grid(nyt), lean_block, 0,
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
  // a time step handed over by the fixed-grid calls rides on the first fill
  // launch (or gets a launch of its own when no fill runs)
  LevelCtl* dt_ctl = c->dt_ctl;
  const double dt = c->dt_value;
  c->dt_ctl = nullptr;
  if (count > 0) {
    const FillPatch* f = LL.fp[fpar * 2 + cpar] + first;
    if (l > 0) {
      hipLaunchKernelGGL(k_ghost_fill, dim3((maxring + 255) / 256, count), dim3(256), 0, c->stream, f, 0, theta,
                         dt_ctl, dt);
      HIPCHK(c, hipGetLastError());
      dt_ctl = nullptr;
    }
    // the second pass only mirrors frame cells outside the domain
    if (walls) {
      hipLaunchKernelGGL(k_ghost_fill, dim3((maxring + 255) / 256, count), dim3(256), 0, c->stream, f, 1, theta,
                         dt_ctl, dt);
      HIPCHK(c, hipGetLastError());
      dt_ctl = nullptr;
    }
  }
  if (dt_ctl) {
    hipLaunchKernelGGL(k_set_dt, dim3(1), dim3(1), 0, c->stream, dt_ctl, dt);
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
  // one wave per problem suffices for a few tiles; a problem with many gets 16,
  // and one with tens of thousands gets a block per 8192 of them (at most 32),
  // combined by a second launch
  const int big = LL.max_info_tiles > 256;
  const int slices = std::min(AFTER_MAX_SLICES, std::max(1, LL.max_info_tiles / 8192));
  const LevelInfo* li = LL.li + (size_t)runs * LL.nli + first;
  hipLaunchKernelGGL(k_after_substep, dim3(n, slices), dim3(big ? 1024 : 64), 0, c->stream, c->ctl, c->cnt, li,
                     LL.parts, c->cfg.cfl_max, LL.red, c->halt, c->skip);
  if (slices > 1) {
    HIPCHK(c, hipGetLastError());
    hipLaunchKernelGGL(k_after_combine, dim3((n + 63) / 64), dim3(64), 0, c->stream, c->ctl, c->cnt, li, n, slices,
                       LL.red, c->cfg.cfl_max, c->halt, c->skip);
  }
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
int coarsen_level(mlswe_ctx* c, int lf, int p0, int p1, bool apply_reflux) {
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
    HIPCHK(c, host_wait(c));
  }
  return timed(c, 6, [&]() -> int {
    hipLaunchKernelGGL(k_next_dt, dim3((p1 - p0 + 63) / 64), dim3(64), 0, c->stream, c->ctl, c->pdt + p0, p1 - p0,
                       c->cfg.cfl_desired, initial ? 1 : 0, c->halt);
    HIPCHK(c, hipGetLastError());
    return MLSWE_OK;
  });
}

// Control blocks of problems [p0, p1) (contiguous, problem-major) in one copy.
int read_ctls(mlswe_ctx* c, int p0, int p1, std::vector<LevelCtl>& h) {
  const int a = c->probs[p0].ctl0, b = c->probs[p1 - 1].ctl0 + c->probs[p1 - 1].nlev;
  h.resize((size_t)(b - a));
  HIPCHK(c, hipMemcpyAsync(h.data(), c->ctl + a, sizeof(LevelCtl) * h.size(), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, host_wait(c));
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

}  // namespace mlswe_host
