"""Union ("run") tiles, host side: the library's own tile lists (the host-only
entry point mlswe_run_tiles) checked on the CPU against patch-by-patch sweeps.

The kernels' per-lane rules are restated here: an x tile's lane l holds column
i0 - 2 + l, updates lanes 2 .. ncols + 1 and owns their left edges plus, with
flags bit 0, the edge after its last column; a y tile marches rows j0 - 2 ..
j0 + nrows + 1, owns the lower edges of its rows plus, with bit 0, the edge
above its last row, and writes a row only where the coverage byte says
interior.  An owned edge counts ia + ib - (ia and ib and b starts no patch in
that direction), from the coverage bytes of its two cells a, b.  Patch by
patch, a patch counts every edge of its interior rows from its first column's
left edge to its last column's right edge (x; columns likewise for y), and
every cell of its interior.  The two counts must agree edge by edge, the x
tiles must update every cell of the patches' rows and two frame rows on each
side exactly once, and the y tiles must write every interior cell exactly
once."""
import numpy as np
import pytest

from paper_1803_01450_amd import binding

IN, COL0, ROW0 = 1, 2, 4


def coverage(nx, ny, boxes):
    M = np.zeros((ny + 4, nx + 4), dtype=np.int64)  # [j + 2, i + 2]
    for (ilo, jlo, bnx, bny) in boxes:
        M[jlo + 2:jlo + bny + 2, ilo + 2:ilo + bnx + 2] = IN
        M[jlo + 2, ilo + 2:ilo + bnx + 2] |= ROW0
        M[jlo + 2:jlo + bny + 2, ilo + 2] |= COL0
    return M


def patch_counts(nx, ny, boxes):
    ex = np.zeros((ny + 4, nx + 5), dtype=np.int64)  # x edge e (left of column e) of row j
    ey = np.zeros((nx + 4, ny + 5), dtype=np.int64)  # y edge e (below row e) of column i
    for (ilo, jlo, bnx, bny) in boxes:
        ex[jlo + 2:jlo + bny + 2, ilo + 2:ilo + bnx + 3] += 1
        ey[ilo + 2:ilo + bnx + 2, jlo + 2:jlo + bny + 3] += 1
    return ex, ey


def tile_counts(nx, ny, boxes, rx, ry):
    M = coverage(nx, ny, boxes)
    m = lambda i, j: int(M[j + 2, i + 2])
    ex = np.zeros((ny + 4, nx + 5), dtype=np.int64)
    ey = np.zeros((nx + 4, ny + 5), dtype=np.int64)
    xw = np.zeros((ny + 4, nx + 4), dtype=np.int64)
    cells = np.zeros((ny + 4, nx + 4), dtype=np.int64)
    for (i0, ncol, j0, nrow, fl) in binding.run_tiles(nx, ny, boxes, 0, rx):
        assert -2 <= j0 and j0 + nrow <= ny + 2 and 0 <= i0 and i0 + ncol <= nx and 1 <= ncol <= 60
        for j in range(j0, j0 + nrow):
            for l in range(ncol + 4):
                c = i0 - 2 + l
                upd = 2 <= l < ncol + 2
                own = upd or (l == ncol + 2 and fl & 1)
                if upd:
                    xw[j + 2, c + 2] += 1
                    cells[j + 2, c + 2] += m(c, j) & IN
                if own:
                    cb = m(c, j)
                    ia, ib = m(c - 1, j) & IN, cb & IN
                    ex[j + 2, c + 2] += ia + ib - (ia & ib & (0 if cb & COL0 else 1))
    yw = np.zeros((ny + 4, nx + 4), dtype=np.int64)
    for (i0, ncol, j0, nrow, last) in binding.run_tiles(nx, ny, boxes, 1, ry):
        assert 0 <= j0 and j0 + nrow <= ny and 0 <= i0 and i0 + ncol <= nx and 1 <= ncol <= 64
        for l in range(ncol):
            i = i0 + l
            for k in range(1, nrow + 4):
                jj = j0 - 2 + k
                if (j0 <= jj < j0 + nrow) or (last & 1 and jj == j0 + nrow):
                    cb = m(i, jj)
                    ia, ib = m(i, jj - 1) & IN, cb & IN
                    ey[i + 2, jj + 2] += ia + ib - (ia & ib & (0 if cb & ROW0 else 1))
                if k >= 4 and m(i, jj - 2) & IN:
                    yw[jj, i + 2] += 1
    return M, ex, ey, xw, cells, yw


def check(nx, ny, boxes, rx, ry):
    M, ex, ey, xw, cells, yw = tile_counts(nx, ny, boxes, rx, ry)
    px, py = patch_counts(nx, ny, boxes)
    assert np.array_equal(ex, px), "x edge multiplicities"
    assert np.array_equal(ey, py), "y edge multiplicities"
    assert np.array_equal(cells, M & IN), "x fix-up cells"
    assert np.array_equal(yw, M & IN), "y writes"
    region = np.zeros_like(xw)
    for (ilo, jlo, bnx, bny) in boxes:
        region[jlo:jlo + bny + 4, ilo + 2:ilo + bnx + 2] = 1
    assert xw.max() <= 1 and np.all(xw[region == 1] == 1), "x region covered once"


def random_layout(rng, nx, ny, n):
    cov = np.zeros((ny, nx), dtype=bool)
    out = []
    for _ in range(200):
        if len(out) >= n:
            break
        w, h = 2 * int(rng.integers(1, 40)), 2 * int(rng.integers(1, 40))
        if w > nx or h > ny:
            continue
        i, j = 2 * int(rng.integers(0, (nx - w) // 2 + 1)), 2 * int(rng.integers(0, (ny - h) // 2 + 1))
        if cov[j:j + h, i:i + w].any():
            continue
        cov[j:j + h, i:i + w] = True
        out.append((i, j, w, h))
    return out


def test_gpu_test_layout():
    boxes = [(16, 16, 32, 32), (48, 16, 16, 32), (24, 48, 72, 16), (96, 40, 20, 30), (116, 40, 10, 30)]
    for rx, ry in [(32, 128), (4, 8), (8, 16)]:
        check(128, 128, boxes, rx, ry)


@pytest.mark.parametrize("seed", range(6))
def test_random_layouts(seed):
    rng = np.random.default_rng(seed)
    for _ in range(5):
        nx, ny = 2 * int(rng.integers(10, 90)), 2 * int(rng.integers(10, 90))
        boxes = random_layout(rng, nx, ny, int(rng.integers(1, 12)))
        for rx, ry in [(4, 8), (32, 128), (3, 5), (1, 1)]:
            check(nx, ny, boxes, rx, ry)


def test_single_patch_tiles_match_patch_tiles():
    """One patch covering the level: the union tiles are the patch tiles."""
    t = binding.run_tiles(130, 70, [(0, 0, 130, 70)], 0, 32)
    strips = sorted(set(int(x) for x in t[:, 0]))
    assert strips == [0, 60, 120]
    assert sorted(set(int(x) for x in t[:, 2])) == [-2, 30, 62]
    assert int(t[:, 3].sum()) == 3 * 74


def test_bad_arguments():
    with pytest.raises(binding.MlsweError):
        binding.run_tiles(10, 10, [(0, 0, 12, 4)], 0, 4)
    with pytest.raises(binding.MlsweError):
        binding.run_tiles(10, 10, [(0, 0, 4, 4)], 2, 4)
