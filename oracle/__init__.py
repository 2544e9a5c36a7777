"""Reference oracle for the two-layer shallow-water hot path -- TEST INFRASTRUCTURE.

A plain, single-threaded FP64 CPU implementation (C++ in this folder, loaded with
ctypes).  It shares no code with the HIP library in ``paper_1803_01450_amd`` and
neither side imports the other.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may use it; the product path never does.

Passages of the paper it follows (Schwarzschild & Mandli, arXiv 1803.01450):
level hierarchy and ratios (Sec. 2, Eqs. 1-2), time refinement (Sec. 2), wet
ordering, surface (not depth) refinement, effective bathymetry and the
minmod-limited interpolant (Sec. 2.1, Eqs. 3-10), coarsening by averaging
(Sec. 2.2, Eq. 11).  The solver itself is not written in the paper (Sec. 1 cites
it); the readings used are stated in the comments of ``ora_core.hpp``.
"""
from __future__ import annotations

import contextlib
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "liboracle.so")
_SRCS = ["ora_amr.cpp", "ora_adjoint.cpp", "ora_count.cpp"]

G = 9.81
HDRY = 1.0e-3
KMIN = 1.0e-6


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (FP64, no contraction, no fast-math)."""
    srcs = [os.path.join(_HERE, s) for s in _SRCS]
    if not force and os.path.exists(_LIB):
        newest = max(os.path.getmtime(s) for s in srcs + [os.path.join(_HERE, "ora_core.hpp")])
        if os.path.getmtime(_LIB) >= newest:
            return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-pthread",
           "-o", tmp] + srcs
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None

_D = ctypes.c_double
_I = ctypes.c_int
_P = ctypes.c_void_p
_DP = ctypes.POINTER(ctypes.c_double)
_IP = ctypes.POINTER(ctypes.c_int)


def _configure(L):
    L.ora_create.restype = _P
    L.ora_create.argtypes = [_D, _D, _D, _D, _D, _D, _I, _IP, _I, _I, _D, _D]
    L.ora_destroy.argtypes = [_P]
    for name in ["ora_set_bathymetry"]:
        getattr(L, name).argtypes = [_P, _DP]
    L.ora_get_bathymetry.argtypes = [_P, _I, _DP]
    L.ora_get_step_state.argtypes = [_P, _DP]
    L.ora_set_reflux.argtypes = [_P, _I]
    L.ora_set_dynamic_rt.argtypes = [_P, _I]
    L.ora_get_rt.argtypes = [_P, _IP]
    L.ora_set_step_state.argtypes = [_P, _DP]
    L.ora_set_state.argtypes = [_P, _I, _DP]
    L.ora_get_state.argtypes = [_P, _I, _DP]
    L.ora_level_shape.argtypes = [_P, _I, _IP, _IP, _DP, _DP]
    L.ora_set_patches.argtypes = [_P, _I, _I, _IP]
    L.ora_get_npatches.argtypes = [_P, _I]
    L.ora_get_patches.argtypes = [_P, _I, _IP]
    L.ora_step_level.argtypes = [_P, _I, _D, _D, _DP]
    L.ora_coarsen.argtypes = [_P, _I]
    L.ora_flag.argtypes = [_P, _I, _D, _I, ctypes.POINTER(ctypes.c_ubyte)]
    L.ora_cluster.argtypes = [_P, _I, ctypes.POINTER(ctypes.c_ubyte), _IP, _I]
    L.ora_regrid.argtypes = [_P, _DP, _I]
    L.ora_advance.argtypes = [_P, _I, _I, _DP, _I, _DP]
    L.ora_next_dt.restype = _D
    L.ora_next_dt.argtypes = [_P]
    L.ora_counters.argtypes = [_P, _DP]
    L.ora_refine_point.argtypes = [_D, _I, _I, _I, _DP, _I, _I, _D, _DP]
    L.ora_riemann.argtypes = [_D, _D, _D, _D, _DP, _DP, _DP, _DP, _IP, _DP, _DP]
    L.ora_fixed_steps.argtypes = [_I, _I, _D, _D, _D, _D, _D, _D, _DP, _DP, _I, _DP, _DP, _DP]
    L.ora_time_fixed.restype = _D
    L.ora_time_fixed.argtypes = [_I, _I, _D, _D, _D, _D, _D, _D, _DP, _DP, _I, _D, _DP]
    L.ora_time_fixed_mt.restype = _D
    L.ora_time_fixed_mt.argtypes = [_I, _I, _D, _D, _D, _D, _D, _D, _DP, _DP, _I, _D, _I, _DP, _DP]
    L.ora_count_ops.argtypes = [_I, _I, _D, _D, _D, _D, _D, _D, _DP, _DP, _D,
                                ctypes.POINTER(ctypes.c_longlong)]
    L.ora_step_window.argtypes = [_I, _I, _D, _D, _D, _D, _D, _D, _DP, _DP, _IP, _D, _DP, _DP]
    L.ora_gauge_loss.restype = _D
    L.ora_gauge_loss.argtypes = [_I, _D, _D, _D, _D, _D, _DP, _DP, _D, _I, _DP, _I, _I, _I, _I,
                                 _DP, _DP, _DP, _DP]
    L.ora_set_retries.argtypes = [_P, _I]
    L.ora_ghost_fill.argtypes = [_P, _I, _D]
    L.ora_get_level_raw.argtypes = [_P, _I, _I, _DP]
    L.ora_mc_limiter.restype = _D
    L.ora_mc_limiter.argtypes = [_D]
    return L


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = _configure(ctypes.CDLL(_LIB))
    return _lib


@contextlib.contextmanager
def variant(path):
    """Runs the oracle's Python helpers against another build of the oracle
    (the mutation tests plant a slip in a copy of the sources)."""
    global _lib
    saved = lib()
    _lib = _configure(ctypes.CDLL(path))
    try:
        yield
    finally:
        _lib = saved


def sources():
    """Paths of the oracle's C++ sources and header (for rebuilding a copy)."""
    return [os.path.join(_HERE, s) for s in _SRCS] + [os.path.join(_HERE, "ora_core.hpp")]


def compile_to(srcdir, out):
    """Compiles the oracle sources found in srcdir into the library out, with
    the flags of build()."""
    cmd = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-pthread",
           "-o", out] + [os.path.join(srcdir, s) for s in _SRCS]
    subprocess.check_call(cmd)
    return out


def mc_limiter(theta):
    """The oracle's limiter function phi(theta)."""
    return lib().ora_mc_limiter(float(theta))


def _dp(a):
    return a.ctypes.data_as(_DP)


def _ip(a):
    return a.ctypes.data_as(_IP)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ------------------------------------------------------------------ single edge
def riemann(qL, qR, r=0.95, g=G, hdry=HDRY, kmin=KMIN):
    """Layered f-wave solve at one edge.  q = (h1, m1, t1, h2, m2, t2, B) with m the
    normal and t the transverse momentum.  Returns dict(s, Z, mode, amdq, apdq, hyp)."""
    qL = _f64(qL); qR = _f64(qR)
    s = np.zeros(6); Z = np.zeros(36); mode = np.zeros(6, dtype=np.int32)
    am = np.zeros(6); ap = np.zeros(6)
    hyp = lib().ora_riemann(g, r, hdry, kmin, _dp(qL), _dp(qR), _dp(s), _dp(Z), _ip(mode), _dp(am), _dp(ap))
    return dict(s=s, Z=Z.reshape(6, 6), mode=mode, amdq=am, apdq=ap, hyp=hyp)


def refine_point(q5, r, a, b, Bf, inx=True, iny=True, hdry=HDRY):
    """Refine one fine cell from a 5-point coarse stencil q5[5][7] (centre, left,
    right, down, up; values h1 hu1 hv1 h2 hu2 hv2 B)."""
    q5 = _f64(q5).reshape(-1)
    out = np.zeros(6)
    rep = lib().ora_refine_point(hdry, r, a, b, _dp(q5), int(inx), int(iny), float(Bf), _dp(out))
    return out, rep


# ------------------------------------------------------------------ fixed grid
def fixed_steps(B, q, dx, dy, dts, r=0.95, g=G, hdry=HDRY, kmin=KMIN):
    """Wall-bounded single-level run with a given dt sequence.  B [ny][nx],
    q [6][ny][nx].  Returns (q_new, smax[n][2], counters[5])."""
    B = _f64(B); q = _f64(q).copy(); dts = _f64(dts)
    ny, nx = B.shape
    sm = np.zeros(2 * len(dts)); cnt = np.zeros(5)
    lib().ora_fixed_steps(nx, ny, dx, dy, g, r, hdry, kmin, _dp(B), _dp(q), len(dts), _dp(dts), _dp(sm), _dp(cnt))
    return q, sm.reshape(-1, 2), cnt


def step_window(B, q, dx, dy, box, dt, r=0.95, g=G, hdry=HDRY, kmin=KMIN):
    """One step of the window box=(ilo, jlo, nx, ny) of a wall-bounded level."""
    B = _f64(B); q = _f64(q)
    ny, nx = B.shape
    bx = np.asarray(box, dtype=np.int32)
    out = np.zeros((6, box[3], box[2])); sm = np.zeros(2)
    rc = lib().ora_step_window(nx, ny, dx, dy, g, r, hdry, kmin, _dp(B), _dp(q), _ip(bx), dt, _dp(out), _dp(sm))
    if rc:
        raise ValueError("bad window")
    return out, sm


def time_fixed(B, q, dx, dy, nsteps, dt, r=0.95, g=G, hdry=HDRY, kmin=KMIN):
    """(cell updates per second, seconds) of the oracle's step on this grid."""
    B = _f64(B); q = _f64(q)
    ny, nx = B.shape
    sec = ctypes.c_double(0.0)
    rate = lib().ora_time_fixed(nx, ny, dx, dy, g, r, hdry, kmin, _dp(B), _dp(q), nsteps, dt, ctypes.byref(sec))
    return rate, sec.value


def time_fixed_mt(B, q, dx, dy, nsteps, dt, threads, r=0.95, g=G, hdry=HDRY, kmin=KMIN, want_state=False):
    """(cell updates per second, seconds[, final state]) of the same step on
    `threads` host threads (rows cut into strips, each stepped as a box)."""
    B = _f64(B); q = _f64(q)
    ny, nx = B.shape
    sec = ctypes.c_double(0.0)
    out = np.zeros((6, ny, nx)) if want_state else None
    rate = lib().ora_time_fixed_mt(nx, ny, dx, dy, g, r, hdry, kmin, _dp(B), _dp(q), nsteps, dt, int(threads),
                                   ctypes.byref(sec), _dp(out) if want_state else None)
    return (rate, sec.value, out) if want_state else (rate, sec.value)


def count_ops(B, q, dx, dy, dt, r=0.95, g=G, hdry=HDRY, kmin=KMIN):
    """FP64 operations of one oracle step of this grid, per sweep:
    {"x": {...}, "y": {...}} with counts of add (incl. subtract), mul, div, sqrt,
    neg and fma, the flops (fma counted as two, negation as none) and the
    cells each pass updates."""
    B = _f64(B); q = _f64(q)
    ny, nx = B.shape
    out = (ctypes.c_longlong * 12)()
    rc = lib().ora_count_ops(nx, ny, dx, dy, g, r, hdry, kmin, _dp(B), _dp(q), dt, out)
    if rc != 0:
        raise ValueError("grid below 2 x 2")
    names = ("add", "mul", "div", "sqrt", "neg", "fma")
    x = {k: int(out[i]) for i, k in enumerate(names)}
    y = {k: int(out[6 + i]) for i, k in enumerate(names)}
    for d in (x, y):
        # a sign change is an operand modifier, not an operation
        d["flops"] = d["add"] + d["mul"] + d["div"] + d["sqrt"] + 2 * d["fma"]
    x["cells"] = nx * (ny + 4)
    y["cells"] = nx * ny
    return {"x": x, "y": y}


def gauge_loss(eta1_0, B, dx, eta2_0, dts, every, gauge, targets, v_eta=None, v_B=None, r=0.95,
               g=G, hdry=HDRY, kmin=KMIN):
    """Gauge misfit of a fixed-grid run (and its directional derivative along
    (v_eta, v_B) when given).  gauge = (i0, j0, n)."""
    e = _f64(eta1_0); B = _f64(B); dts = _f64(dts); tg = _f64(targets)
    n = e.shape[0]
    ve = _f64(v_eta) if v_eta is not None else None
    vb = _f64(v_B) if v_B is not None else None
    d = ctypes.c_double(0.0)
    L = lib().ora_gauge_loss(n, dx, g, r, hdry, kmin, _dp(e), _dp(B), eta2_0, len(dts), _dp(dts), every,
                             gauge[0], gauge[1], gauge[2], _dp(tg),
                             _dp(ve) if ve is not None else None, _dp(vb) if vb is not None else None,
                             ctypes.byref(d))
    return (L, d.value) if (ve is not None or vb is not None) else L


# ------------------------------------------------------------------ hierarchy
class Hierarchy:
    """Level hierarchy (dense level arrays, patches as boxes) with the oracle's
    refine / coarsen / flag / cluster / step / advance."""

    def __init__(self, nx0, ny0, dx0, dy0, ratios=(), r=0.95, cfl=0.9, cflmax=1.0, g=G, hdry=HDRY, kmin=KMIN):
        self.nlev = len(ratios) + 1
        rat = np.asarray(list(ratios) + [1], dtype=np.int32)
        self.h = lib().ora_create(g, r, hdry, kmin, cfl, cflmax, self.nlev, _ip(rat), nx0, ny0, dx0, dy0)
        if not self.h:
            raise ValueError("bad hierarchy")
        self.shapes = []
        for l in range(self.nlev):
            nx = ctypes.c_int(); ny = ctypes.c_int(); dx = ctypes.c_double(); dy = ctypes.c_double()
            lib().ora_level_shape(self.h, l, ctypes.byref(nx), ctypes.byref(ny), ctypes.byref(dx), ctypes.byref(dy))
            self.shapes.append((nx.value, ny.value, dx.value, dy.value))

    def __del__(self):
        if getattr(self, "h", None):
            lib().ora_destroy(self.h)
            self.h = None

    def set_bathymetry(self, Bf):
        Bf = _f64(Bf)
        nx, ny = self.shapes[-1][:2]
        assert Bf.shape == (ny, nx)
        lib().ora_set_bathymetry(self.h, _dp(Bf))

    def bathymetry(self, l):
        nx, ny = self.shapes[l][:2]
        B = np.zeros((ny, nx))
        lib().ora_get_bathymetry(self.h, l, _dp(B))
        return B

    def set_state(self, l, q):
        q = _f64(q)
        nx, ny = self.shapes[l][:2]
        assert q.shape == (6, ny, nx)
        lib().ora_set_state(self.h, l, _dp(q))

    def state(self, l):
        nx, ny = self.shapes[l][:2]
        q = np.zeros((6, ny, nx))
        lib().ora_get_state(self.h, l, _dp(q))
        return q

    def set_patches(self, l, boxes):
        b = np.ascontiguousarray(np.asarray(boxes, dtype=np.int32).reshape(-1, 4))
        rc = lib().ora_set_patches(self.h, l, b.shape[0], _ip(b))
        if rc:
            raise ValueError("invalid patches")

    def patches(self, l):
        n = lib().ora_get_npatches(self.h, l)
        b = np.zeros((max(n, 1), 4), dtype=np.int32)
        lib().ora_get_patches(self.h, l, _ip(b))
        return b[:n]

    def step_level(self, l, dt, theta=0.0):
        sm = np.zeros(2)
        rc = lib().ora_step_level(self.h, l, dt, theta, _dp(sm))
        return rc, sm

    def coarsen(self, lf):
        lib().ora_coarsen(self.h, lf)

    def flag(self, l, tau, nbuf=2):
        nx, ny = self.shapes[l][:2]
        f = np.zeros((ny, nx), dtype=np.uint8)
        lib().ora_flag(self.h, l, tau, nbuf, f.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)))
        return f

    def cluster(self, l, flags):
        f = np.ascontiguousarray(flags, dtype=np.uint8)
        cap = f.size
        b = np.zeros((cap, 4), dtype=np.int32)
        n = lib().ora_cluster(self.h, l, f.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)), _ip(b), cap)
        return b[:n]

    def regrid(self, tau, nbuf=2):
        t = _f64(list(tau) + [0.0] * 8)
        return lib().ora_regrid(self.h, _dp(t), nbuf)

    def advance(self, nsteps, regrid_every=0, tau=(), nbuf=2):
        t = _f64(list(tau) + [0.0] * 8)
        dts = np.zeros(nsteps)
        rc = lib().ora_advance(self.h, nsteps, regrid_every, _dp(t), nbuf, _dp(dts))
        return rc, dts

    def next_dt(self):
        return lib().ora_next_dt(self.h)

    def set_reflux(self, on=True):
        """Mass flux correction at coarse-fine edges (off by default)."""
        lib().ora_set_reflux(self.h, 1 if on else 0)

    def set_dynamic_rt(self, on=True):
        """Time-refinement ratios chosen per coarse step from the last speeds
        (off by default: each equals the space ratio)."""
        lib().ora_set_dynamic_rt(self.h, 1 if on else 0)

    def time_ratios(self):
        """The time ratios of the last coarse step (one per level above 0)."""
        out = np.zeros(max(1, self.nlev - 1), dtype=np.int32)
        lib().ora_get_rt(self.h, _ip(out))
        return out[:self.nlev - 1]

    def step_state(self):
        """[t, speeds-known flag, per level largest x / y speeds of the last
        coarse step]: what a resumed run needs besides states and patches."""
        out = np.zeros(2 + 2 * self.nlev)
        lib().ora_get_step_state(self.h, _dp(out))
        return out

    def set_step_state(self, v):
        v = _f64(v)
        assert v.shape == (2 + 2 * self.nlev,)
        lib().ora_set_step_state(self.h, _dp(v))

    def set_retries(self, n):
        """Rejected coarse steps are retaken at most n times (default 8)."""
        lib().ora_set_retries(self.h, int(n))

    def ghost_fill(self, l, theta):
        """Fills the frame cells of level l's patches at time fraction theta of
        the coarser level's last step (as a substep of level l does first)."""
        lib().ora_ghost_fill(self.h, l, float(theta))

    def level_raw(self, l, which=0):
        """Level l's buffer with its two-cell frame, [6][ny + 4][nx + 4];
        which = 1: the state before the level's last step."""
        nx, ny = self.shapes[l][:2]
        q = np.zeros((6, ny + 4, nx + 4))
        lib().ora_get_level_raw(self.h, l, int(which), _dp(q))
        return q

    def counters(self):
        c = np.zeros(15)
        lib().ora_counters(self.h, _dp(c))
        return dict(hyp=int(c[0]), nclip=int(c[1]), repair=int(c[2]), clip1=c[3], clip2=c[4], t=c[5],
                    updates=[int(x) for x in c[6:6 + self.nlev]], rejected=int(c[14]))
