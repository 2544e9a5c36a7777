"""Python binding of the C ABI in include/mlswe.h (argument marshalling only).

Every step of the computation runs in the HIP library ``libmlswe.so``; this
module only converts arrays and codes.  It refuses to run without the library:
there is no CPU fallback.

Callers that pass torch device tensors initialise torch's GPU runtime
(``torch.cuda.init()``) before creating a Solver, and give the Solver torch's
stream so that the library's launches and torch's work are ordered.
"""
from __future__ import annotations

import ctypes
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libmlswe.so")

OK, EINVAL, ENOMEM, EDEVICE, ECFL, ENAN, ESTATE = 0, -1, -2, -3, -4, -5, -6
HOST, DEVICE = 0, 1
PLAIN, BATCHED, GRAPH, PER_PATCH = 0, 1, 2, 3
MAXLEV = 8

ERRNAMES = {EINVAL: "EINVAL", ENOMEM: "ENOMEM", EDEVICE: "EDEVICE", ECFL: "ECFL", ENAN: "ENAN", ESTATE: "ESTATE"}


class Config(ctypes.Structure):
    _fields_ = [("g", ctypes.c_double), ("hdry", ctypes.c_double), ("kmin", ctypes.c_double),
                ("cfl_desired", ctypes.c_double), ("cfl_max", ctypes.c_double),
                ("y_rows", ctypes.c_int), ("x_rows", ctypes.c_int),
                ("max_device_bytes", ctypes.c_int64), ("max_retries", ctypes.c_int), ("reflux", ctypes.c_int),
                ("dynamic_rt", ctypes.c_int), ("pad_", ctypes.c_int)]


class CountersC(ctypes.Structure):
    _fields_ = [("cell_updates", ctypes.c_int64 * 8), ("hyp", ctypes.c_int64), ("nclip", ctypes.c_int64),
                ("repair", ctypes.c_int64), ("clip1", ctypes.c_double), ("clip2", ctypes.c_double),
                ("t", ctypes.c_double), ("status", ctypes.c_int), ("rejected", ctypes.c_int64)]


class Tuning(ctypes.Structure):
    _fields_ = [("x_rows", ctypes.c_int), ("y_rows", ctypes.c_int), ("sched_x", ctypes.c_int),
                ("sched_y", ctypes.c_int), ("grid_x", ctypes.c_int), ("grid_y", ctypes.c_int),
                ("fast", ctypes.c_int)]


class MlsweError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (ERRNAMES.get(code, "?"), code, msg))
        self.code = code


_lib = None


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise RuntimeError("libmlswe.so is not built (run __graft_entry__.build()); "
                               "there is no fallback path")
        L = ctypes.CDLL(LIBPATH)
        P, I, D, V = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
        IP = ctypes.POINTER(ctypes.c_int)
        DP = ctypes.POINTER(ctypes.c_double)
        I32P = ctypes.POINTER(ctypes.c_int32)
        sig = {
            "mlswe_version": (I, []),
            "mlswe_last_error": (ctypes.c_char_p, [P]),
            "mlswe_create": (I, [ctypes.POINTER(Config), V, ctypes.POINTER(P)]),
            "mlswe_destroy": (I, [P]),
            "mlswe_problem_define": (I, [P, IP, D, I, I, D, D, I, IP]),
            "mlswe_set_bathymetry": (I, [P, I, V, I]),
            "mlswe_set_patches": (I, [P, I, I, I, I32P]),
            "mlswe_get_patches": (I, [P, I, I, I, I32P, IP]),
            "mlswe_set_state": (I, [P, I, I, V, I]),
            "mlswe_get_state": (I, [P, I, I, V, I]),
            "mlswe_step_level": (I, [P, I, DP, D, DP]),
            "mlswe_coarsen": (I, [P, I, I]),
            "mlswe_flag": (I, [P, I, I, D, I, ctypes.POINTER(ctypes.c_uint8)]),
            "mlswe_flag_noalloc": (I, [P, I, I, D, I, V]),
            "mlswe_refine": (I, [P, I, I, I, I32P]),
            "mlswe_regrid": (I, [P, I, DP, I]),
            "mlswe_advance": (I, [P, I, I, DP, I, I, DP]),
            "mlswe_get_counters": (I, [P, I, ctypes.POINTER(CountersC)]),
            "mlswe_synchronize": (I, [P]),
            "mlswe_sync_counts": (I, [P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                      ctypes.POINTER(ctypes.c_int64)]),
            "mlswe_set_kernel_timing": (I, [P, I]),
            "mlswe_kernel_times": (I, [P, DP, ctypes.POINTER(ctypes.c_int64)]),
            "mlswe_phase_times": (I, [P, DP, ctypes.POINTER(ctypes.c_int64), I]),
            "mlswe_run_fixed": (I, [P, I, I, DP]),
            "mlswe_adjoint_step": (I, [P, I, V, V, V, V, D]),
            "mlswe_param_map": (I, [P, I, V, D, V]),
            "mlswe_param_map_adjoint": (I, [P, I, V, D, V, V, V]),
            "mlswe_gauge_misfit": (I, [P, I, V, I, I, I, V, V, V, V]),
            "mlswe_branch_signature": (I, [P, I, I, ctypes.POINTER(ctypes.c_uint64)]),
            "mlswe_get_tuning": (I, [P, ctypes.POINTER(Tuning)]),
            "mlswe_set_tuning": (I, [P, ctypes.POINTER(Tuning)]),
            "mlswe_autotune": (I, [P, ctypes.c_char_p, I]),
            "mlswe_run_tiles": (I, [I, I, I, I32P, I, I, I32P, I]),
            "mlswe_get_step_state": (I, [P, I, DP]),
            "mlswe_get_time_ratios": (I, [P, I, I32P]),
            "mlswe_set_step_state": (I, [P, I, DP]),
            "mlswe_refine_layers": (I, [P, I, I, V, V, I, I, I, I, I, I, V, V, ctypes.POINTER(ctypes.c_int64)]),
            "mlswe_coarsen_layers": (I, [P, I, I, V, I, I, I, I, V, I, I]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def run_tiles(nx, ny, boxes, axis, rows):
    """The union tiles of one level (host only): rows of (i0, ncols, j0, nrows,
    flags) in launch order."""
    L = lib()
    b = np.ascontiguousarray(np.asarray(boxes, dtype=np.int32).reshape(-1, 4))
    bp = b.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    n = L.mlswe_run_tiles(nx, ny, b.shape[0], bp, axis, rows, None, 0)
    if n < 0:
        raise MlsweError(n, "bad run-tile arguments")
    out = np.zeros((max(n, 1), 5), dtype=np.int32)
    L.mlswe_run_tiles(nx, ny, b.shape[0], bp, axis, rows, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), n)
    return out[:n]


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, shape, device=None):
    """(pointer, where) of a numpy array or a torch tensor holding exactly
    `shape` float64 values contiguously (device pointers of GPU tensors are
    passed as device memory; they must live on the context's GPU `device`).
    Anything else raises MlsweError(EINVAL) before the library reads it."""
    shape = tuple(int(v) for v in shape)
    if isinstance(a, np.ndarray):
        if a.dtype != np.float64 or not a.flags.c_contiguous:
            raise MlsweError(-1, "expected a contiguous float64 array, got %s" % a.dtype)
        if a.shape != shape:
            raise MlsweError(-1, "array of shape %s, expected %s" % (a.shape, shape))
        return a.ctypes.data_as(ctypes.c_void_p), HOST
    if hasattr(a, "data_ptr") and hasattr(a, "is_cuda"):
        if str(a.dtype) != "torch.float64" or not a.is_contiguous():
            raise MlsweError(-1, "expected a contiguous float64 tensor, got %s" % a.dtype)
        if tuple(a.shape) != shape:
            raise MlsweError(-1, "tensor of shape %s, expected %s" % (tuple(a.shape), shape))
        if a.is_cuda:
            if device is not None and a.device.index != device:
                raise MlsweError(-1, "tensor on cuda:%s, the context runs on cuda:%d" % (a.device.index, device))
            return ctypes.c_void_p(a.data_ptr()), DEVICE
        return ctypes.c_void_p(a.data_ptr()), HOST
    raise MlsweError(-1, "expected a numpy array or a torch tensor")


class Solver:
    """One library context (one GPU stream) holding any number of problems."""

    def __init__(self, g=9.81, hdry=1e-3, kmin=1e-6, cfl=0.9, cfl_max=1.0, y_rows=0, x_rows=0,
                 max_device_bytes=0, stream=None, max_retries=0, reflux=False, dynamic_rt=False):
        self.L = lib()
        cfg = Config(g, hdry, kmin, cfl, cfl_max, y_rows, x_rows, max_device_bytes, max_retries, 1 if reflux else 0,
                     1 if dynamic_rt else 0, 0)
        h = ctypes.c_void_p()
        rc = self.L.mlswe_create(ctypes.byref(cfg), stream, ctypes.byref(h))
        if rc:
            raise MlsweError(rc, "mlswe_create failed (no usable GPU?)")
        self.h = h
        self.shapes = []   # per problem: list of (nx, ny, dx, dy)
        self.dev = None
        if "torch" in sys.modules:
            import torch
            if torch.cuda.is_available():
                self.dev = torch.cuda.current_device()

    def close(self):
        if getattr(self, "h", None):
            self.L.mlswe_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc:
            raise MlsweError(rc, self.L.mlswe_last_error(self.h).decode())

    # ------------------------------------------------------------ set-up
    def define(self, nx0, ny0, dx0, dy0, r, ratios=()):
        p = ctypes.c_int()
        rat = (ctypes.c_int * max(1, len(ratios)))(*ratios) if ratios else None
        self._check(self.L.mlswe_problem_define(self.h, ctypes.byref(p), r, nx0, ny0, dx0, dy0,
                                                len(ratios) + 1, rat))
        shp = [(nx0, ny0, dx0, dy0)]
        for rr in ratios:
            nx, ny, dx, dy = shp[-1]
            shp.append((nx * rr, ny * rr, dx / rr, dy / rr))
        self.shapes.append(shp)
        return p.value

    def _device(self):
        """Index of the GPU the context was created on (torch's numbering)."""
        if self.dev is None and "torch" in sys.modules:
            import torch
            if torch.cuda.is_available():
                self.dev = torch.cuda.current_device()
        return self.dev

    def set_bathymetry(self, p, Bf):
        if isinstance(Bf, np.ndarray):
            Bf = _f64(Bf)
        nx, ny = self.shapes[p][-1][:2]
        ptr, where = _ptr(Bf, (ny, nx), self._device())
        self._check(self.L.mlswe_set_bathymetry(self.h, p, ptr, where))

    def set_patches(self, p, level, boxes):
        b = np.ascontiguousarray(np.asarray(boxes, dtype=np.int32).reshape(-1, 4))
        self._check(self.L.mlswe_set_patches(self.h, p, level, b.shape[0],
                                             b.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))

    def refine(self, p, level, boxes):
        b = np.ascontiguousarray(np.asarray(boxes, dtype=np.int32).reshape(-1, 4))
        self._check(self.L.mlswe_refine(self.h, p, level, b.shape[0],
                                        b.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))

    def patches(self, p, level):
        nx, ny = self.shapes[p][level][:2]
        cap = (nx // 1) * (ny // 1) // 256 + 16
        b = np.zeros((cap, 4), dtype=np.int32)
        n = ctypes.c_int()
        self._check(self.L.mlswe_get_patches(self.h, p, level, cap, b.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                             ctypes.byref(n)))
        return b[:n.value]

    def set_state(self, p, level, q):
        if isinstance(q, np.ndarray):
            q = _f64(q)
        nx, ny = self.shapes[p][level][:2]
        ptr, where = _ptr(q, (6, ny, nx), self._device())
        self._check(self.L.mlswe_set_state(self.h, p, level, ptr, where))

    def state(self, p, level):
        nx, ny = self.shapes[p][level][:2]
        q = np.zeros((6, ny, nx))
        self._check(self.L.mlswe_get_state(self.h, p, level, q.ctypes.data_as(ctypes.c_void_p), HOST))
        return q

    # ------------------------------------------------------------ operators
    def step_level(self, level, dts=None, theta=0.0, want_smax=True):
        n = len(self.shapes)
        d = None
        if dts is not None:
            dd = _f64(np.broadcast_to(np.asarray(dts, dtype=np.float64), (n,)))
            d = dd.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        sm = np.zeros((n, 2)) if want_smax else None
        rc = self.L.mlswe_step_level(self.h, level, d, theta,
                                     sm.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if want_smax else None)
        self._check(rc)
        return sm

    def coarsen(self, p, fine_level):
        self._check(self.L.mlswe_coarsen(self.h, p, fine_level))

    def flag(self, p, level, tau, nbuf=2):
        nx, ny = self.shapes[p][level][:2]
        f = np.zeros((ny, nx), dtype=np.uint8)
        self._check(self.L.mlswe_flag(self.h, p, level, tau, nbuf, f.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))
        return f

    def flag_noalloc(self, p, level, tau, out, nbuf=2):
        """Flags of a level into `out`, a contiguous uint8 CUDA tensor of shape
        (ny, nx) on the context's GPU, with no device allocation by the library
        (asynchronous on the context's stream)."""
        nx, ny = self.shapes[p][level][:2]
        if not (hasattr(out, "data_ptr") and getattr(out, "is_cuda", False)):
            raise MlsweError(-1, "expected a CUDA tensor")
        if str(out.dtype) != "torch.uint8" or not out.is_contiguous() or tuple(out.shape) != (ny, nx):
            raise MlsweError(-1, "expected a contiguous uint8 tensor of shape %s" % ((ny, nx),))
        if self.dev is not None and out.device.index != self.dev:
            raise MlsweError(-1, "tensor on cuda:%s, the context runs on cuda:%d" % (out.device.index, self.dev))
        self._check(self.L.mlswe_flag_noalloc(self.h, p, level, tau, nbuf, ctypes.c_void_p(out.data_ptr())))

    def regrid(self, p, tau, nbuf=2):
        t = _f64(list(tau) + [0.0] * (MAXLEV - len(tau)))
        self._check(self.L.mlswe_regrid(self.h, p, t.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), nbuf))

    def advance(self, nsteps, regrid_every=0, tau=None, nbuf=2, mode=PLAIN, want_dts=False):
        n = len(self.shapes)
        t = None
        if tau is not None:
            tt = np.zeros((n, MAXLEV))
            tau = np.asarray(tau, dtype=np.float64)
            if tau.ndim == 1:
                tau = np.broadcast_to(tau, (n, tau.shape[0]))
            tt[:, :tau.shape[1]] = tau
            t = tt.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            self._tau_keep = tt
        dts = np.zeros((n, nsteps)) if want_dts else None
        rc = self.L.mlswe_advance(self.h, nsteps, regrid_every, t, nbuf, mode,
                                  dts.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if want_dts else None)
        self._check(rc)
        return dts

    def time_ratios(self, p):
        """Time ratios of problem p's last coarse step (one per level above 0)."""
        n = len(self.shapes[p]) - 1
        out = np.zeros(max(1, n), dtype=np.int32)
        self._check(self.L.mlswe_get_time_ratios(self.h, p, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return out[:n]

    def counters(self, p):
        c = CountersC()
        self._check(self.L.mlswe_get_counters(self.h, p, ctypes.byref(c)))
        nl = len(self.shapes[p])
        return dict(updates=[int(c.cell_updates[l]) for l in range(nl)], hyp=int(c.hyp), nclip=int(c.nclip),
                    repair=int(c.repair), clip1=c.clip1, clip2=c.clip2, t=c.t, status=int(c.status),
                    rejected=int(c.rejected))

    def run_fixed(self, p, dts):
        d = _f64(dts)
        self._check(self.L.mlswe_run_fixed(self.h, p, d.shape[0], d.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))

    def tuning(self):
        t = Tuning()
        self._check(self.L.mlswe_get_tuning(self.h, ctypes.byref(t)))
        return dict(x_rows=t.x_rows, y_rows=t.y_rows, sched_x=t.sched_x, sched_y=t.sched_y,
                    grid_x=t.grid_x, grid_y=t.grid_y, fast=t.fast)

    def set_tuning(self, **kw):
        cur = self.tuning()
        cur.update(kw)
        t = Tuning(cur["x_rows"], cur["y_rows"], cur["sched_x"], cur["sched_y"], cur["grid_x"], cur["grid_y"],
                   cur["fast"])
        self._check(self.L.mlswe_set_tuning(self.h, ctypes.byref(t)))

    def autotune(self, cache_path=None, reps=3):
        self._check(self.L.mlswe_autotune(self.h, cache_path.encode() if cache_path else None, reps))
        return self.tuning()

    def branch_signature(self, p, enable=-1):
        """Returns and clears problem p's branch signature; enable 1/0 switches
        the accumulation on/off (-1 leaves it)."""
        v = ctypes.c_uint64()
        self._check(self.L.mlswe_branch_signature(self.h, enable, p, ctypes.byref(v)))
        return v.value

    def synchronize(self):
        self._check(self.L.mlswe_synchronize(self.h))

    def sync_counts(self):
        """(host waits on the stream, graphs captured, graphs replayed) so far."""
        a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        self._check(self.L.mlswe_sync_counts(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return int(a.value), int(b.value), int(c.value)

    def set_kernel_timing(self, on=True):
        self._check(self.L.mlswe_set_kernel_timing(self.h, 1 if on else 0))

    PHASES = ("x_sweep", "y_sweep", "ghost_fill", "substep_reduction", "coarsen", "flux_correction", "dt_rule",
              "regrid")

    def phase_times(self):
        """{phase: (milliseconds, count)} since timing was enabled."""
        ms = (ctypes.c_double * 8)()
        n = (ctypes.c_int64 * 8)()
        rc = self.L.mlswe_phase_times(self.h, ms, n, 8)
        if rc < 0:
            self._check(rc)
        return {name: (ms[k], int(n[k])) for k, name in enumerate(self.PHASES)}

    def kernel_times(self):
        ms = (ctypes.c_double * 2)()
        n = (ctypes.c_int64 * 2)()
        self._check(self.L.mlswe_kernel_times(self.h, ms, n))
        return [ms[0], ms[1]], [int(n[0]), int(n[1])]

    # ------------------------------------------------------------ checkpoint / resume
    def step_state(self, p):
        """[t, speeds-known flag, per level largest x / y speeds of the last
        coarse step] of problem p."""
        n = len(self.shapes[p])
        out = np.zeros(2 + 2 * n)
        self._check(self.L.mlswe_get_step_state(self.h, p, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def set_step_state(self, p, v):
        v = _f64(v)
        if v.shape != (2 + 2 * len(self.shapes[p]),):
            raise ValueError("expected %d values" % (2 + 2 * len(self.shapes[p])))
        self._check(self.L.mlswe_set_step_state(self.h, p, v.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))

    # ------------------------------------------------------------ M layers
    def _dev(self, t, shape):
        if not (hasattr(t, "is_cuda") and t.is_cuda):
            raise MlsweError(-1, "expected a float64 device tensor")
        return _ptr(t, shape, self._device())[0]

    def refine_layers(self, qc, Bc, Bf, qf, r, box=None, want_repairs=False):
        """Fine cells of box (fi0, fj0, fnx, fny) (default: the whole fine grid)
        refined from the coarse state qc [3M][nyc][nxc] with bathymetry Bc into
        qf [3M][fny][fnx], fine bathymetry Bf [fny][fnx] (device float64
        tensors).  Returns the number of wet-ordering repairs if asked."""
        M = qc.shape[0] // 3
        nyc, nxc = Bc.shape
        fi0, fj0, fnx, fny = box if box is not None else (0, 0, r * nxc, r * nyc)
        n = ctypes.c_int64()
        self._check(self.L.mlswe_refine_layers(
            self.h, M, r, self._dev(qc, (3 * M, nyc, nxc)), self._dev(Bc, (nyc, nxc)), nxc, nyc, fi0, fj0, fnx, fny,
            self._dev(Bf, (fny, fnx)), self._dev(qf, (3 * M, fny, fnx)), ctypes.byref(n) if want_repairs else None))
        return n.value if want_repairs else None

    def coarsen_layers(self, qf, qc, r, origin=(0, 0)):
        """Coarse cells of the box at origin (ci0, cj0) of qc [3M][nyc][nxc]
        from their children qf [3M][r cny][r cnx] (device float64 tensors)."""
        M = qc.shape[0] // 3
        _, nyc, nxc = qc.shape
        cny, cnx = qf.shape[1] // r, qf.shape[2] // r
        self._check(self.L.mlswe_coarsen_layers(
            self.h, M, r, self._dev(qf, (3 * M, r * cny, r * cnx)), origin[0], origin[1], cnx, cny,
            self._dev(qc, (3 * M, nyc, nxc)), nxc, nyc))
