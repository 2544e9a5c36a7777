"""Gradient of a gauge misfit with respect to the initial top surface and the
bathymetry, through the library's hand-written adjoint of the fixed-grid step.

The forward run keeps a checkpoint every `ckpt` steps; the backward pass
recomputes each segment from its checkpoint, then applies the adjoint steps in
reverse, adding the misfit's source at the sampled steps.  Every arithmetic
step runs in the HIP library; this module only orders the calls and holds the
device buffers (torch tensors).
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import binding


def _vp(t):
    """Device pointer of a contiguous float64 GPU tensor (MlsweError otherwise)."""
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise binding.MlsweError(-1, "expected a contiguous float64 device tensor")
    return ctypes.c_void_p(t.data_ptr())


class MisfitProblem:
    """Single-level problem p of `solver`: loss = sum over the samples k (after
    steps every, 2 every, ...) of sum over the gauge cells of
    (eta1 - target_k)^2, with a frozen dt sequence."""

    def __init__(self, solver, p, eta2_0, dts, every, gauge, targets, ckpt=20):
        self.S = solver
        self.L = solver.L
        self.p = p
        self.eta2 = float(eta2_0)
        self.dts = np.ascontiguousarray(dts, dtype=np.float64)
        self.every = int(every)
        self.gauge = tuple(int(x) for x in gauge)
        self.targets = targets  # device tensor [n_samples][gn][gn]
        self.ckpt = int(ckpt)
        nx, ny = solver.shapes[p][0][:2]
        self.nx, self.ny = nx, ny
        self._pool = None  # states of one recomputed segment, allocated once

    def _buffers(self):
        if self._pool is None:
            self._pool = [torch.empty((6, self.ny, self.nx), dtype=torch.float64, device="cuda")
                          for _ in range(self.ckpt)]
        return self._pool

    def _check(self, rc):
        self.S._check(rc)

    def _run(self, s0, s1):
        if s1 > s0:
            d = self.dts[s0:s1]
            self._check(self.L.mlswe_run_fixed(self.S.h, self.p, s1 - s0,
                                               d.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))

    def _state(self, out=None):
        q = out if out is not None else torch.empty((6, self.ny, self.nx), dtype=torch.float64, device="cuda")
        self._check(self.L.mlswe_get_state(self.S.h, self.p, 0, _vp(q), binding.DEVICE))
        return q

    def _set_state(self, q):
        self._check(self.L.mlswe_set_state(self.S.h, self.p, 0, _vp(q), binding.DEVICE))

    def _gauge(self, k, q, loss=None, lam=None, Bbar=None):
        i0, j0, gn = self.gauge
        tgt = self.targets[k]
        self._check(self.L.mlswe_gauge_misfit(
            self.S.h, self.p, _vp(q) if q is not None else None, i0, j0, gn, _vp(tgt),
            _vp(loss) if loss is not None else None, _vp(lam) if lam is not None else None,
            _vp(Bbar) if Bbar is not None else None))

    def forward(self, eta1_0, B):
        """Loss (device scalar tensor) and the checkpoints of the run."""
        _vp(eta1_0)
        _vp(B)
        self.S.set_bathymetry(self.p, B)
        q0 = torch.empty((6, self.ny, self.nx), dtype=torch.float64, device="cuda")
        self._check(self.L.mlswe_param_map(self.S.h, self.p, _vp(eta1_0), self.eta2, _vp(q0)))
        self._set_state(q0)
        loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        ckpts = [q0]
        n = len(self.dts)
        s = 0
        while s < n:
            nxt = min(n, (s // self.every + 1) * self.every, (s // self.ckpt + 1) * self.ckpt)
            self._run(s, nxt)
            s = nxt
            if s % self.every == 0:
                self._gauge(s // self.every - 1, None, loss=loss)
            if s % self.ckpt == 0 and s < n:
                ckpts.append(self._state())
        return loss, ckpts

    def backward(self, eta1_0, ckpts):
        n = len(self.dts)
        lam = torch.zeros((6, self.ny, self.nx), dtype=torch.float64, device="cuda")
        lam2 = torch.empty_like(lam)
        Bbar = torch.zeros((self.ny, self.nx), dtype=torch.float64, device="cuda")
        nseg = (n + self.ckpt - 1) // self.ckpt
        for seg in reversed(range(nseg)):
            s0, s1 = seg * self.ckpt, min(n, (seg + 1) * self.ckpt)
            self._set_state(ckpts[seg])
            pool = self._buffers()
            states = [ckpts[seg]]
            for s in range(s0, s1):
                self._run(s, s + 1)
                states.append(self._state(pool[s - s0]))
            for s in reversed(range(s0, s1)):
                if (s + 1) % self.every == 0:
                    self._gauge((s + 1) // self.every - 1, states[s + 1 - s0], lam=lam, Bbar=Bbar)
                self._check(self.L.mlswe_adjoint_step(self.S.h, self.p, _vp(states[s - s0]), _vp(lam), _vp(lam2),
                                                      _vp(Bbar), float(self.dts[s])))
                lam, lam2 = lam2, lam
        eta1_bar = torch.empty((self.ny, self.nx), dtype=torch.float64, device="cuda")
        self._check(self.L.mlswe_param_map_adjoint(self.S.h, self.p, _vp(eta1_0), self.eta2, _vp(lam),
                                                   _vp(eta1_bar), _vp(Bbar)))
        return eta1_bar, Bbar


class GaugeMisfit(torch.autograd.Function):
    """loss = GaugeMisfit.apply(eta1_0, B, problem) with eta1_0, B float64 CUDA
    tensors [ny][nx]; backward gives d loss / d eta1_0 and d loss / d B."""

    @staticmethod
    def forward(ctx, eta1_0, B, problem):
        e = eta1_0.detach().contiguous()
        b = B.detach().contiguous()
        loss, ckpts = problem.forward(e, b)
        ctx.problem = problem
        ctx.ckpts = ckpts
        ctx.save_for_backward(e, b)
        return loss.reshape(())

    @staticmethod
    def backward(ctx, g):
        e, b = ctx.saved_tensors
        pr = ctx.problem
        pr.S.set_bathymetry(pr.p, b)
        eb, bb = pr.backward(e, ctx.ckpts)
        return g * eb, g * bb, None
