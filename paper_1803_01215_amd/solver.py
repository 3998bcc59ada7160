"""Torch-facing wrapper over the C ABI: allocates outputs, checks tensors.

All numerical work happens in libhjpd's kernels.  Tensors must already be on
the GPU with the context's dtype; nothing is moved or converted here, and a
missing library or a CPU tensor is an error.
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from . import hjpd as C


@dataclass
class SolveOutput:
    phi: torch.Tensor
    iters: torch.Tensor
    status: torch.Tensor
    x_traj: torch.Tensor | None
    p_traj: torch.Tensor | None


def _need(t, name, dtype, numel=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a GPU tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if numel is not None and t.numel() != numel:
        raise ValueError("%s must have %d elements, got %d" % (name, numel, t.numel()))


_DISC_FLAGS = {"be": 0, "fe": C.HJPD_FORWARD_EULER, "trap": C.HJPD_TRAPEZOID}


class Solver:
    """One hjpd context (problem families, dimension, dtype, step sizes)."""

    def __init__(self, *, d, H, g, N_max, sigma, tau, theta=1.0, tol=1e-6, max_iter=20000, seed=0, d_y=0,
                 dtype=torch.float32, plain=False, fixed_iters=False, graph=False, timing=False,
                 lanes_per_point=0, nodes_per_lane=0, order_hint=True, hopf=False, starts=1, restarts=0,
                 sigma_inc=0.0, value_tol=0.0, disc="be", refill=True):
        # disc: time discretisation of the Lax saddle, "be" backward Euler (Algorithm 1),
        # "fe" forward Euler, "trap" trapezoid (eikonal family)
        if disc not in _DISC_FLAGS:
            raise ValueError("disc must be one of %s" % sorted(_DISC_FLAGS))
        self.dtype = dtype
        self.d, self.N_max = d, N_max
        flags = ((C.HJPD_PLAIN if plain else 0) | (C.HJPD_FIXED_ITERS if fixed_iters else 0)
                 | (C.HJPD_GRAPH if graph else 0) | (C.HJPD_TIMING if timing else 0)
                 | (0 if order_hint else C.HJPD_NO_ORDER_HINT) | (C.HJPD_HOPF if hopf else 0)
                 | _DISC_FLAGS[disc] | (0 if refill else C.HJPD_NO_REFILL))
        self.desc = C.hjpd_desc(d=d, d_y=d_y, H=H, g=g, dtype=C.HJPD_F64 if dtype == torch.float64 else C.HJPD_F32,
                                N_max=N_max, sigma=sigma, tau=tau, theta=theta, tol=tol, max_iter=max_iter,
                                seed=seed & (2**64 - 1), flags=flags, lanes_per_point=lanes_per_point,
                                nodes_per_lane=nodes_per_lane, starts=starts, restarts=restarts, sigma_inc=sigma_inc,
                                value_tol=value_tol)
        self.ctx = C.hjpd_create(self.desc)

    def close(self):
        if self.ctx:
            C.hjpd_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def alloc(self, n, traj=False, device="cuda"):
        dev = torch.device(device)
        out = SolveOutput(torch.empty(n, dtype=self.dtype, device=dev), torch.empty(n, dtype=torch.int32, device=dev),
                          torch.full((n,), -1, dtype=torch.int32, device=dev), None, None)
        if traj:
            out.x_traj = torch.zeros(n, self.N_max + 1, self.d, dtype=self.dtype, device=dev)
            out.p_traj = torch.zeros(n, self.N_max + 1, self.d, dtype=self.dtype, device=dev)
        return out

    def _check_inputs(self, x, t, N, hp, gp):
        n = t.numel()
        _need(x, "x", self.dtype, n * self.d)
        _need(t, "t", self.dtype)
        _need(N, "N", torch.int32, n)
        _need(hp, "h_params", self.dtype)
        _need(gp, "g_params", self.dtype)
        return n

    def solve(self, x, t, N, h_params, g_params, traj=False, out: SolveOutput | None = None, stream=None):
        n = self._check_inputs(x, t, N, h_params, g_params)
        if out is None:
            out = self.alloc(n, traj, x.device)
        if stream is None:
            stream = torch.cuda.current_stream(x.device)
        C.hjpd_solve_batch(self.ctx, n, x, t, N, h_params, g_params, out.phi, out.x_traj, out.p_traj, out.iters,
                           out.status, stream)
        return out

    def autotune(self, x, t, N, h_params, g_params, probe_iters=200, stream=None):
        n = self._check_inputs(x, t, N, h_params, g_params)
        scratch = self.alloc(n, False, x.device)
        if stream is None:
            stream = torch.cuda.current_stream(x.device)
        C.hjpd_autotune(self.ctx, n, x, t, N, h_params, g_params, scratch.phi, scratch.iters, scratch.status,
                        probe_iters, stream)

    def timing(self):
        return C.hjpd_get_timing(self.ctx)

    def plan(self):
        """([(hi, L, K), ...], from_cache): the persistent path's capacity classes and tiles."""
        return C.hjpd_get_plan(self.ctx)

    def set_plan(self, classes):
        C.hjpd_set_plan(self.ctx, classes)

    def set_pop_counter(self, counts):
        """counts: zeroed int32 GPU tensor with one entry per point (None turns counting off)."""
        if counts is not None:
            _need(counts, "counts", torch.int32)
        C.hjpd_set_pop_counter(self.ctx, counts)

    def launch_timings(self):
        """Per persistent launch of the last timed eager solve: dicts with ms,
        the N range of its capacity class and its tile."""
        _, nl = C.hjpd_get_timing(self.ctx)
        out = []
        for i in range(nl):
            ms, lo, hi, L, K = C.hjpd_get_launch_timing(self.ctx, i)
            out.append({"ms": ms, "N_lo": lo, "N_hi": hi, "L": L, "K": K})
        return out
