"""torch.autograd.Function over hjpd_value_grad (linear-tanh family).

HJValue.apply(x, t, N, hp, Q, solver) returns phi [n] after exactly
`solver.max_iter` iterations of the splitting (fixed-iteration mode); its
backward calls hjpd_value_grad, which differentiates through those iterations
on the GPU (checkpoints every `ckpt_every` iterations) and returns gradients
for x [n, d], hp = [eps, A] [1 + d*d] and Q [d*d].
"""
from __future__ import annotations

import torch

from . import hjpd as C
from .solver import Solver


class LinearTanhValue:
    """Context for H = -<p, A x + eps tanh x> + |p|^2/2, g = x^T Q x / 2 (float32)."""

    def __init__(self, d, N_max, sigma, tau, K, ckpt_every=50, theta=1.0, seed=0, timing=False):
        self.K, self.ckpt_every = int(K), int(ckpt_every)
        self.solver = Solver(d=d, H=C.HJPD_H_LINEAR_TANH, g=C.HJPD_G_QUAD_FORM, N_max=N_max, sigma=sigma, tau=tau,
                             theta=theta, tol=1e-30, max_iter=K, seed=seed, dtype=torch.float32, fixed_iters=True,
                             timing=timing)
        self.d = d

    def value(self, x, t, N, hp, Q):
        return self.solver.solve(x, t, N, hp, Q).phi

    def value_grad(self, x, t, N, hp, Q, grad_phi, stream=None):
        n = t.numel()
        dev = x.device
        phi = torch.empty(n, dtype=torch.float32, device=dev)
        dx = torch.empty(n, self.d, dtype=torch.float32, device=dev)
        dh = torch.empty(1 + self.d * self.d, dtype=torch.float32, device=dev)
        dg = torch.empty(self.d * self.d, dtype=torch.float32, device=dev)
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        C.hjpd_value_grad(self.solver.ctx, n, x, t, N, hp, Q, grad_phi.contiguous(), self.K, self.ckpt_every, phi,
                          dx, dh, dg, stream)
        return phi, dx, dh, dg

    def close(self):
        self.solver.close()


class HJValue(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, t, N, hp, Q, lt: LinearTanhValue):
        x, hp, Q = x.contiguous(), hp.contiguous(), Q.contiguous()
        ctx.save_for_backward(x, t, N, hp, Q)
        ctx.lt = lt
        return lt.value(x, t, N, hp, Q)

    @staticmethod
    def backward(ctx, grad_phi):
        x, t, N, hp, Q = ctx.saved_tensors
        _, dx, dh, dg = ctx.lt.value_grad(x, t, N, hp, Q, grad_phi.to(torch.float32))
        return dx, None, None, dh, dg, None


def hj_value(x, t, N, eps, A, Q, lt: LinearTanhValue):
    """phi(x, t) for the linear-tanh family; differentiable in x, eps, A and Q."""
    hp = torch.cat([eps.reshape(1), A.reshape(-1)])
    return HJValue.apply(x, t, N, hp, Q.reshape(-1), lt)
