"""Seeded synthetic workloads shaped like the paper's examples.

This module only draws inputs (query points, horizons, step counts and
problem parameters) from NumPy's PCG64 generator.  It holds none of the
method's arithmetic, so both the GPU path and the oracle may use it.

Six workloads:
  eikonal2d   2-D eikonal H = ||p||, g = ||x|| - 1, t = 1, N = 16, 256 points,
              x ~ U[-2,2]^2 (section 6.1 family, closed form known).
  cnorm10     d = 10, H = c(x)||p||, c = 1 + 0.5 sin(x1) cos(x2),
              g = ||x - a||^2/2 - 1, a ~ N(0,I), t ~ U[0.2,1], N = 32,
              65,536 points x ~ N(0,I) (state-dependent eikonal, section 6.1).
  quadrotor12 12-state quadrotor-like control, cost |u|^2/2,
              g = ||x||^2/2, x ~ U[-1,1]^12, t ~ U[0.5,3], N = ceil(t/0.05),
              131,072 points (section 6.4 analogue).
  pursuit12   pursuit-evasion game of two 3-D point masses with drag 0.1,
              g = ||r_P - r_E|| - 0.5, r ~ U[-2,2]^3, v ~ U[-0.5,0.5]^3,
              t ~ U[0.5,4], N = clamp(ceil(24 t), 16, 96), 262,144 points
              (section 6.2 / Algorithm 3 analogue).
  lintanh100  d = 100, H_c = <p, Ax + 0.1 tanh x> - ||p||^2/2, A ~ N(0,1/d),
              g = x^T Q x / 2, Q = M M^T/d + 0.5 I, x ~ N(0,I), t = 1, N = 50,
              16,384 points, 500 fixed iterations (differentiation workload).
  isaacs2     Isaacs' game of section 6.3 with the convex-concave initial cost:
              x, y scalars, H = -c(x,y) q + 2|p| - sqrt(p^2+q^2) - 1, bump
              speed c, g = (2.5 x)^2/2 - 1/2 - y^2/2; the section's 73 x 73 grid
              on [-3,3]^2 at t = 0.025, 0.05, 0.075, 0.1 (delta = 0.005),
              21,316 points (game Hopf formulation, Algorithm 4).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Family ids (same numbering as the public C header).
H_CNORM, H_QUADROTOR, H_PURSUIT_EVASION, H_LINEAR_TANH, H_ISAACS = 0, 1, 2, 3, 4
G_NORM, G_QUAD_SHIFT, G_PAIR_DIST, G_QUAD_FORM, G_SADDLE_QUAD = 0, 1, 2, 3, 4

SEED_BASE = 1803 * 10


@dataclass
class Workload:
    name: str
    index: int
    H: int
    g: int
    d: int
    d_y: int
    n: int
    N_max: int
    dtype: str            # "f32" or "f64" (the configuration's primary precision)
    sigma: float
    tau: float
    theta: float
    tol: float
    max_iter: int
    fixed_iters: bool
    x: np.ndarray         # [n, d] float64
    t: np.ndarray         # [n] float64
    N: np.ndarray         # [n] int32
    hp: np.ndarray        # Hamiltonian parameters (float64)
    gp: np.ndarray        # initial-cost parameters (float64)
    init_seed: int = 0
    extra: dict = field(default_factory=dict)

    def subset(self, idx) -> "Workload":
        idx = np.asarray(idx)
        w = Workload(**{k: getattr(self, k) for k in self.__dataclass_fields__})
        w.x, w.t, w.N = self.x[idx], self.t[idx], self.N[idx]
        w.n = int(len(idx))
        w.extra = dict(self.extra, ids=np.asarray(self.extra.get("ids", np.arange(self.n)))[idx])
        return w

    @property
    def ids(self) -> np.ndarray:
        return np.asarray(self.extra.get("ids", np.arange(self.n)), dtype=np.int64)


def _rng(index: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + index))


def eikonal2d(n: int = 256) -> Workload:
    r = _rng(0)
    x = r.uniform(-2.0, 2.0, size=(n, 2))
    sigma = 8.0
    return Workload("eikonal2d", 0, H_CNORM, G_NORM, 2, 0, n, 16, "f64", sigma, 0.25 / sigma, 1.0, 1e-8, 5000,
                    False, x, np.full(n, 1.0), np.full(n, 16, np.int32), np.array([0.0]), np.array([1.0]),
                    init_seed=SEED_BASE + 100)


def cnorm10(n: int = 65536, alpha: float = 0.5) -> Workload:
    r = _rng(1)
    d = 10
    a = r.standard_normal(d)
    x = r.standard_normal((n, d))
    t = r.uniform(0.2, 1.0, size=n)
    sigma = 1.0
    gp = np.concatenate([[1.0], a])
    return Workload("cnorm10", 1, H_CNORM, G_QUAD_SHIFT, d, 0, n, 32, "f32", sigma, 0.25 / sigma, 1.0, 1e-6,
                    20000, False, x, t, np.full(n, 32, np.int32), np.array([alpha]), gp,
                    init_seed=SEED_BASE + 101)


QUAD_PARAMS = np.array([0.5, 4.5e-3, 4.5e-3, 8.1e-3, 9.81, 1.3])  # m, J1, J2, J3, g_z, pitch clamp


def quadrotor12(n: int = 131072) -> Workload:
    r = _rng(2)
    x = r.uniform(-1.0, 1.0, size=(n, 12))
    t = r.uniform(0.5, 3.0, size=n)
    N = np.ceil(t / 0.05).astype(np.int32)
    sigma = 2.0
    gp = np.zeros(13)  # c0 = 0, x_goal = 0
    return Workload("quadrotor12", 2, H_QUADROTOR, G_QUAD_SHIFT, 12, 0, n, 60, "f32", sigma, 0.25 / sigma, 1.0,
                    1e-6, 20000, False, x, t, N, QUAD_PARAMS.copy(), gp, init_seed=SEED_BASE + 102)


PE_PARAMS = np.array([0.1, 1.0, 0.25])  # kappa, pursuer control weight, evader control weight


def pursuit12(n: int = 262144) -> Workload:
    r = _rng(3)
    rp = r.uniform(-2.0, 2.0, size=(n, 3))
    vp = r.uniform(-0.5, 0.5, size=(n, 3))
    re = r.uniform(-2.0, 2.0, size=(n, 3))
    ve = r.uniform(-0.5, 0.5, size=(n, 3))
    x = np.concatenate([rp, vp, re, ve], axis=1)
    t = r.uniform(0.5, 4.0, size=n)
    N = np.clip(np.ceil(24.0 * t), 16, 96).astype(np.int32)
    sigma = 32.0
    return Workload("pursuit12", 3, H_PURSUIT_EVASION, G_PAIR_DIST, 12, 6, n, 96, "f32", sigma, 0.25 / sigma, 1.0,
                    1e-6, 20000, False, x, t, N, PE_PARAMS.copy(), np.array([0.5]), init_seed=SEED_BASE + 103)


def lintanh100(n: int = 16384, eps: float = 0.1) -> Workload:
    r = _rng(4)
    d = 100
    A = r.standard_normal((d, d)) / math.sqrt(d)
    M = r.standard_normal((d, d))
    Q = M @ M.T / d + 0.5 * np.eye(d)
    x = r.standard_normal((n, d))
    sigma = 1.0
    hp = np.concatenate([[eps], A.ravel()])
    return Workload("lintanh100", 4, H_LINEAR_TANH, G_QUAD_FORM, d, 0, n, 50, "f32", sigma, 0.25 / sigma, 1.0,
                    1e-6, 500, True, x, np.full(n, 1.0), np.full(n, 50, np.int32), hp, Q.ravel().copy(),
                    init_seed=SEED_BASE + 104, extra={"A": A, "Q": Q})


# Isaacs' game of section 6.3: bump speed c = b0 (1 + b1 exp(-b2 |(x,y) - (cx,cy)|^2)) and the
# convex-concave initial cost (a x)^2/2 - c0 - (b y)^2/2.
ISAACS_PARAMS = np.array([2.0, 3.0, 4.0, 1.0, 1.0])   # b0, b1, b2, cx, cy
ISAACS_G = np.array([0.5, 2.5, 1.0])                   # c0, a, b


def isaacs2(n: int | None = None, mesh: float = 1.0 / 12.0) -> Workload:
    """Section 6.3's grid: [-3,3]^2 with spacing 1/12 (73 x 73 points) at the
    four times 0.025, 0.05, 0.075, 0.1 with delta = 0.005 (N = 5, 10, 15, 20),
    times major.  n (optional) keeps a seeded random subset of that many
    points, in grid order, as a batch of its own (random starts keyed by the
    position in that batch)."""
    g = np.arange(-3.0, 3.0 + 0.5 * mesh, mesh)
    X, Y = np.meshgrid(g, g, indexing="ij")
    xy = np.stack([X.ravel(), Y.ravel()], axis=1)
    times = np.array([0.025, 0.05, 0.075, 0.1])
    x = np.tile(xy, (len(times), 1))
    t = np.repeat(times, len(xy))
    N = np.round(t / 0.005).astype(np.int32)
    if n is not None and n < len(x):
        keep = np.sort(_rng(5).choice(len(x), n, replace=False))
        x, t, N = x[keep], t[keep], N[keep]
    sigma = 2.0
    return Workload("isaacs2", 5, H_ISAACS, G_SADDLE_QUAD, 2, 1, len(x), 20, "f32", sigma, 0.25 / sigma, 1.0,
                    1e-8, 20000, False, x, t, N, ISAACS_PARAMS.copy(), ISAACS_G.copy(), init_seed=SEED_BASE + 105)


ALL = {"eikonal2d": eikonal2d, "cnorm10": cnorm10, "quadrotor12": quadrotor12, "pursuit12": pursuit12,
       "lintanh100": lintanh100, "isaacs2": isaacs2}


def get(name: str, n: int | None = None) -> Workload:
    f = ALL[name]
    return f() if n is None else f(n)
