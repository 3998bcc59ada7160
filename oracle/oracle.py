"""Python access to the FP64 CPU oracle — TEST INFRASTRUCTURE ONLY.

The oracle (``hjpd_oracle.c``) is a plain sequential double-precision
implementation of the primal-dual splitting of Lin, Chow and Osher
(arXiv 1803.01215, section 5.1 Algorithm 1 and Appendix A.1.1 for optimal
control; Algorithm 3 and Appendix A.2.1 for games).  Only ``tests/``, the
smoke check and the CPU-baseline leg of the benchmark may import this module.
It shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hjpd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

H_CNORM, H_QUADROTOR, H_PURSUIT_EVASION, H_LINEAR_TANH = 0, 1, 2, 3
G_NORM, G_QUAD_SHIFT, G_PAIR_DIST, G_QUAD_FORM = 0, 1, 2, 3
PT_CONVERGED, PT_MAXITER, PT_NONFINITE, PT_BADINPUT = 0, 1, 2, 3
ARR_X, ARR_P, ARR_Y, ARR_Q = 0, 1, 2, 3


# Rounding variants of the same source (see the C file's header): the oracle
# itself ("f64"), binary64 with FMA contraction, and binary32 without / with
# FMA contraction.  The variants only measure rounding floors for the parity
# tests; every reference value comes from "f64".
_VARIANT_FLAGS = {
    "f64": [],
    "f64fma": ["-mfma", "-ffp-contract=fast"],
    "f32": ["-DOR_BINARY32", "-fsingle-precision-constant"],
    "f32fma": ["-DOR_BINARY32", "-fsingle-precision-constant", "-mfma", "-ffp-contract=fast"],
}


# HJPD_ORACLE_SANITIZE=1: every build is instrumented with AddressSanitizer and
# UndefinedBehaviorSanitizer (any finding aborts) and kept apart from the plain
# builds; the process must preload the sanitizer runtimes (tests/test_sanitizers.py).
_SANITIZE = os.environ.get("HJPD_ORACLE_SANITIZE") == "1"
_SANITIZE_FLAGS = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                   "-fno-sanitize-recover=undefined"]


def _lib_path(variant: str) -> str:
    if _SANITIZE:
        return os.path.join(_HERE, "liboracle_%s_sanitized.so" % variant)
    return _LIB if variant == "f64" else os.path.join(_HERE, "liboracle_%s.so" % variant)


def build(force: bool = False, variant: str = "f64") -> str:
    """Compile the oracle with gcc (plain -O2, OpenMP across points only);
    `variant` selects one of the rounding variants."""
    path = _lib_path(variant)
    if force or not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
        tmp = path + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", *_VARIANT_FLAGS[variant],
                               *(_SANITIZE_FLAGS if _SANITIZE else []), "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, path)
    return path


def build_all(force: bool = False) -> None:
    for v in _VARIANT_FLAGS:
        build(force, v)


class _Problem(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int), ("g", ctypes.c_int), ("d", ctypes.c_int), ("d_y", ctypes.c_int),
                ("hp", ctypes.POINTER(ctypes.c_double)), ("gp", ctypes.POINTER(ctypes.c_double))]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        D = ctypes.POINTER(ctypes.c_double)
        I = ctypes.POINTER(ctypes.c_int)
        P = ctypes.POINTER(_Problem)
        _lib.or_solve.argtypes = [P, ctypes.c_long, D, D, I, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(ctypes.c_int64),
                                  D, I, I, D, D, ctypes.c_int]
        _lib.or_solve.restype = ctypes.c_int
        _lib.or_solve_hopf.argtypes = _lib.or_solve.argtypes
        _lib.or_solve_hopf.restype = ctypes.c_int
        _lib.or_solve_recipe.argtypes = [P, ctypes.c_long, D, D, I, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_uint64,
                                         ctypes.c_int, ctypes.POINTER(ctypes.c_int64), ctypes.c_int, ctypes.c_int,
                                         ctypes.c_double, ctypes.c_double, D, I, I, D, D, ctypes.c_int]
        _lib.or_solve_recipe.restype = ctypes.c_int
        _lib.or_solve_mix.argtypes = [P, ctypes.c_long, D, D, I, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(ctypes.c_int64),
                                      ctypes.c_double, ctypes.c_double, D, I, I, D, D, ctypes.c_int]
        _lib.or_solve_mix.restype = ctypes.c_int
        for nm, at in [("or_isaacs_H", [D, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double]),
                       ("or_saddle_estar", [D, ctypes.c_double]), ("or_saddle_hstar", [D, ctypes.c_double]),
                       ("or_saddle_g", [D, ctypes.c_double, ctypes.c_double]),
                       ("or_isaacs_dual_p", [D, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                             ctypes.c_double, ctypes.c_int]),
                       ("or_isaacs_dual_q", [D, D, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                             ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                             ctypes.c_int])]:
            getattr(_lib, nm).argtypes = at
            getattr(_lib, nm).restype = ctypes.c_double
        _lib.or_gstar.argtypes = [P, D]
        _lib.or_gstar.restype = ctypes.c_double
        _lib.or_hopf_prox1.argtypes = [P, D, D, ctypes.c_double, ctypes.c_double, D]
        _lib.or_hopf_prox1.restype = ctypes.c_int
        _lib.or_splitmix64_mix.argtypes = [ctypes.c_uint64]
        _lib.or_splitmix64_mix.restype = ctypes.c_uint64
        _lib.or_splitmix64_at.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        _lib.or_splitmix64_at.restype = ctypes.c_uint64
        _lib.or_init_noise.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        _lib.or_init_noise.restype = ctypes.c_double
        _lib.or_shrink2.argtypes = [D, ctypes.c_double, ctypes.c_int, D]
        _lib.or_H.argtypes = [P, D, D, ctypes.c_double]
        _lib.or_H.restype = ctypes.c_double
        _lib.or_grad_x_H.argtypes = [P, D, D, ctypes.c_double, D]
        _lib.or_prox_p.argtypes = [P, D, D, ctypes.c_double, ctypes.c_double, D]
        _lib.or_g.argtypes = [P, D]
        _lib.or_g.restype = ctypes.c_double
        _lib.or_prox_g.argtypes = [P, D, ctypes.c_double, D]
        _lib.or_prox_g.restype = ctypes.c_int
        _lib.or_game_H.argtypes = [P, D, D, D, D]
        _lib.or_game_H.restype = ctypes.c_double
        _lib.or_game_prox_p.argtypes = [P, D, D, D, D, ctypes.c_double, D]
        _lib.or_game_prox_q.argtypes = [P, D, D, D, D, ctypes.c_double, D]
        _lib.or_game_grad_x.argtypes = [P, D, D, D, D, D]
        _lib.or_game_grad_y.argtypes = [P, D, D, D, D, D]
        _lib.or_game_prox_x0.argtypes = [P, D, D, ctypes.c_double, D]
        _lib.or_game_stretch_y0.argtypes = [P, D, D, ctypes.c_double, D]
    return _lib


_vlibs = {}


def _variant_lib(variant: str):
    """ctypes handle of a rounding variant's batch solvers (binary32 variants
    take float arrays and float scalars where the oracle takes double)."""
    if variant == "f64":
        return lib()
    if variant not in _vlibs:
        L = ctypes.CDLL(build(variant=variant))
        R = ctypes.c_float if variant.startswith("f32") else ctypes.c_double
        Rp = ctypes.POINTER(R)
        I = ctypes.POINTER(ctypes.c_int)

        class _P(ctypes.Structure):
            _fields_ = [("H", ctypes.c_int), ("g", ctypes.c_int), ("d", ctypes.c_int), ("d_y", ctypes.c_int),
                        ("hp", Rp), ("gp", Rp)]
        L.Problem = _P
        L.real = np.float32 if variant.startswith("f32") else np.float64
        L.or_solve.argtypes = [ctypes.POINTER(_P), ctypes.c_long, Rp, Rp, I, R, R, R, R, ctypes.c_int, ctypes.c_int,
                               ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(ctypes.c_int64), Rp, I, I, Rp, Rp,
                               ctypes.c_int]
        L.or_solve.restype = ctypes.c_int
        L.or_solve_hopf.argtypes = L.or_solve.argtypes
        L.or_solve_hopf.restype = ctypes.c_int
        L.or_solve_mix.argtypes = [ctypes.POINTER(_P), ctypes.c_long, Rp, Rp, I, R, R, R, R, ctypes.c_int,
                                   ctypes.c_int, ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(ctypes.c_int64), R, R,
                                   Rp, I, I, Rp, Rp, ctypes.c_int]
        L.or_solve_mix.restype = ctypes.c_int
        L.or_solve_recipe.argtypes = [ctypes.POINTER(_P), ctypes.c_long, Rp, Rp, I, R, R, R, R, ctypes.c_int,
                                      ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(ctypes.c_int64), ctypes.c_int,
                                      ctypes.c_int, R, R, Rp, I, I, Rp, Rp, ctypes.c_int]
        L.or_solve_recipe.restype = ctypes.c_int
        _vlibs[variant] = L
    return _vlibs[variant]


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class Problem:
    """One problem family instance: Hamiltonian H, initial cost g and their parameters."""
    H: int
    g: int
    d: int
    d_y: int
    hp: np.ndarray
    gp: np.ndarray

    def __post_init__(self):
        self.hp = np.ascontiguousarray(self.hp, dtype=np.float64).ravel()
        self.gp = np.ascontiguousarray(self.gp, dtype=np.float64).ravel()
        self._c = _Problem(self.H, self.g, self.d, self.d_y, _dp(self.hp), _dp(self.gp))

    @property
    def c(self):
        return ctypes.byref(self._c)

    # --- point-wise pieces (for pinning tests) ---
    def H_val(self, x, p, s=0.0):
        x = np.ascontiguousarray(x, np.float64); p = np.ascontiguousarray(p, np.float64)
        return lib().or_H(self.c, _dp(x), _dp(p), s)

    def grad_x_H(self, x, p, s=0.0):
        x = np.ascontiguousarray(x, np.float64); p = np.ascontiguousarray(p, np.float64)
        out = np.zeros(self.d)
        lib().or_grad_x_H(self.c, _dp(x), _dp(p), s, _dp(out))
        return out

    def prox_p(self, x, v, lam, s=0.0):
        x = np.ascontiguousarray(x, np.float64); v = np.ascontiguousarray(v, np.float64)
        out = np.zeros(self.d)
        lib().or_prox_p(self.c, _dp(x), _dp(v), lam, s, _dp(out))
        return out

    def g_val(self, x0):
        x0 = np.ascontiguousarray(x0, np.float64)
        return lib().or_g(self.c, _dp(x0))

    def prox_g(self, v, tau):
        v = np.ascontiguousarray(v, np.float64)
        out = np.zeros(self.d)
        assert lib().or_prox_g(self.c, _dp(v), tau, _dp(out)) == 0
        return out

    def gstar(self, p):
        p = np.ascontiguousarray(p, np.float64)
        return lib().or_gstar(self.c, _dp(p))

    def hopf_prox1(self, x1, v, sigma, delta):
        x1 = np.ascontiguousarray(x1, np.float64); v = np.ascontiguousarray(v, np.float64)
        out = np.zeros(self.d)
        assert lib().or_hopf_prox1(self.c, _dp(x1), _dp(v), sigma, delta, _dp(out)) == 0
        return out

    def game_H(self, x, y, p, q):
        a = [np.ascontiguousarray(z, np.float64) for z in (x, y, p, q)]
        return lib().or_game_H(self.c, *[_dp(z) for z in a])

    def _game_vec(self, fn, n_out, *args):
        a = [np.ascontiguousarray(z, np.float64) if isinstance(z, (np.ndarray, list, tuple)) else z for z in args]
        out = np.zeros(n_out)
        conv = [(_dp(z) if isinstance(z, np.ndarray) else z) for z in a]
        fn(self.c, *conv, _dp(out))
        return out

    def game_prox_p(self, x, y, q, v, lam):
        return self._game_vec(lib().or_game_prox_p, self.d - self.d_y, x, y, q, v, lam)

    def game_prox_q(self, x, y, p, v, lam):
        return self._game_vec(lib().or_game_prox_q, self.d_y, x, y, p, v, lam)

    def game_grad_x(self, x, y, p, q):
        return self._game_vec(lib().or_game_grad_x, self.d - self.d_y, x, y, p, q)

    def game_grad_y(self, x, y, p, q):
        return self._game_vec(lib().or_game_grad_y, self.d_y, x, y, p, q)

    def game_prox_x0(self, v, y0, tau):
        return self._game_vec(lib().or_game_prox_x0, self.d - self.d_y, v, y0, tau)

    def game_stretch_y0(self, v, x0, tau):
        return self._game_vec(lib().or_game_stretch_y0, self.d_y, v, x0, tau)


@dataclass
class Result:
    phi: np.ndarray
    iters: np.ndarray
    status: np.ndarray
    x_traj: np.ndarray | None
    p_traj: np.ndarray | None


# Hamiltonian weights (wl, wr) of the interval (j-1, j): H at its left and right node.
DISC_WEIGHTS = {"be": (0.0, 1.0), "fe": (1.0, 0.0), "trap": (0.5, 0.5)}


def solve_variant(variant: str, pb: Problem, x, t, N, *, sigma, tau, theta=1.0, tol=1e-8, max_iter=5000,
                  fixed_iters=False, seed=0, N_max=None, ids=None, traj=False, threads=0, hopf=False,
                  disc="be", starts=1, restarts=0, sigma_inc=0.0, value_tol=0.0) -> Result:
    """solve() (Algorithms 1 to 3, the Hopf formulation, the weighted
    discretisations, the recipes) in one of the rounding variants: "f64fma",
    "f32" or "f32fma".  Binary32 variants take their inputs rounded to
    binary32; results are returned as float64 arrays."""
    rec = dict(starts=starts, restarts=restarts, sigma_inc=sigma_inc, value_tol=value_tol)
    recipe = starts > 1 or restarts > 0 or value_tol > 0.0
    if variant == "f64":
        return solve(pb, x, t, N, sigma=sigma, tau=tau, theta=theta, tol=tol, max_iter=max_iter,
                     fixed_iters=fixed_iters, seed=seed, N_max=N_max, ids=ids, traj=traj, threads=threads, hopf=hopf,
                     disc=disc, **rec)
    if recipe and (hopf or fixed_iters or disc != "be"):
        raise ValueError("oracle: recipes are for the Lax path in tolerance mode")
    L = _variant_lib(variant)
    R = L.real
    Rp = ctypes.POINTER(ctypes.c_float if R == np.float32 else ctypes.c_double)
    rp = lambda a: a.ctypes.data_as(Rp)  # noqa: E731
    hp = np.ascontiguousarray(pb.hp, R)
    gp = np.ascontiguousarray(pb.gp, R)
    P = L.Problem(pb.H, pb.g, pb.d, pb.d_y, rp(hp), rp(gp))
    x = np.ascontiguousarray(np.asarray(x, np.float64).reshape(-1, pb.d), R)
    n = x.shape[0]
    t = np.ascontiguousarray(np.broadcast_to(np.asarray(t, np.float64), (n,)), R)
    N = np.ascontiguousarray(np.broadcast_to(np.asarray(N, np.int32), (n,))).astype(np.int32)
    if N_max is None:
        N_max = int(N.max()) if n else 1
    phi = np.zeros(n, R); iters = np.zeros(n, np.int32); status = np.zeros(n, np.int32)
    xt = np.zeros((n, N_max + 1, pb.d), R) if traj else None
    pt = np.zeros((n, N_max + 1, pb.d), R) if traj else None
    idp = None
    if ids is not None:
        ids = np.ascontiguousarray(ids, np.int64)
        idp = ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    I = ctypes.POINTER(ctypes.c_int)
    common = (ctypes.byref(P), n, rp(x), rp(t), N.ctypes.data_as(I), sigma, tau, theta, tol, int(max_iter),
              int(bool(fixed_iters)), int(seed) & (2**64 - 1), int(N_max), idp)
    outs = (rp(phi), iters.ctypes.data_as(I), status.ctypes.data_as(I), rp(xt) if traj else None,
            rp(pt) if traj else None, int(threads))
    if recipe:
        rc = L.or_solve_recipe(ctypes.byref(P), n, rp(x), rp(t), N.ctypes.data_as(I), sigma, tau, theta, tol,
                               int(max_iter), int(seed) & (2**64 - 1), int(N_max), idp, int(starts), int(restarts),
                               float(sigma_inc), float(value_tol), *outs)
    elif disc != "be":
        wl, wr = (float(v) for v in (DISC_WEIGHTS.get(disc, disc) if isinstance(disc, str) else disc))
        rc = L.or_solve_mix(*common, wl, wr, *outs)
    else:
        rc = (L.or_solve_hopf if hopf else L.or_solve)(*common, *outs)
    if rc != 0:
        raise ValueError("oracle: unsupported problem")
    f = lambda a: None if a is None else a.astype(np.float64)  # noqa: E731
    return Result(f(phi), iters, status, f(xt), f(pt))


def solve(pb: Problem, x, t, N, *, sigma, tau, theta=1.0, tol=1e-8, max_iter=5000, fixed_iters=False,
          seed=0, N_max=None, ids=None, traj=False, threads=0, hopf=False, starts=1, restarts=0, sigma_inc=0.0,
          value_tol=0.0, disc="be") -> Result:
    """Run the oracle over a batch of points.

    x: [n, d]; t: [n]; N: [n] (intervals per point).  ids: each point's
    index in the full workload (selects its random start), default 0..n-1.
    In fixed-iteration mode exactly max_iter iterations are run (unless a
    non-finite value stops the point first).  hopf=True runs the Hopf
    formulation (Algorithm 2; eikonal family with NORM or QUAD_SHIFT g); its
    trajectories have node 0 = 0.  starts / restarts / sigma_inc / value_tol
    select the robustness recipes (tolerance mode; control path, and the
    pursuit-evasion game with starts = 1): see the
    C source's header comment.  disc selects the time discretisation of the
    Lax path: "be" backward Euler (Algorithm 1), "fe" forward Euler,
    "trap" the trapezoidal average of the two (eikonal and quadrotor
    families), or a pair
    (wl, wr) of Hamiltonian weights; "be" is Algorithm 1 itself, any other
    value runs the weighted-discretisation solver.
    """
    x = np.ascontiguousarray(x, np.float64).reshape(-1, pb.d)
    n = x.shape[0]
    t = np.ascontiguousarray(np.broadcast_to(np.asarray(t, np.float64), (n,)))
    N = np.ascontiguousarray(np.broadcast_to(np.asarray(N, np.int32), (n,))).astype(np.int32)
    if N_max is None:
        N_max = int(N.max()) if n else 1
    phi = np.zeros(n); iters = np.zeros(n, np.int32); status = np.zeros(n, np.int32)
    xt = np.zeros((n, N_max + 1, pb.d)) if traj else None
    pt = np.zeros((n, N_max + 1, pb.d)) if traj else None
    idp = None
    if ids is not None:
        ids = np.ascontiguousarray(ids, np.int64)
        idp = ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    I = ctypes.POINTER(ctypes.c_int)
    weights = DISC_WEIGHTS.get(disc, disc) if isinstance(disc, str) else tuple(disc)
    if disc != "be":
        if hopf or starts > 1 or restarts > 0 or value_tol > 0.0:
            raise ValueError("oracle: the weighted discretisations are for the plain Lax control path")
        wl, wr = (float(w) for w in weights)
        rc = lib().or_solve_mix(pb.c, n, _dp(x), _dp(t), N.ctypes.data_as(I), sigma, tau, theta, tol,
                                int(max_iter), int(bool(fixed_iters)), int(seed) & (2**64 - 1), int(N_max), idp,
                                wl, wr, _dp(phi), iters.ctypes.data_as(I), status.ctypes.data_as(I),
                                _dp(xt) if traj else None, _dp(pt) if traj else None, int(threads))
    elif starts > 1 or restarts > 0 or value_tol > 0.0:
        if hopf or fixed_iters:
            raise ValueError("oracle: recipes are for the Lax path in tolerance mode")
        rc = lib().or_solve_recipe(pb.c, n, _dp(x), _dp(t), N.ctypes.data_as(I), sigma, tau, theta, tol,
                                   int(max_iter), int(seed) & (2**64 - 1), int(N_max), idp, int(starts),
                                   int(restarts), float(sigma_inc), float(value_tol), _dp(phi),
                                   iters.ctypes.data_as(I), status.ctypes.data_as(I),
                                   _dp(xt) if traj else None, _dp(pt) if traj else None, int(threads))
    else:
        fn = lib().or_solve_hopf if hopf else lib().or_solve
        rc = fn(pb.c, n, _dp(x), _dp(t), N.ctypes.data_as(I), sigma, tau, theta, tol, int(max_iter),
                int(bool(fixed_iters)), int(seed) & (2**64 - 1), int(N_max), idp, _dp(phi),
                iters.ctypes.data_as(I), status.ctypes.data_as(I),
                _dp(xt) if traj else None, _dp(pt) if traj else None, int(threads))
    if rc != 0:
        raise ValueError("oracle: unsupported problem")
    return Result(phi, iters, status, xt, pt)


def init_noise(seed, point, arr, j, i):
    return lib().or_init_noise(int(seed) & (2**64 - 1), int(point), arr, j, i)


def splitmix64_at(seed, k):
    return lib().or_splitmix64_at(int(seed) & (2**64 - 1), int(k))


def shrink2(v, lam):
    v = np.ascontiguousarray(v, np.float64)
    out = np.zeros_like(v)
    lib().or_shrink2(_dp(v), lam, v.size, _dp(out))
    return out
