"""Pins of the FP64 oracle against things other than itself.

Each test checks the oracle against a fact the paper or plain mathematics
fixes: a published generator test vector, the proximal-map definition (eq.
prox) solved by brute force, the Hamiltonian as a max/min over controls
(section 2) evaluated by brute force on dynamics written independently here,
central differences, the classical Hopf-Lax closed form (section 2.1), the
discrete Riccati recursion of the linear-quadratic case, the envelope identity
of the discrete saddle, direct shooting of the discretised control problem
(section 4.1), and stationarity of an independently written Lagrangian.
"""
import os

import numpy as np
import pytest
from scipy.optimize import minimize

import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def _rng(k):
    return np.random.default_rng(9000 + k)


# --------------------------------------------------------------------------
# Random start generator
# --------------------------------------------------------------------------

def test_splitmix64_matches_published_vectors(oracle_mod):
    vals = [int(l) for l in open(os.path.join(HERE, "golden", "splitmix64_seed1234567.txt"))
            if l.strip() and not l.startswith("#")]
    got = [oracle_mod.splitmix64_at(1234567, k) for k in range(1, 6)]
    assert got == vals


def test_init_noise_range_and_spread(oracle_mod):
    v = np.array([oracle_mod.init_noise(77, pt, arr, j, i)
                  for pt in range(8) for arr in range(4) for j in range(6) for i in range(5)])
    assert v.min() >= -0.1 and v.max() < 0.1
    assert abs(v.mean()) < 0.01
    assert len(np.unique(v)) == v.size
    # uniform on [-0.1, 0.1]: variance 0.01/3
    assert abs(v.var() - 0.01 / 3) < 0.0008


# --------------------------------------------------------------------------
# Dynamics written independently of the oracle (physical, forward time).
# --------------------------------------------------------------------------

def _rot(axis, a):
    c, s = np.cos(a), np.sin(a)
    if axis == "x":
        return np.array([[1, 0, 0], [0, c, -s], [0, s, c]])
    if axis == "y":
        return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])


def quad_f_phys(x, u, hp):
    """Quadrotor-like dynamics: r' = v, v' = (u1/m) R e3 - g e3, eta' = W omega,
    omega' = J^{-1} u_{2:4}; R = Rz(psi) Ry(theta) Rx(phi); W is the inverse of
    the map from Euler-angle rates to body rates, pitch clamped inside it."""
    m, J, gz, clamp = hp[0], hp[1:4], hp[4], hp[5]
    v, eta, om = x[3:6], x[6:9], x[9:12]
    ph, th, ps = eta
    R = _rot("z", ps) @ _rot("y", th) @ _rot("x", ph)
    thc = np.clip(th, -clamp, clamp)
    E = np.array([[1, 0, -np.sin(thc)],
                  [0, np.cos(ph), np.sin(ph) * np.cos(thc)],
                  [0, -np.sin(ph), np.cos(ph) * np.cos(thc)]])
    Wm = np.linalg.inv(E)
    f = np.zeros(12)
    f[0:3] = v
    f[3:6] = (u[0] / m) * R[:, 2] - gz * np.array([0, 0, 1.0])
    f[6:9] = Wm @ om
    f[9:12] = u[1:4] / J
    return f


def pe_f_phys(X, uP, uE, kappa):
    def pm(s, u):
        v = s[3:6]
        return np.concatenate([v, -kappa * np.linalg.norm(v) * v + u])
    return np.concatenate([pm(X[0:6], uP), pm(X[6:12], uE)])


def lt_f_phys(x, u, A, eps):
    return A @ x + eps * np.tanh(x) + u


def H_by_max_over_controls(f_phys, L, p, m_u, rng):
    """Paper's initial-value Hamiltonian H = max_u <-f_phys(u), p> - L(u)
    (time-reversed dynamics, section 2.1), by numerical maximisation."""
    obj = lambda u: -(np.dot(-f_phys(u), p) - L(u))
    best = None
    for _ in range(3):
        r = minimize(obj, rng.standard_normal(m_u), method="BFGS", options={"gtol": 1e-11})
        if best is None or r.fun < best.fun:
            best = r
    return -best.fun


# --------------------------------------------------------------------------
# Hamiltonians vs brute force over the controls
# --------------------------------------------------------------------------

def test_cnorm_H_is_max_over_unit_ball(oracle_mod):
    rng = _rng(1)
    alpha = 0.5
    pb = oracle_mod.Problem(W.H_CNORM, W.G_NORM, 3, 0, [alpha], [1.0])
    for _ in range(20):
        x, p = rng.standard_normal(3), rng.standard_normal(3)
        c = 1 + alpha * np.sin(x[0]) * np.cos(x[1])
        # max over ||u|| <= 1 of <c u, p>: dense sampling of the sphere, then polish
        u = rng.standard_normal((200000, 3))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        brute = (c * u @ p).max()
        h = pb.H_val(x, p)
        assert brute <= h + 1e-12
        assert h - brute < 1e-3 * np.linalg.norm(p) * c
        # exact maximiser u = p/|p| attains it
        assert abs(c * np.linalg.norm(p) - h) < 1e-12


def test_quadrotor_H_is_max_over_controls(oracle_mod):
    rng = _rng(2)
    hp = W.QUAD_PARAMS
    pb = oracle_mod.Problem(W.H_QUADROTOR, W.G_QUAD_SHIFT, 12, 0, hp, np.zeros(13))
    for _ in range(12):
        x = rng.uniform(-1, 1, 12)
        x[7] = rng.uniform(-1.6, 1.6)  # pitch on both sides of the clamp
        p = rng.standard_normal(12) * np.array([1, 1, 1, 1, 1, 1, 1, 1, 1, 0.01, 0.01, 0.01])
        brute = H_by_max_over_controls(lambda u: quad_f_phys(x, u, hp), lambda u: 0.5 * u @ u, p, 4, rng)
        assert abs(brute - pb.H_val(x, p)) < 1e-8 * max(1, abs(brute))


def test_pursuit_H_is_minmax_over_controls_and_isaacs(oracle_mod):
    rng = _rng(3)
    kappa, wP, wE = W.PE_PARAMS
    pb = oracle_mod.Problem(W.H_PURSUIT_EVASION, W.G_PAIR_DIST, 12, 6, W.PE_PARAMS, [0.5])
    for _ in range(10):
        X = rng.uniform(-1, 1, 12)
        p, q = rng.standard_normal(6), rng.standard_normal(6)
        P = np.concatenate([p, -q])  # full costate (p, -q), section 4.2
        # terminal-value H_c = min_uP max_uE <P, f> + |uP|^2/2 - |uE|^2/(2 wE)
        def inner_max(uP):
            obj = lambda uE: -(P @ pe_f_phys(X, uP, uE, kappa) + 0.5 * uP @ uP - 0.5 / wE * uE @ uE)
            return -minimize(obj, np.zeros(3), method="BFGS", options={"gtol": 1e-11}).fun
        minmax = minimize(inner_max, np.zeros(3), method="BFGS", options={"gtol": 1e-10}).fun

        def inner_min(uE):
            obj = lambda uP: P @ pe_f_phys(X, uP, uE, kappa) + 0.5 * uP @ uP - 0.5 / wE * uE @ uE
            return minimize(obj, np.zeros(3), method="BFGS", options={"gtol": 1e-11}).fun
        maxmin = -minimize(lambda uE: -inner_min(uE), np.zeros(3), method="BFGS", options={"gtol": 1e-10}).fun
        assert abs(minmax - maxmin) < 1e-7  # Isaacs condition holds
        H_paper = -minmax                   # initial-value convention
        assert abs(H_paper - pb.game_H(X[:6], X[6:], p, q)) < 1e-7
        assert abs(H_paper - pb.H_val(X, P)) < 1e-7


def test_linear_tanh_H_is_max_over_controls(oracle_mod):
    rng = _rng(4)
    d, eps = 5, 0.1
    A = rng.standard_normal((d, d)) / np.sqrt(d)
    pb = oracle_mod.Problem(W.H_LINEAR_TANH, W.G_QUAD_FORM, d, 0, np.concatenate([[eps], A.ravel()]), np.eye(d))
    for _ in range(10):
        x, p = rng.standard_normal(d), rng.standard_normal(d)
        brute = H_by_max_over_controls(lambda u: lt_f_phys(x, u, A, eps), lambda u: 0.5 * u @ u, p, d, rng)
        assert abs(brute - pb.H_val(x, p)) < 1e-8 * max(1, abs(brute))


# --------------------------------------------------------------------------
# Gradients in x vs central differences
# --------------------------------------------------------------------------

def _fd_grad(f, x, h=1e-6):
    g = np.zeros_like(x)
    for i in range(x.size):
        e = np.zeros_like(x); e[i] = h
        g[i] = (f(x + e) - f(x - e)) / (2 * h)
    return g


@pytest.mark.parametrize("family", ["cnorm", "quadrotor", "lintanh"])
def test_grad_x_H_matches_central_differences(oracle_mod, family):
    rng = _rng(5)
    if family == "cnorm":
        pb = oracle_mod.Problem(W.H_CNORM, W.G_NORM, 4, 0, [0.7], [1.0]); d = 4
    elif family == "quadrotor":
        pb = oracle_mod.Problem(W.H_QUADROTOR, W.G_QUAD_SHIFT, 12, 0, W.QUAD_PARAMS, np.zeros(13)); d = 12
    else:
        d = 6
        A = rng.standard_normal((d, d))
        pb = oracle_mod.Problem(W.H_LINEAR_TANH, W.G_QUAD_FORM, d, 0, np.concatenate([[0.3], A.ravel()]), np.eye(d))
    for _ in range(15):
        x, p = rng.uniform(-1.2, 1.2, d), rng.standard_normal(d)
        if family == "quadrotor":
            x[7] = rng.choice([rng.uniform(-1.25, 1.25), rng.uniform(1.35, 1.5)])
            p[9:] *= 0.01  # keeps |H| moderate so differences are not rounding-bound
        g = pb.grad_x_H(x, p)
        fd = _fd_grad(lambda z: pb.H_val(z, p), x)
        assert np.max(np.abs(g - fd)) < 1e-6 * max(1, np.max(np.abs(fd)))


def test_game_grads_match_central_differences(oracle_mod):
    rng = _rng(6)
    pb = oracle_mod.Problem(W.H_PURSUIT_EVASION, W.G_PAIR_DIST, 12, 6, W.PE_PARAMS, [0.5])
    for _ in range(15):
        x, y, p, q = rng.uniform(-1, 1, 6), rng.uniform(-1, 1, 6), rng.standard_normal(6), rng.standard_normal(6)
        gx = pb.game_grad_x(x, y, p, q)
        gy = pb.game_grad_y(x, y, p, q)
        assert np.allclose(gx, _fd_grad(lambda z: pb.game_H(z, y, p, q), x), atol=1e-7)
        assert np.allclose(gy, _fd_grad(lambda z: pb.game_H(x, z, p, q), y), atol=1e-7)
        # full-state gradient in the (X, P) form agrees
        g = pb.grad_x_H(np.concatenate([x, y]), np.concatenate([p, -q]))
        assert np.allclose(g, np.concatenate([gx, gy]), atol=1e-12)


# --------------------------------------------------------------------------
# Proximal maps vs their definition (eq. prox), by brute-force minimisation
# --------------------------------------------------------------------------

def _argmin(obj, x0, rng, starts=4):
    best = None
    for k in range(starts):
        s = x0 if k == 0 else x0 + 0.3 * rng.standard_normal(x0.size)
        r = minimize(obj, s, method="Powell", options={"xtol": 1e-12, "ftol": 1e-15, "maxfev": 200000})
        if best is None or r.fun < best.fun:
            best = r
    return best


def test_shrink2_is_prox_of_scaled_norm(oracle_mod):
    rng = _rng(7)
    for _ in range(20):
        v = rng.standard_normal(4) * rng.choice([0.1, 1, 3])
        lam = rng.uniform(0.05, 2)
        out = oracle_mod.shrink2(v, lam)
        obj = lambda y: lam * np.linalg.norm(y) + 0.5 * np.sum((y - v) ** 2)
        r = _argmin(obj, v.copy(), rng)
        assert obj(out) <= r.fun + 1e-10
        assert np.allclose(out, r.x, atol=1e-5)
    assert np.all(oracle_mod.shrink2(np.zeros(3), 0.5) == 0)


@pytest.mark.parametrize("family", ["cnorm", "quadrotor", "lintanh"])
def test_prox_p_is_argmin(oracle_mod, family):
    rng = _rng(8)
    if family == "cnorm":
        d = 3
        pb = oracle_mod.Problem(W.H_CNORM, W.G_NORM, d, 0, [0.5], [1.0])
        Hf = lambda x, p: (1 + 0.5 * np.sin(x[0]) * np.cos(x[1])) * np.linalg.norm(p)
    elif family == "quadrotor":
        d = 12
        hp = W.QUAD_PARAMS
        pb = oracle_mod.Problem(W.H_QUADROTOR, W.G_QUAD_SHIFT, d, 0, hp, np.zeros(13))
        # H = -<p, f0> + |B^T p|^2/2, with f0 and B from the independent dynamics
        def Hf(x, p):
            f0 = quad_f_phys(x, np.zeros(4), hp)
            B = np.stack([quad_f_phys(x, e, hp) - f0 for e in np.eye(4)], axis=1)
            return -p @ f0 + 0.5 * np.sum((B.T @ p) ** 2)
    else:
        d = 4
        A = rng.standard_normal((d, d))
        pb = oracle_mod.Problem(W.H_LINEAR_TANH, W.G_QUAD_FORM, d, 0, np.concatenate([[0.2], A.ravel()]), np.eye(d))
        Hf = lambda x, p: -p @ (A @ x + 0.2 * np.tanh(x)) + 0.5 * p @ p
    for _ in range(8):
        x, v = rng.uniform(-1, 1, d), rng.standard_normal(d)
        lam = rng.uniform(0.01, 0.5) if family != "quadrotor" else rng.uniform(1e-6, 1e-4)
        out = pb.prox_p(x, v, lam)
        obj = lambda p: lam * Hf(x, p) + 0.5 * np.sum((p - v) ** 2)
        if family == "cnorm":
            r = _argmin(obj, v.copy(), rng)
            assert obj(out) <= r.fun + 1e-10
            assert np.allclose(out, r.x, atol=1e-5)
        else:
            # smooth strongly convex objective: its gradient vanishes at the prox
            g = _fd_grad(obj, out, h=1e-6)
            assert np.max(np.abs(g)) < 1e-6 * max(1, np.max(np.abs(v)))


def test_prox_g_is_argmin(oracle_mod):
    rng = _rng(9)
    d = 4
    a = rng.standard_normal(d)
    Q = rng.standard_normal((d, d))
    Q = Q @ Q.T + np.eye(d) + 0.3 * rng.standard_normal((d, d))  # not symmetric: g uses (Q+Q^T)/2
    cases = [
        (oracle_mod.Problem(W.H_CNORM, W.G_NORM, d, 0, [0.0], [1.5]), lambda y: np.linalg.norm(y) - 1.5),
        (oracle_mod.Problem(W.H_CNORM, W.G_QUAD_SHIFT, d, 0, [0.0], np.concatenate([[1.0], a])),
         lambda y: 0.5 * np.sum((y - a) ** 2) - 1.0),
        (oracle_mod.Problem(W.H_LINEAR_TANH, W.G_QUAD_FORM, d, 0, np.zeros(1 + d * d), Q.ravel()),
         lambda y: 0.5 * y @ Q @ y),
    ]
    for pb, gf in cases:
        for _ in range(6):
            v, tau = rng.standard_normal(d) * 2, rng.uniform(0.05, 1.0)
            assert abs(pb.g_val(v) - gf(v)) < 1e-12
            out = pb.prox_g(v, tau)
            obj = lambda y: tau * gf(y) + 0.5 * np.sum((y - v) ** 2)
            r = _argmin(obj, v.copy(), rng)
            assert obj(out) <= r.fun + 1e-10
            assert np.allclose(out, r.x, atol=1e-5)


def test_game_node0_maps_are_argmin_argmax(oracle_mod):
    rng = _rng(10)
    pb = oracle_mod.Problem(W.H_PURSUIT_EVASION, W.G_PAIR_DIST, 12, 6, W.PE_PARAMS, [0.5])
    g = lambda x, y: np.linalg.norm(x[:3] - y[:3]) - 0.5
    for _ in range(6):
        v, y0, x0 = rng.uniform(-1, 1, 6), rng.uniform(-1, 1, 6), rng.uniform(-1, 1, 6)
        tau = rng.uniform(0.005, 0.2)
        assert abs(pb.g_val(np.concatenate([x0, y0])) - g(x0, y0)) < 1e-12
        out = pb.game_prox_x0(v, y0, tau)
        obj = lambda x: tau * g(x, y0) + 0.5 * np.sum((x - v) ** 2)
        r = _argmin(obj, v.copy(), rng)
        assert obj(out) <= r.fun + 1e-10 and np.allclose(out, r.x, atol=1e-5)
        out = pb.game_stretch_y0(v, x0, tau)
        obj = lambda y: -tau * g(x0, y) + 0.5 * np.sum((y - v) ** 2)
        r = _argmin(obj, v.copy(), rng)
        assert obj(out) <= r.fun + 1e-10 and np.allclose(out, r.x, atol=1e-5)
    # tie-break at v = r_P: move by tau along e_1
    x0 = np.array([0.3, -0.2, 0.1, 0, 0, 0.0])
    out = pb.game_stretch_y0(x0.copy(), x0, 0.1)
    assert np.allclose(out[:3], x0[:3] + [0.1, 0, 0])


# --------------------------------------------------------------------------
# Whole-path pins
# --------------------------------------------------------------------------

def test_eikonal_matches_hopf_lax_closed_form(oracle_mod):
    """H = ||p||, g = ||x|| - 1: the discrete problem is min over ||x_0 - x|| <= t
    of g(x_0) exactly, i.e. phi = max(||x|| - t, 0) - 1 (classical Lax formula,
    section 2.1).  For ||x|| > t the minimiser x_0 = x (1 - t/||x||) is unique and
    every multiplier equals x/||x||."""
    w = W.eikonal2d(64)
    pb = oracle_mod.Problem(w.H, w.g, w.d, w.d_y, w.hp, w.gp)
    r = oracle_mod.solve(pb, w.x, w.t, w.N, sigma=w.sigma, tau=w.tau, tol=1e-26, max_iter=30000,
                         seed=w.init_seed, traj=True)
    nx = np.linalg.norm(w.x, axis=1)
    exact = np.maximum(nx - w.t, 0) - 1
    assert np.max(np.abs(r.phi - exact)) < 1e-9
    far = nx > w.t + 0.05
    x0_exact = w.x * (1 - w.t / nx)[:, None]
    assert np.max(np.abs(r.x_traj[far, 0, :] - x0_exact[far])) < 1e-6
    assert np.max(np.abs(r.p_traj[far, -1, :] - (w.x / nx[:, None])[far])) < 1e-6
    # default tolerance of the workload: value still within 1e-6
    r2 = oracle_mod.solve(pb, w.x, w.t, w.N, sigma=w.sigma, tau=w.tau, tol=w.tol, max_iter=w.max_iter,
                          seed=w.init_seed)
    assert np.all(r2.status == 0)
    assert np.max(np.abs(r2.phi - exact)) < 1e-6


@pytest.mark.parametrize("variant,bound", [("f64fma", 1e-12), ("f32", 2e-5), ("f32fma", 2e-5)])
def test_rounding_variants_compute_the_same_method(oracle_mod, variant, bound):
    """The oracle's rounding variants (binary64 with FMA contraction, binary32
    without and with it), which the parity tests use to measure rounding
    floors, run the same iteration: on the eikonal workload, whose value is
    the classical Lax closed form, each reaches max(||x|| - t, 0) - 1 to its
    precision, and at a fixed iteration count each stays within its
    precision of the binary64 oracle."""
    w = W.eikonal2d(64)
    pb = oracle_mod.Problem(w.H, w.g, w.d, w.d_y, w.hp, w.gp)
    exact = np.maximum(np.linalg.norm(w.x, axis=1) - w.t, 0) - 1
    tol = 1e-26 if variant == "f64fma" else 1e-10
    r = oracle_mod.solve_variant(variant, pb, w.x, w.t, w.N, sigma=w.sigma, tau=w.tau, tol=tol, max_iter=30000,
                                 seed=w.init_seed, traj=True)
    assert np.max(np.abs(r.phi - exact)) < (1e-9 if variant == "f64fma" else 5e-5)
    # fixed count, against the oracle itself
    K = 400
    a = oracle_mod.solve(pb, w.x, w.t, w.N, sigma=w.sigma, tau=w.tau, max_iter=K, fixed_iters=True,
                         seed=w.init_seed, traj=True)
    b = oracle_mod.solve_variant(variant, pb, w.x, w.t, w.N, sigma=w.sigma, tau=w.tau, max_iter=K,
                                 fixed_iters=True, seed=w.init_seed, traj=True)
    assert np.all(b.iters == K)
    assert np.max(np.abs(a.phi - b.phi)) < bound
    assert np.max(np.abs(a.x_traj - b.x_traj)) < 10 * bound
    # a planted difference in the arithmetic is not hidden by the comparison
    c = oracle_mod.solve_variant(variant, pb, w.x, w.t, w.N, sigma=1.01 * w.sigma, tau=w.tau, max_iter=K,
                                 fixed_iters=True, seed=w.init_seed, traj=True)
    assert np.max(np.abs(a.phi - c.phi)) > 10 * bound


def test_cnorm_constant_speed_matches_closed_form(oracle_mod):
    """c = 1 (alpha = 0), g = ||x-a||^2/2 - 1: phi = max(||x - a|| - t, 0)^2/2 - 1 exactly."""
    w = W.cnorm10(48, alpha=0.0)
    pb = oracle_mod.Problem(w.H, w.g, w.d, w.d_y, w.hp, w.gp)
    r = oracle_mod.solve(pb, w.x, w.t, w.N, sigma=w.sigma, tau=w.tau, tol=1e-26, max_iter=40000,
                         seed=w.init_seed)
    a = w.gp[1:]
    exact = 0.5 * np.maximum(np.linalg.norm(w.x - a, axis=1) - w.t, 0) ** 2 - 1
    assert np.max(np.abs(r.phi - exact)) < 1e-9


def test_linear_quadratic_matches_discrete_riccati(oracle_mod):
    """eps = 0: H = -<p, A x> + |p|^2/2, g = x^T Q x/2.  Eliminating p_j gives
    min sum |M x_j - x_{j-1}|^2/(2 delta) + g(x_0), M = I + delta A, whose value is
    x^T P_N x / 2 with P_0 = Q_s, P_j = M^T P_{j-1} (I + delta P_{j-1})^{-1} M."""
    rng = _rng(11)
    d, N, t = 6, 12, 0.8
    A = rng.standard_normal((d, d)) / np.sqrt(d)  # not symmetric: catches A vs A^T
    Mq = rng.standard_normal((d, d))
    Q = Mq @ Mq.T / d + 0.5 * np.eye(d)
    pb = oracle_mod.Problem(W.H_LINEAR_TANH, W.G_QUAD_FORM, d, 0, np.concatenate([[0.0], A.ravel()]), Q.ravel())
    x = rng.standard_normal((6, d))
    r = oracle_mod.solve(pb, x, t, N, sigma=1.0, tau=0.25, tol=1e-28, max_iter=20000, seed=5)
    delta = t / N
    M = np.eye(d) + delta * A
    P = Q.copy()
    for _ in range(N):
        P = M.T @ P @ np.linalg.solve(np.eye(d) + delta * P, M)
    exact = 0.5 * np.einsum("ni,ij,nj->n", x, P, x)
    assert np.max(np.abs(r.phi - exact) / np.maximum(1, np.abs(exact))) < 1e-10


def _envelope_check(oracle_mod, pb, x, t, N, sigma, h=1e-5, tol=1e-28, max_iter=30000, rtol=1e-6):
    r = oracle_mod.solve(pb, x[None], t, N, sigma=sigma, tau=0.25 / sigma, tol=tol, max_iter=max_iter,
                         seed=3, traj=True)
    pN = r.p_traj[0, N]
    delta = t / N
    env = pN - delta * pb.grad_x_H(x, pN, t)
    fd = np.zeros_like(x)
    for i in range(x.size):
        e = np.zeros_like(x); e[i] = h
        rp = oracle_mod.solve(pb, (x + e)[None], t, N, sigma=sigma, tau=0.25 / sigma, tol=tol, max_iter=max_iter, seed=3)
        rm = oracle_mod.solve(pb, (x - e)[None], t, N, sigma=sigma, tau=0.25 / sigma, tol=tol, max_iter=max_iter, seed=3)
        fd[i] = (rp.phi[0] - rm.phi[0]) / (2 * h)
    assert np.max(np.abs(env - fd)) < rtol * max(1, np.max(np.abs(fd))), (env, fd)


def test_envelope_identity_state_dependent_eikonal(oracle_mod):
    """grad_x phi_delta = p_N - delta grad_x H(x, p_N): the value is the
    Lagrangian at a stationary point and x enters only as x_N."""
    rng = _rng(12)
    w = W.cnorm10(4)
    pb = oracle_mod.Problem(w.H, w.g, w.d, w.d_y, w.hp, w.gp)
    for k in range(2):
        _envelope_check(oracle_mod, pb, w.x[k], float(w.t[k]), 32, w.sigma)


def test_envelope_identity_linear_tanh(oracle_mod):
    rng = _rng(13)
    d = 5
    A = rng.standard_normal((d, d)) / np.sqrt(d)
    Q = np.eye(d) + 0.2 * np.ones((d, d))
    pb = oracle_mod.Problem(W.H_LINEAR_TANH, W.G_QUAD_FORM, d, 0, np.concatenate([[0.1], A.ravel()]), Q.ravel())
    _envelope_check(oracle_mod, pb, rng.standard_normal(d), 1.0, 10, 1.0)


def _shoot_min(f_phys_step, g, x, N, t, m_u, rng, starts=4, bounds_unit_ball=False):
    """Direct shooting of the backward-Euler discretisation (section 4.1):
    from x_N = x, x_{j-1} = x_j + delta f_phys(x_j, u_j) (physical time runs
    from node N down to node 0), cost g(x_0) + delta sum_j L(u_j)."""
    delta = t / N

    def cost(U):
        U = U.reshape(N, m_u)
        s = x.copy()
        run = 0.0
        for j in range(N, 0, -1):
            f, L = f_phys_step(s, U[j - 1])
            s = s + delta * f
            run += delta * L
        return g(s) + run
    best = None
    for k in range(starts):
        U0 = 0.1 * rng.standard_normal(N * m_u)
        if bounds_unit_ball:
            cons = [{"type": "ineq", "fun": (lambda U, j=j: 1.0 - np.sum(U.reshape(N, m_u)[j] ** 2))} for j in range(N)]
            r = minimize(cost, U0, method="SLSQP", constraints=cons, options={"ftol": 1e-14, "maxiter": 2000})
        else:
            r = minimize(cost, U0, method="BFGS", options={"gtol": 1e-10})
        if best is None or r.fun < best.fun:
            best = r
    return best.fun


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_state_dependent_eikonal_matches_direct_shooting(oracle_mod, N):
    """alpha != 0: phi equals the minimum over feasible discrete trajectories
    (speed c(x_j) with ||u_j|| <= 1), found by SLSQP from several starts."""
    rng = _rng(14 + N)
    alpha, d = 0.5, 2
    a = np.array([0.4, -0.3])
    pb = oracle_mod.Problem(W.H_CNORM, W.G_QUAD_SHIFT, d, 0, [alpha], np.concatenate([[1.0], a]))
    c = lambda z: 1 + alpha * np.sin(z[0]) * np.cos(z[1])
    g = lambda z: 0.5 * np.sum((z - a) ** 2) - 1.0
    step = lambda s, u: (c(s) * u, 0.0)
    for _ in range(3):
        x = rng.uniform(-1.5, 1.5, d)
        t = rng.uniform(0.2, 0.8)
        r = oracle_mod.solve(pb, x[None], t, N, sigma=1.0, tau=0.25, tol=1e-26, max_iter=40000, seed=1)
        assert r.status[0] == 0
        brute = _shoot_min(step, g, x, N, t, d, rng, bounds_unit_ball=True)
        assert abs(r.phi[0] - brute) < 1e-6, (r.phi[0], brute)


@pytest.mark.parametrize("N", [1, 2, 3])
def test_quadrotor_matches_direct_shooting(oracle_mod, N):
    rng = _rng(20 + N)
    hp = W.QUAD_PARAMS
    pb = oracle_mod.Problem(W.H_QUADROTOR, W.G_QUAD_SHIFT, 12, 0, hp, np.zeros(13))
    g = lambda z: 0.5 * z @ z
    step = lambda s, u: (quad_f_phys(s, u, hp), 0.5 * u @ u)
    for _ in range(2):
        x = rng.uniform(-0.5, 0.5, 12)
        t = 0.05 * N
        r = oracle_mod.solve(pb, x[None], t, N, sigma=2.0, tau=0.125, tol=1e-26, max_iter=60000, seed=2)
        brute = _shoot_min(step, g, x, N, t, 4, rng)
        assert abs(r.phi[0] - brute) < 1e-6 * max(1, abs(brute)), (r.phi[0], brute)


def test_linear_tanh_matches_direct_shooting(oracle_mod):
    rng = _rng(30)
    d, N, t, eps = 3, 3, 0.6, 0.4
    A = rng.standard_normal((d, d))
    Q = np.diag([1.0, 2.0, 0.5])
    pb = oracle_mod.Problem(W.H_LINEAR_TANH, W.G_QUAD_FORM, d, 0, np.concatenate([[eps], A.ravel()]), Q.ravel())
    step = lambda s, u: (lt_f_phys(s, u, A, eps), 0.5 * u @ u)
    for _ in range(3):
        x = rng.standard_normal(d)
        r = oracle_mod.solve(pb, x[None], t, N, sigma=1.0, tau=0.25, tol=1e-28, max_iter=20000, seed=4)
        brute = _shoot_min(step, lambda z: 0.5 * z @ Q @ z, x, N, t, d, rng)
        assert abs(r.phi[0] - brute) < 1e-7 * max(1, abs(brute))


def _pe_lagrangian(Z, N, dx, dy, hp, x_t, y_t, gp, delta):
    """Lagrangian of eq. discgenlaxhopfdg written independently: free variables
    x_0..x_{N-1}, y_0..y_{N-1}, p_1..p_N, q_1..q_N; H from the independent
    dynamics at the full costate (p, -q)."""
    kappa, wP, wE = hp
    o = 0
    xs = Z[o:o + N * dx].reshape(N, dx); o += N * dx
    ys = Z[o:o + N * dy].reshape(N, dy); o += N * dy
    ps = Z[o:o + N * dx].reshape(N, dx); o += N * dx
    qs = Z[o:o + N * dy].reshape(N, dy)
    xs = np.vstack([xs, x_t]); ys = np.vstack([ys, y_t])
    L = np.linalg.norm(xs[0, :3] - ys[0, :3]) - gp[0]
    for j in range(1, N + 1):
        X = np.concatenate([xs[j], ys[j]])
        P = np.concatenate([ps[j - 1], -qs[j - 1]])
        f0 = pe_f_phys(X, np.zeros(3), np.zeros(3), kappa)
        Hc = P @ f0 - 0.5 * wP * P[3:6] @ P[3:6] + 0.5 * wE * P[9:12] @ P[9:12]
        L += ps[j - 1] @ (xs[j] - xs[j - 1]) - qs[j - 1] @ (ys[j] - ys[j - 1]) - delta * (-Hc)
    return L


def test_pursuit_fixed_point_is_stationary_for_independent_lagrangian(oracle_mod):
    """Parity beyond H for the game is pinned by first-order optimality: at the
    oracle's converged iterate, the Lagrangian written independently above has
    zero gradient in every free block."""
    rng = _rng(31)
    pb = oracle_mod.Problem(W.H_PURSUIT_EVASION, W.G_PAIR_DIST, 12, 6, W.PE_PARAMS, [0.5])
    for _ in range(2):
        X = np.concatenate([rng.uniform(-1, 1, 3), rng.uniform(-.3, .3, 3), rng.uniform(-1, 1, 3) + 2,
                            rng.uniform(-.3, .3, 3)])
        N, t = 6, 0.3
        r = oracle_mod.solve(pb, X[None], t, N, sigma=8.0, tau=0.25 / 8, tol=1e-28, max_iter=200000, seed=6,
                             traj=True)
        xt, pt = r.x_traj[0], r.p_traj[0]
        Z = np.concatenate([xt[:N, :6].ravel(), xt[:N, 6:].ravel(), pt[1:, :6].ravel(), pt[1:, 6:].ravel()])
        Lf = lambda z: _pe_lagrangian(z, N, 6, 6, W.PE_PARAMS, X[:6], X[6:], [0.5], t / N)
        g = _fd_grad(Lf, Z, h=1e-6)
        assert np.max(np.abs(g)) < 1e-6, np.max(np.abs(g))
        # and the value is the Lagrangian there
        assert abs(Lf(Z) - r.phi[0]) < 1e-10


def _pe_shoot_minmax(X, N, t, r, hp, UP=None, UE=None):
    """Direct shooting of the discretised game: from X_N = X, X_{j-1} = X_j +
    delta f_phys(X_j, uP_j, uE_j); payoff g(X_0) + delta sum_j (|uP_j|^2/(2 wP)
    - |uE_j|^2/(2 wE)).  The two players' states evolve independently, so the
    open-loop value is min over uP of max over uE (the inner problem is
    strictly concave where the pair is apart, the outer one convex).  With UP
    and UE given, returns the payoff of those controls instead."""
    kappa, wP, wE = hp
    delta = t / N

    def G(up, ue):
        up, ue = up.reshape(N, 3), ue.reshape(N, 3)
        s, run = X.copy(), 0.0
        for j in range(N, 0, -1):
            s = s + delta * pe_f_phys(s, up[j - 1], ue[j - 1], kappa)
            run += delta * (0.5 / wP * up[j - 1] @ up[j - 1] - 0.5 / wE * ue[j - 1] @ ue[j - 1])
        return np.linalg.norm(s[0:3] - s[6:9]) - r + run
    if UP is not None:
        return G(UP, UE)

    def inner(up):
        return -minimize(lambda ue: -G(up, ue), np.zeros(3 * N), method="BFGS", options={"gtol": 1e-12}).fun
    return minimize(inner, np.zeros(3 * N), method="BFGS", options={"gtol": 1e-11}).fun


@pytest.mark.parametrize("N,t", [(2, 0.4), (2, 0.8), (3, 0.6)])
def test_pursuit_matches_minmax_shooting(oracle_mod, N, t):
    """The game value is the open-loop min-max of the discretised game over
    both players' controls (section 4.2, eq. discgenlaxhopfdg with the
    Lagrangian's p and q maximised and minimised out), found by nested BFGS
    on dynamics written independently in this file."""
    rng = _rng(40 + N + int(10 * t))
    r0 = 0.5
    pb = oracle_mod.Problem(W.H_PURSUIT_EVASION, W.G_PAIR_DIST, 12, 6, W.PE_PARAMS, [r0])
    X = np.concatenate([rng.uniform(-1, 1, 3), rng.uniform(-.3, .3, 3), rng.uniform(-1, 1, 3) + 2,
                        rng.uniform(-.3, .3, 3)])
    res = oracle_mod.solve(pb, X[None], t, N, sigma=8.0, tau=0.25 / 8, tol=1e-28, max_iter=200000, seed=6)
    assert res.status[0] == 0
    brute = _pe_shoot_minmax(X, N, t, r0, W.PE_PARAMS)
    assert abs(res.phi[0] - brute) < 1e-9 * max(1, abs(brute)), (res.phi[0], brute)
    # the controls move the value well beyond the tolerance: the pin sees the running payoff
    idle = _pe_shoot_minmax(X, N, t, r0, W.PE_PARAMS, np.zeros(3 * N), np.zeros(3 * N))
    assert abs(brute - idle) > 1e-4


def _quad_lagrangian(Z, N, hp, x_t, delta):
    xs = np.vstack([Z[:N * 12].reshape(N, 12), x_t])
    ps = Z[N * 12:].reshape(N, 12)
    L = 0.5 * xs[0] @ xs[0]
    for j in range(1, N + 1):
        f0 = quad_f_phys(xs[j], np.zeros(4), hp)
        B = np.stack([quad_f_phys(xs[j], e, hp) - f0 for e in np.eye(4)], axis=1)
        H = -ps[j - 1] @ f0 + 0.5 * np.sum((B.T @ ps[j - 1]) ** 2)
        L += ps[j - 1] @ (xs[j] - xs[j - 1]) - delta * H
    return L


def test_quadrotor_fixed_point_is_stationary_for_independent_lagrangian(oracle_mod):
    rng = _rng(32)
    hp = W.QUAD_PARAMS
    pb = oracle_mod.Problem(W.H_QUADROTOR, W.G_QUAD_SHIFT, 12, 0, hp, np.zeros(13))
    x = rng.uniform(-0.6, 0.6, 12)
    N, t = 8, 0.4
    r = oracle_mod.solve(pb, x[None], t, N, sigma=2.0, tau=0.125, tol=1e-28, max_iter=200000, seed=7, traj=True)
    Z = np.concatenate([r.x_traj[0, :N].ravel(), r.p_traj[0, 1:].ravel()])
    Lf = lambda z: _quad_lagrangian(z, N, hp, x, t / N)
    g = _fd_grad(Lf, Z, h=1e-6)
    assert np.max(np.abs(g)) < 1e-6 * max(1, np.max(np.abs(Z)))
    assert abs(Lf(Z) - r.phi[0]) < 1e-9 * max(1, abs(r.phi[0]))


def _quad_lagrangian_w(Z, N, hp, x_t, delta, wl, wr):
    """The weighted Lax saddle of the quadrotor written out here:
    g(x_0) + sum_j <p_j, x_j - x_{j-1}> - delta sum_j (wl H(x_{j-1}, p_j) + wr H(x_j, p_j)),
    H = -<p, f0> + |B^T p|^2 / 2 from the dynamics in this file, g = |x|^2/2."""
    xs = np.vstack([Z[:N * 12].reshape(N, 12), x_t])
    ps = Z[N * 12:].reshape(N, 12)

    def H(xx, pp):
        f0 = quad_f_phys(xx, np.zeros(4), hp)
        B = np.stack([quad_f_phys(xx, e, hp) - f0 for e in np.eye(4)], axis=1)
        return -pp @ f0 + 0.5 * np.sum((B.T @ pp) ** 2)
    L = 0.5 * xs[0] @ xs[0]
    for j in range(1, N + 1):
        L += ps[j - 1] @ (xs[j] - xs[j - 1]) - delta * (wl * H(xs[j - 1], ps[j - 1]) + wr * H(xs[j], ps[j - 1]))
    return L


@pytest.mark.parametrize("disc,w", [("fe", (1.0, 0.0)), ("trap", (0.5, 0.5))])
def test_quadrotor_weighted_fixed_point_is_stationary(oracle_mod, disc, w):
    """Forward Euler and trapezoid for the quadrotor (section 4.1, eq.
    disclaxFE; the averaged rule): at the oracle's converged iterate the
    weighted saddle written independently above has zero gradient in every
    free block (x_0..x_{N-1}, p_1..p_N), and its value is the oracle's.  A
    wrong weight, a weight on the wrong node, or a missing rank in the
    velocity block of the p-step moves the fixed point off stationarity."""
    rng = _rng(33)
    hp = W.QUAD_PARAMS
    pb = oracle_mod.Problem(W.H_QUADROTOR, W.G_QUAD_SHIFT, 12, 0, hp, np.zeros(13))
    for _ in range(2):
        x = rng.uniform(-0.6, 0.6, 12)
        N, t = 8, 0.4
        r = oracle_mod.solve(pb, x[None], t, N, sigma=2.0, tau=0.125, tol=1e-24, max_iter=300000, seed=7, traj=True,
                             disc=disc)
        assert r.status[0] == 0
        Z = np.concatenate([r.x_traj[0, :N].ravel(), r.p_traj[0, 1:].ravel()])
        Lf = lambda z: _quad_lagrangian_w(z, N, hp, x, t / N, *w)  # noqa: E731
        g = _fd_grad(Lf, Z, h=1e-6)
        assert np.max(np.abs(g)) < 1e-6 * max(1, np.max(np.abs(Z))), np.max(np.abs(g))
        assert abs(Lf(Z) - r.phi[0]) < 1e-9 * max(1, abs(r.phi[0]))
        # the backward-Euler weighting of the same saddle is not stationary there
        Lb = lambda z: _quad_lagrangian_w(z, N, hp, x, t / N, 0.0, 1.0)  # noqa: E731
        assert np.max(np.abs(_fd_grad(Lb, Z, h=1e-6))) > 1e-4


def test_quadrotor_weighted_be_is_algorithm_1(oracle_mod):
    """The weighted solver at the backward-Euler weights (0, 1) runs Algorithm
    1's iteration: after 2,000 fixed iterations its values and trajectories
    agree with Algorithm 1's to 1e-9 wherever other rounding sequences of
    Algorithm 1 itself do (its binary64 FMA build, and its inputs moved by
    one unit in the last place): the p-step is the same minimiser, found by
    a linear solve instead of Sherman-Morrison, so the two differ by
    rounding, which the quadrotor's flat attitude directions amplify at a
    few points."""
    w = W.quadrotor12().subset(np.arange(24))
    pb = oracle_mod.Problem(w.H, w.g, w.d, w.d_y, w.hp, w.gp)
    kw = dict(sigma=w.sigma, tau=w.tau, tol=w.tol, max_iter=2000, fixed_iters=True, seed=w.init_seed, traj=True)
    a = oracle_mod.solve(pb, w.x, w.t, w.N, **kw)
    b = oracle_mod.solve(pb, w.x, w.t, w.N, disc=(0.0, 1.0), **kw)
    others = [oracle_mod.solve_variant("f64fma", pb, w.x, w.t, w.N, **kw)]
    others += [oracle_mod.solve(pb, w.x * (1.0 + sg * 2.0 ** -52), w.t, w.N, **kw) for sg in (1.0, -1.0)]
    rel = lambda u, v: np.abs(u - v) / np.maximum(np.abs(v), 1)  # noqa: E731
    tr = lambda u, v: np.max(np.abs(u - v), axis=(1, 2)) / np.maximum(np.max(np.abs(v), axis=(1, 2)), 1)  # noqa: E731
    cond = np.ones(w.n, bool)
    for f in others:
        cond &= (rel(f.phi, a.phi) < 1e-10) & (tr(f.x_traj, a.x_traj) < 1e-10) & (tr(f.p_traj, a.p_traj) < 1e-10)
    assert cond.mean() >= 0.6
    assert np.max(rel(b.phi, a.phi)[cond]) < 1e-9
    assert np.max(tr(b.x_traj, a.x_traj)[cond]) < 1e-9 and np.max(tr(b.p_traj, a.p_traj)[cond]) < 1e-9


def test_value_nonincreasing_in_t_for_nonnegative_H(oracle_mod):
    """H = c(x)||p|| >= 0: a longer horizon reaches more initial states, so
    phi(x, t) cannot increase with t."""
    w = W.cnorm10(8)
    pb = oracle_mod.Problem(w.H, w.g, w.d, w.d_y, w.hp, w.gp)
    ts = [0.2, 0.4, 0.6, 0.8, 1.0]
    vals = np.stack([oracle_mod.solve(pb, w.x, np.full(w.n, tt), w.N, sigma=w.sigma, tau=w.tau, tol=1e-20,
                                      max_iter=40000, seed=w.init_seed).phi for tt in ts])
    assert np.all(np.diff(vals, axis=0) <= 1e-9)


# --------------------------------------------------------------------------
# Driver semantics: invariants, stopping rule and statuses
# --------------------------------------------------------------------------

def test_endpoint_and_dual_boundary_invariants(oracle_mod):
    w = W.cnorm10(16)
    pb = oracle_mod.Problem(w.H, w.g, w.d, w.d_y, w.hp, w.gp)
    r = oracle_mod.solve(pb, w.x, w.t, w.N, sigma=w.sigma, tau=w.tau, tol=w.tol, max_iter=w.max_iter,
                         seed=w.init_seed, traj=True)
    assert np.array_equal(r.x_traj[:, w.N_max, :], w.x)   # x_N = x exactly
    assert np.all(r.p_traj[:, 0, :] == 0)                 # p_0 = 0


def test_fixed_iteration_mode_reproduces_stop_iteration(oracle_mod):
    w = W.cnorm10(16)
    pb = oracle_mod.Problem(w.H, w.g, w.d, w.d_y, w.hp, w.gp)
    r = oracle_mod.solve(pb, w.x, w.t, w.N, sigma=w.sigma, tau=w.tau, tol=w.tol, max_iter=w.max_iter,
                         seed=w.init_seed)
    for i in range(4):
        rf = oracle_mod.solve(pb, w.x[i:i + 1], w.t[i:i + 1], w.N[i:i + 1], sigma=w.sigma, tau=w.tau, tol=w.tol,
                              max_iter=int(r.iters[i]), fixed_iters=True, seed=w.init_seed, ids=[i])
        assert rf.phi[0] == r.phi[i] and rf.iters[0] == r.iters[i] and rf.status[0] == 0


def test_statuses(oracle_mod):
    w = W.cnorm10(6)
    pb = oracle_mod.Problem(w.H, w.g, w.d, w.d_y, w.hp, w.gp)
    x = w.x.copy(); t = w.t.copy(); N = w.N.copy()
    x[1, 3] = np.nan
    t[2] = 0.0
    N[3] = 0
    N[4] = 33  # beyond N_max
    r = oracle_mod.solve(pb, x, t, N, sigma=w.sigma, tau=w.tau, tol=w.tol, max_iter=1, seed=0, N_max=32)
    assert list(r.status) == [1, 3, 3, 3, 3, 1]
    assert list(r.iters) == [1, 0, 0, 0, 0, 1]
    assert np.isnan(r.phi[1:5]).all()
    # a step size far beyond the stable range blows up: NONFINITE
    q = W.quadrotor12()
    q = q.subset(np.arange(4))
    pq = oracle_mod.Problem(q.H, q.g, q.d, q.d_y, q.hp, q.gp)
    r = oracle_mod.solve(pq, q.x, q.t, q.N, sigma=0.05, tau=5.0, tol=1e-6, max_iter=20000, seed=0, N_max=60)
    assert np.all(r.status == 2)


# --------------------------------------------------------------------------
# Hopf formulation (section 4.1 eq. dischopf; Algorithm 2; Appendix A.1.2)
# --------------------------------------------------------------------------

def test_gstar_is_the_convex_conjugate(oracle_mod):
    """g*(p) = sup_x <x,p> - g(x), evaluated by numerical maximisation."""
    rng = _rng(40)
    d = 3
    a = np.array([0.3, -0.2, 0.5])
    pq = oracle_mod.Problem(W.H_CNORM, W.G_QUAD_SHIFT, d, 0, [0.5], np.concatenate([[0.7], a]))
    pn = oracle_mod.Problem(W.H_CNORM, W.G_NORM, d, 0, [0.5], [0.8])
    for _ in range(4):
        p = rng.standard_normal(d)
        r = minimize(lambda x: -(x @ p - pq.g_val(x)), np.zeros(d), method="BFGS", options={"gtol": 1e-12})
        assert abs(pq.gstar(p) - (-r.fun)) < 1e-9
        q = p / np.linalg.norm(p) * rng.uniform(0.1, 0.95)  # inside the unit ball: sup attained at x = 0
        xs = rng.standard_normal((2000, d)) * rng.uniform(0, 5, (2000, 1))
        best = np.max(xs @ q - np.array([pn.g_val(x) for x in xs]))
        assert best <= pn.gstar(q) + 1e-12 and pn.gstar(q) - best < 0.35
        assert abs(pn.gstar(q) - (-pn.g_val(np.zeros(d)))) < 1e-12  # <x,q> - |x| <= 0, equality at x = 0
        assert np.isinf(pn.gstar(p / np.linalg.norm(p) * 1.5))


@pytest.mark.parametrize("g", ["shift", "norm"])
def test_hopf_first_dual_step_is_argmin(oracle_mod, g):
    """p_1 = argmin_p g*(p) + delta H(x_1, p) + |p - v|^2/(2 sigma) (Appendix
    A.1.2, j = 1), minimised directly (NORM: constrained to the unit ball)."""
    rng = _rng(41)
    d, alpha = 3, 0.5
    a = np.array([0.3, -0.2, 0.5])
    pb = (oracle_mod.Problem(W.H_CNORM, W.G_QUAD_SHIFT, d, 0, [alpha], np.concatenate([[0.7], a])) if g == "shift"
          else oracle_mod.Problem(W.H_CNORM, W.G_NORM, d, 0, [alpha], [0.8]))
    for k in range(6):
        x1 = rng.standard_normal(d)
        v = rng.standard_normal(d) * (0.3 if k % 2 else 2.0)
        sigma, delta = rng.uniform(0.5, 4.0), rng.uniform(0.02, 0.2)
        out = pb.hopf_prox1(x1, v, sigma, delta)
        c = 1 + alpha * np.sin(x1[0]) * np.cos(x1[1])
        if g == "shift":
            f = lambda p: 0.5 * p @ p + a @ p + 0.7 + delta * c * np.linalg.norm(p) + np.sum((p - v) ** 2) / (2 * sigma)
            r = minimize(f, v * 0.5 + 0.01, method="Nelder-Mead", options={"xatol": 1e-12, "fatol": 1e-15, "maxiter": 40000})
            ref = r.x
        else:
            f = lambda p: 0.8 + delta * c * np.linalg.norm(p) + np.sum((p - v) ** 2) / (2 * sigma)
            cons = [{"type": "ineq", "fun": lambda p: 1.0 - p @ p}]
            r = minimize(f, np.zeros(d) + 0.01, method="SLSQP", constraints=cons, options={"ftol": 1e-15, "maxiter": 500})
            ref = r.x
        assert f(out) <= f(ref) + 1e-10
        assert np.max(np.abs(out - ref)) < 1e-4


def test_hopf_eikonal_matches_closed_form(oracle_mod):
    """H = ||p||, g = ||x|| - 1: with a state-independent H the discrete Hopf
    problem forces p_1 = .. = p_N and is the classical Hopf formula
    max_{|p|<=1} <x,p> - t|p| - 1 = max(|x| - t, 0) - 1 (section 2.1)."""
    w = W.eikonal2d(64)
    pb = oracle_mod.Problem(w.H, w.g, w.d, w.d_y, w.hp, w.gp)
    r = oracle_mod.solve(pb, w.x, w.t, w.N, sigma=w.sigma, tau=w.tau, tol=1e-26, max_iter=60000,
                         seed=w.init_seed, traj=True, hopf=True)
    nx = np.linalg.norm(w.x, axis=1)
    exact = np.maximum(nx - w.t, 0) - 1
    assert np.max(np.abs(r.phi - exact)) < 1e-9
    far = nx > w.t + 0.05
    # every multiplier equals the unit vector x/|x|; x_N = x; node 0 is unused
    assert np.max(np.abs(r.p_traj[far, 1:, :] - (w.x / nx[:, None])[far][:, None, :])) < 1e-6
    assert np.array_equal(r.x_traj[:, -1, :], w.x) and np.all(r.x_traj[:, 0, :] == 0)


def test_hopf_constant_speed_matches_closed_form(oracle_mod):
    """alpha = 0, g = ||x-a||^2/2 - 1: Hopf formula max_p <x-a,p> - |p|^2/2 - t|p| - 1
    = max(||x - a|| - t, 0)^2/2 - 1."""
    w = W.cnorm10(48, alpha=0.0)
    pb = oracle_mod.Problem(w.H, w.g, w.d, w.d_y, w.hp, w.gp)
    r = oracle_mod.solve(pb, w.x, w.t, w.N, sigma=w.sigma, tau=w.tau, tol=1e-26, max_iter=40000,
                         seed=w.init_seed, hopf=True)
    a = w.gp[1:]
    exact = 0.5 * np.maximum(np.linalg.norm(w.x - a, axis=1) - w.t, 0) ** 2 - 1
    assert np.max(np.abs(r.phi - exact)) < 1e-9


def test_hopf_and_lax_values_agree_state_dependent(oracle_mod):
    """alpha != 0: the discrete Hopf saddle is the Lax saddle with x_0
    minimised out analytically (the derivation of eq. dischopf), so both
    formulations reach the same value, by different iterations."""
    w = W.cnorm10(24)
    pb = oracle_mod.Problem(w.H, w.g, w.d, w.d_y, w.hp, w.gp)
    kw = dict(sigma=w.sigma, tau=w.tau, tol=1e-24, max_iter=60000, seed=w.init_seed)
    rl = oracle_mod.solve(pb, w.x, w.t, w.N, **kw)
    rh = oracle_mod.solve(pb, w.x, w.t, w.N, hopf=True, **kw)
    ok = (rl.status == 0) & (rh.status == 0)
    assert ok.sum() >= 20
    assert np.max(np.abs(rl.phi - rh.phi)[ok]) < 1e-8


@pytest.mark.parametrize("N", [1, 2, 3])
def test_hopf_state_dependent_eikonal_matches_direct_shooting(oracle_mod, N):
    rng = _rng(44 + N)
    alpha, d = 0.5, 2
    a = np.array([0.4, -0.3])
    pb = oracle_mod.Problem(W.H_CNORM, W.G_QUAD_SHIFT, d, 0, [alpha], np.concatenate([[1.0], a]))
    c = lambda z: 1 + alpha * np.sin(z[0]) * np.cos(z[1])
    g = lambda z: 0.5 * np.sum((z - a) ** 2) - 1.0
    step = lambda s, u: (c(s) * u, 0.0)
    for _ in range(3):
        x = rng.uniform(-1.5, 1.5, d)
        t = rng.uniform(0.2, 0.8)
        r = oracle_mod.solve(pb, x[None], t, N, sigma=1.0, tau=0.25, tol=1e-26, max_iter=40000, seed=1, hopf=True)
        assert r.status[0] == 0
        brute = _shoot_min(step, g, x, N, t, d, rng, bounds_unit_ball=True)
        assert abs(r.phi[0] - brute) < 1e-6, (r.phi[0], brute)


# --------------------------------------------------------------------------
# Robustness recipes (section 6: sigma raised at the cap, value-change stop,
# several random starts)
# --------------------------------------------------------------------------

def test_recipes_off_reproduce_algorithm_1(oracle_mod):
    w = W.cnorm10(16)
    pb = oracle_mod.Problem(w.H, w.g, w.d, w.d_y, w.hp, w.gp)
    kw = dict(sigma=w.sigma, tau=w.tau, tol=w.tol, max_iter=3000, seed=w.init_seed, traj=True)
    a = oracle_mod.solve(pb, w.x, w.t, w.N, **kw)
    b = oracle_mod.solve(pb, w.x, w.t, w.N, starts=1, restarts=0, value_tol=0.0, **kw)
    # value_tol = 0 and starts = 1 take the plain path; force the recipe path with a no-op restart budget
    c = oracle_mod.solve(pb, w.x, w.t, w.N, restarts=1, sigma_inc=0.0, **dict(kw, max_iter=100000))
    assert np.array_equal(a.phi, b.phi) and np.array_equal(a.iters, b.iters)
    conv = a.status == 0
    assert np.array_equal(a.phi[conv], c.phi[conv]) and np.array_equal(a.x_traj[conv], c.x_traj[conv])


def test_sigma_raise_continues_to_the_closed_form(oracle_mod):
    """Eikonal at a small sigma and a short cap: Algorithm 1 stops at the cap;
    raising sigma by 20 (tau = 0.25/sigma) and continuing from the iterate
    reaches the exact value max(|x| - t, 0) - 1."""
    w = W.eikonal2d(24)
    pb = oracle_mod.Problem(w.H, w.g, w.d, w.d_y, w.hp, w.gp)
    kw = dict(sigma=0.5, tau=0.5, tol=1e-14, max_iter=400, seed=w.init_seed)
    plain = oracle_mod.solve(pb, w.x, w.t, w.N, **kw)
    assert np.mean(plain.status == 1) > 0.5
    r = oracle_mod.solve(pb, w.x, w.t, w.N, restarts=40, sigma_inc=20.0, **kw)
    exact = np.maximum(np.linalg.norm(w.x, axis=1) - w.t, 0) - 1
    assert np.all(r.status == 0)
    assert np.max(np.abs(r.phi - exact)) < 1e-6
    assert np.all(r.iters[plain.status == 1] > 400)  # those continued past the first cap


def test_value_change_stop_after_the_cap(oracle_mod):
    """After the first cap the value-change rule stops a slowly settling
    eikonal iterate; the value it returns is the exact one to well within the
    residual rule's own accuracy."""
    w = W.eikonal2d(24)
    pb = oracle_mod.Problem(w.H, w.g, w.d, w.d_y, w.hp, w.gp)
    kw = dict(sigma=w.sigma, tau=w.tau, tol=1e-30, max_iter=1500, seed=w.init_seed)
    r = oracle_mod.solve(pb, w.x, w.t, w.N, restarts=3, sigma_inc=0.0, value_tol=1e-10, **kw)
    exact = np.maximum(np.linalg.norm(w.x, axis=1) - w.t, 0) - 1
    assert np.any(r.status == 4)
    assert np.all(r.iters[r.status == 4] > 1500)
    # a stalled value is not a converged iterate: accuracy of order sqrt(value_tol)
    assert np.max(np.abs(r.phi - exact)) < 1e-5
    # before the first cap the rule is off: one long phase equals Algorithm 1
    long = dict(kw, max_iter=6000)
    a = oracle_mod.solve(pb, w.x, w.t, w.N, **long)
    b = oracle_mod.solve(pb, w.x, w.t, w.N, restarts=0, value_tol=1e-10, **long)
    assert np.array_equal(a.phi, b.phi) and np.array_equal(a.status, b.status)


def test_multi_start_keeps_the_lowest_converged_value(oracle_mod):
    """Several random starts (seed, seed+1, ...): the reported value is the
    lowest among the starts that met a stopping rule, and it matches direct
    shooting of the discretised problem (nonconvex speed, alpha = 0.9)."""
    rng = _rng(60)
    alpha, d, N = 0.9, 2, 3
    a = np.array([1.2, -0.9])
    pb = oracle_mod.Problem(W.H_CNORM, W.G_QUAD_SHIFT, d, 0, [alpha], np.concatenate([[1.0], a]))
    c = lambda z: 1 + alpha * np.sin(z[0]) * np.cos(z[1])
    g = lambda z: 0.5 * np.sum((z - a) ** 2) - 1.0
    step = lambda s, u: (c(s) * u, 0.0)
    xs = rng.uniform(-2.0, 2.0, (6, d))
    t = 0.9
    kw = dict(sigma=1.0, tau=0.25, tol=1e-24, max_iter=40000)
    singles = np.stack([oracle_mod.solve(pb, xs, t, N, seed=7 + s, **kw).phi for s in range(5)])
    multi = oracle_mod.solve(pb, xs, t, N, seed=7, starts=5, **kw)
    assert np.all(multi.status == 0)
    assert np.array_equal(multi.phi, singles.min(axis=0))
    for i in range(len(xs)):
        brute = _shoot_min(step, g, xs[i], N, t, d, rng, starts=6, bounds_unit_ball=True)
        assert multi.phi[i] <= brute + 1e-6
        assert abs(multi.phi[i] - brute) < 1e-5


def _pe_problem(oracle_mod, r0=0.5):
    return oracle_mod.Problem(W.H_PURSUIT_EVASION, W.G_PAIR_DIST, 12, 6, W.PE_PARAMS, [r0])


def test_game_recipe_continuation_is_the_longer_run(oracle_mod):
    """The recipe path on the game continues from the iterate at the cap:
    with sigma unchanged (sigma_inc = 0) one restart after a cap of K is
    Algorithm 3 run to 2K, bit for bit (values, iterations, statuses and
    both trajectories); starts > 1 is refused for a game."""
    w = W.pursuit12().subset(np.arange(12))
    pb = _pe_problem(oracle_mod)
    kw = dict(sigma=w.sigma, tau=w.tau, tol=w.tol, seed=w.init_seed, traj=True)
    a = oracle_mod.solve(pb, w.x, w.t, w.N, max_iter=8000, **kw)
    b = oracle_mod.solve(pb, w.x, w.t, w.N, max_iter=4000, restarts=1, sigma_inc=0.0, **kw)
    assert np.any(a.status == 1) and np.any(a.status == 0)
    for f in ("phi", "iters", "status", "x_traj", "p_traj"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f
    with pytest.raises(ValueError):
        oracle_mod.solve(pb, w.x, w.t, w.N, max_iter=600, starts=2, **kw)


def test_game_sigma_raise_reaches_the_minmax(oracle_mod):
    """Section 6.2's recipe on the pursuit-evasion game: at a small sigma and
    a short cap Algorithm 3 stops at the cap; raising sigma by 20 at each cap
    (tau = sigma0 tau0 / sigma) and continuing from the iterate converges, to
    the open-loop min-max of the discretised game found by nested BFGS."""
    rng = _rng(42)
    r0, N, t = 0.5, 2, 0.4
    pb = _pe_problem(oracle_mod, r0)
    X = np.concatenate([rng.uniform(-1, 1, 3), rng.uniform(-.3, .3, 3), rng.uniform(-1, 1, 3) + 2,
                        rng.uniform(-.3, .3, 3)])
    kw = dict(sigma=0.5, tau=0.5, tol=1e-28, max_iter=300, seed=6)
    plain = oracle_mod.solve(pb, X[None], t, N, **kw)
    assert plain.status[0] == 1
    r = oracle_mod.solve(pb, X[None], t, N, restarts=30, sigma_inc=20.0, **dict(kw, max_iter=20000))
    assert r.status[0] == 0 and r.iters[0] > 300
    brute = _pe_shoot_minmax(X, N, t, r0, W.PE_PARAMS)
    assert abs(r.phi[0] - brute) < 1e-9 * max(1, abs(brute)), (r.phi[0], brute)


def test_game_value_change_stop_after_the_cap(oracle_mod):
    """After the first cap the value-change rule stops game points whose value
    has settled (status VALUE_STALLED); their values agree with a long
    Algorithm 3 run that converges, to the accuracy of a settled value; before
    the first cap the rule is off."""
    w = W.pursuit12().subset(np.arange(24))
    pb = _pe_problem(oracle_mod)
    kw = dict(sigma=w.sigma, tau=w.tau, seed=w.init_seed)
    ref = oracle_mod.solve(pb, w.x, w.t, w.N, tol=1e-12, max_iter=100000, **kw)
    r = oracle_mod.solve(pb, w.x, w.t, w.N, tol=1e-30, max_iter=2000, restarts=20, sigma_inc=0.0, value_tol=1e-12,
                         **kw)
    stalled = r.status == 4
    assert stalled.mean() >= 0.4 and np.all(r.iters[stalled] > 2000)
    assert np.all(r.status[~stalled] == 1)  # the others oscillate through every phase to the last cap
    ok = stalled & (ref.status == 0)
    assert ok.sum() >= 8
    assert np.max(np.abs(r.phi[ok] - ref.phi[ok]) / np.maximum(np.abs(ref.phi[ok]), 1)) < 1e-6
    # a single phase: the rule never engages and the run is Algorithm 3
    a = oracle_mod.solve(pb, w.x, w.t, w.N, tol=w.tol, max_iter=3000, **kw)
    b = oracle_mod.solve(pb, w.x, w.t, w.N, tol=w.tol, max_iter=3000, restarts=0, value_tol=1e-12, **kw)
    assert np.array_equal(a.phi, b.phi) and np.array_equal(a.status, b.status)


# --------------------------------------------------------------------------
# Forward Euler and trapezoidal discretisations (section 4.1, eq. disclaxFE;
# the remark after Algorithm 1 on averaging the two Euler approximations)
# --------------------------------------------------------------------------

def _eik2(oracle_mod, alpha, a=(0.4, -0.3)):
    a = np.asarray(a, float)
    pb = oracle_mod.Problem(W.H_CNORM, W.G_QUAD_SHIFT, 2, 0, [alpha], np.concatenate([[1.0], a]))
    c = lambda z: 1 + alpha * np.sin(z[0]) * np.cos(z[1])
    g = lambda z: 0.5 * np.sum((z - a) ** 2) - 1.0
    return pb, c, g, a


def test_disc_backward_weights_reproduce_algorithm_1(oracle_mod):
    """Weights (0, 1) are the backward-Euler saddle: the weighted solver
    then reproduces Algorithm 1 bit for bit (values, stop iterations and
    both trajectories)."""
    w = W.cnorm10(16)
    pb = oracle_mod.Problem(w.H, w.g, w.d, w.d_y, w.hp, w.gp)
    kw = dict(sigma=w.sigma, tau=w.tau, tol=w.tol, max_iter=w.max_iter, seed=w.init_seed, traj=True)
    a = oracle_mod.solve(pb, w.x, w.t, w.N, **kw)
    b = oracle_mod.solve(pb, w.x, w.t, w.N, disc=(0.0, 1.0), **kw)
    for u, v in [(a.phi, b.phi), (a.iters, b.iters), (a.x_traj, b.x_traj), (a.p_traj, b.p_traj)]:
        assert np.array_equal(u, v)


@pytest.mark.parametrize("disc", ["fe", "trap"])
def test_disc_constant_speed_matches_closed_forms(oracle_mod, disc):
    """c = 1: H does not depend on x, so every discretisation has the
    Hopf-Lax value exactly: max(||x-a|| - t, 0)^2/2 - 1 for the shifted
    quadratic g and max(||x|| - t, 0) - 1 for the norm g."""
    w = W.cnorm10(24, alpha=0.0)
    pb = oracle_mod.Problem(w.H, w.g, w.d, w.d_y, w.hp, w.gp)
    r = oracle_mod.solve(pb, w.x, w.t, w.N, sigma=w.sigma, tau=w.tau, tol=1e-26, max_iter=40000,
                         seed=w.init_seed, disc=disc)
    exact = 0.5 * np.maximum(np.linalg.norm(w.x - w.gp[1:], axis=1) - w.t, 0) ** 2 - 1
    assert np.all(r.status == 0)
    assert np.max(np.abs(r.phi - exact)) < 1e-9
    e = W.eikonal2d(32)
    pe = oracle_mod.Problem(e.H, e.g, e.d, e.d_y, e.hp, e.gp)
    r = oracle_mod.solve(pe, e.x, e.t, e.N, sigma=e.sigma, tau=e.tau, tol=1e-26, max_iter=30000,
                         seed=e.init_seed, disc=disc)
    assert np.max(np.abs(r.phi - (np.maximum(np.linalg.norm(e.x, axis=1) - e.t, 0) - 1))) < 1e-9


def _transcription_min(c_eff, g, x, N, t, d, rng, starts=4):
    """min g(x_0) over node positions x_0..x_{N-1} (x_N = x) with every step
    inside its speed ball: ||x_j - x_{j-1}|| <= delta c_eff(x_{j-1}, x_j).
    The p-maximisation of the eikonal saddle is exactly this constraint."""
    delta = t / N

    def nodes(Z):
        return np.vstack([Z.reshape(N, d), x])
    cons = [{"type": "ineq",
             "fun": (lambda Z, j=j: delta * c_eff(nodes(Z)[j - 1], nodes(Z)[j])
                     - np.linalg.norm(nodes(Z)[j] - nodes(Z)[j - 1]))} for j in range(1, N + 1)]
    best = None
    for _ in range(starts):
        Z0 = np.tile(x, N) + 0.05 * rng.standard_normal(N * d)
        r = minimize(lambda Z: g(nodes(Z)[0]), Z0, method="SLSQP", constraints=cons,
                     options={"ftol": 1e-15, "maxiter": 3000})
        if r.success and (best is None or r.fun < best):
            best = r.fun
    return best


@pytest.mark.parametrize("disc", ["fe", "trap"])
@pytest.mark.parametrize("N", [1, 2, 3])
def test_disc_state_dependent_matches_direct_transcription(oracle_mod, disc, N):
    """alpha != 0: the forward-Euler (trapezoid) value is the least g(x_0)
    over discrete paths whose step j has length at most delta c(x_{j-1})
    (delta (c(x_{j-1}) + c(x_j))/2), found by SLSQP over the node positions."""
    rng = _rng(70 + N + (10 if disc == "trap" else 0))
    pb, c, g, _ = _eik2(oracle_mod, 0.5)
    wl, wr = oracle_mod.DISC_WEIGHTS[disc]
    c_eff = lambda u, v: wl * c(u) + wr * c(v)
    for _ in range(3):
        x = rng.uniform(-1.5, 1.5, 2)
        t = rng.uniform(0.2, 0.8)
        r = oracle_mod.solve(pb, x[None], t, N, sigma=1.0, tau=0.25, tol=1e-26, max_iter=40000, seed=1, disc=disc)
        assert r.status[0] == 0
        best = _transcription_min(c_eff, g, x, N, t, 2, rng)
        assert abs(r.phi[0] - best) < 1e-6, (r.phi[0], best)


def _mix_lagrangian(xs, ps, c, g, delta, wl, wr):
    """The weighted saddle's Lagrangian, written here from its definition:
    g(x_0) + sum_j <p_j, x_j - x_{j-1}> - delta sum_j (wl c(x_{j-1}) + wr c(x_j)) |p_j|."""
    L = g(xs[0])
    for j in range(1, len(xs)):
        L += ps[j] @ (xs[j] - xs[j - 1]) - delta * (wl * c(xs[j - 1]) + wr * c(xs[j])) * np.linalg.norm(ps[j])
    return L


@pytest.mark.parametrize("disc", ["fe", "trap"])
def test_disc_fixed_point_is_stationary_for_independent_lagrangian(oracle_mod, disc):
    """At convergence the free nodes x_0..x_{N-1} are stationary points of the
    Lagrangian above (central differences), and every step x_j - x_{j-1}
    equals delta c_eff p_j/|p_j| (optimality of the p_j with |p_j| > 0)."""
    pb, c, g, a = _eik2(oracle_mod, 0.5)
    wl, wr = oracle_mod.DISC_WEIGHTS[disc]
    rng = _rng(80)
    N, t, h = 6, 0.7, 1e-6
    delta = t / N
    for _ in range(2):
        # far enough from the minimiser of g that every step is at full speed (p_j != 0)
        u = rng.standard_normal(2)
        x = a + 1.6 * u / np.linalg.norm(u)
        r = oracle_mod.solve(pb, x[None], t, N, sigma=1.0, tau=0.25, tol=1e-28, max_iter=60000, seed=2,
                             disc=disc, traj=True)
        assert r.status[0] == 0
        xs, ps = r.x_traj[0].copy(), r.p_traj[0]
        assert np.array_equal(xs[N], x)
        for j in range(N):
            for i in range(2):
                xp = xs.copy(); xp[j, i] += h
                xm = xs.copy(); xm[j, i] -= h
                dL = (_mix_lagrangian(xp, ps, c, g, delta, wl, wr) - _mix_lagrangian(xm, ps, c, g, delta, wl, wr)) / (2 * h)
                assert abs(dL) < 1e-7, (j, i, dL)
        for j in range(1, N + 1):
            npj = np.linalg.norm(ps[j])
            assert npj > 1e-3
            step = delta * (wl * c(xs[j - 1]) + wr * c(xs[j])) * ps[j] / npj
            assert np.max(np.abs((xs[j] - xs[j - 1]) - step)) < 1e-9


def test_trapezoid_is_second_order_and_euler_first_order(oracle_mod):
    """The trapezoid (average of the two Euler Hamiltonian sums) is the more
    accurate rule: halving delta divides its error by about 4, while the
    backward- and forward-Euler errors halve and bracket the limit from
    opposite sides.  The limit is estimated by Richardson extrapolation of the
    trapezoid at N = 64 and 128."""
    pb, _, _, a = _eik2(oracle_mod, 0.5)
    rng = _rng(90)
    u = rng.standard_normal((3, 2))
    x = a + 1.5 * u / np.linalg.norm(u, axis=1, keepdims=True)   # out of reach: the value depends on delta
    t = 0.6
    kw = dict(sigma=1.0, tau=0.25, tol=1e-26, max_iter=200000, seed=1)
    v = {(dz, N): oracle_mod.solve(pb, x, t, N, disc=dz, **kw).phi for dz in ["be", "fe", "trap"] for N in [8, 16, 32]}
    t64 = oracle_mod.solve(pb, x, t, 64, disc="trap", **kw).phi
    t128 = oracle_mod.solve(pb, x, t, 128, disc="trap", **kw).phi
    ref = t128 + (t128 - t64) / 3
    moving = np.abs(v["be", 8] - ref) > 1e-4
    assert moving.sum() == 3
    for dz, lo, hi in [("be", 1.7, 2.3), ("fe", 1.7, 2.3), ("trap", 3.5, 4.5)]:
        e = [np.abs(v[dz, N] - ref)[moving] for N in [8, 16, 32]]
        assert np.all(lo < e[0] / e[1]) and np.all(e[0] / e[1] < hi), (dz, e)
        assert np.all(lo < e[1] / e[2]) and np.all(e[1] / e[2] < hi), (dz, e)
    assert np.all(np.sign(v["be", 16] - ref)[moving] == -np.sign(v["fe", 16] - ref)[moving])
    assert np.all(np.abs(v["trap", 16] - ref)[moving] < 0.1 * np.abs(v["be", 16] - ref)[moving])


# --------------------------------------------------------------------------
# Game Hopf formulation (section 4.2, eq. discgenlaxhopfdghopf; Algorithm 4)
# on Isaacs' game of section 6.3
# --------------------------------------------------------------------------

def _isaacs_pb(oracle_mod, hp=None, gp=None):
    hp = W.ISAACS_PARAMS if hp is None else np.asarray(hp, float)
    gp = W.ISAACS_G if gp is None else np.asarray(gp, float)
    return oracle_mod.Problem(W.H_ISAACS, W.G_SADDLE_QUAD, 2, 1, hp, gp), hp, gp


def _isaacs_c(hp, x, y):
    return hp[0] * (1 + hp[1] * np.exp(-hp[2] * ((x - hp[3]) ** 2 + (y - hp[4]) ** 2)))


def test_isaacs_H_is_the_min_max_over_controls(oracle_mod):
    """H(x,y,p,q) = min over alpha in [0, 2 pi] of max over beta in [-1, 1] of
    <(2 beta + sin alpha, -c(x,y) + cos alpha), (p, q)> - 1, evaluated by
    brute force on the dynamics written here (section 6.3)."""
    hp = W.ISAACS_PARAMS
    lib = oracle_mod.lib()
    rng = _rng(100)
    al = np.linspace(0, 2 * np.pi, 200001)
    for _ in range(20):
        x, y, p, q = rng.uniform(-2, 2, 4)
        c = _isaacs_c(hp, x, y)
        inner = np.maximum(2 * p, -2 * p) + np.sin(al) * p + (-c + np.cos(al)) * q - 1   # max over beta = +-1
        brute = inner.min()
        assert abs(lib.or_isaacs_H(np.ascontiguousarray(hp).ctypes.data_as(oracle_mod.ctypes.POINTER(oracle_mod.ctypes.c_double)), x, y, p, q) - brute) < 1e-9


def _dp_arr(oracle_mod, a):
    return np.ascontiguousarray(a, float).ctypes.data_as(oracle_mod.ctypes.POINTER(oracle_mod.ctypes.c_double))


def test_isaacs_conjugates_match_numerical_sup_and_inf(oracle_mod):
    """e*(p) = sup_x p x - e(x) (convex conjugate), h_*(q) = inf_y q y - h(y)
    (concave conjugate) for e(x) = (a x)^2/2 - c0, h(y) = -(b y)^2/2."""
    from scipy.optimize import minimize_scalar
    lib = oracle_mod.lib()
    gp = np.array([0.5, 2.5, 1.3])
    c0, a, b = gp
    for v in np.linspace(-3, 3, 13):
        sup = -minimize_scalar(lambda x: -(v * x - (0.5 * (a * x) ** 2 - c0))).fun
        inf = minimize_scalar(lambda y: v * y + 0.5 * (b * y) ** 2).fun
        assert abs(lib.or_saddle_estar(_dp_arr(oracle_mod, gp), v) - sup) < 1e-9
        assert abs(lib.or_saddle_hstar(_dp_arr(oracle_mod, gp), v) - inf) < 1e-9


def test_isaacs_costate_steps_solve_their_subproblems(oracle_mod):
    """The p-step maximises -2 delta |p| + delta (the root term linearised at
    the current p) [- e*(p) at the Hopf node 1] - |p - v|^2/(2 sigma); the
    q-step minimises -delta c q + delta (root term linearised at the current
    q) [+ q^2/(2 b^2) at node 1] + |q - u|^2/(2 sigma).  Both checked against
    a dense grid search of those objectives, written here."""
    lib = oracle_mod.lib()
    hp, gp = W.ISAACS_PARAMS, W.ISAACS_G
    a, b = gp[1], gp[2]
    rng = _rng(101)
    grid = np.linspace(-6, 6, 1200001)
    for _ in range(12):
        po, qo, v, u = rng.uniform(-1.5, 1.5, 4)
        x, y = rng.uniform(-2, 2, 2)
        sigma, delta = rng.choice([2.0, 10.0]), 0.005 * rng.integers(1, 4)
        s = np.hypot(po, qo)
        for first in (0, 1):
            f = (-2 * delta * np.abs(grid) + delta * grid * po / s - (first * grid ** 2 / (2 * a * a))
                 - (grid - v) ** 2 / (2 * sigma))
            pg = grid[np.argmax(f)]
            pn = lib.or_isaacs_dual_p(_dp_arr(oracle_mod, gp), po, qo, v, sigma, delta, first)
            assert abs(pn - pg) < 2e-5
            s2 = np.hypot(pn, qo)
            c = _isaacs_c(hp, x, y)
            fq = (-delta * c * grid + delta * grid * qo / s2 + first * grid ** 2 / (2 * b * b)
                  + (grid - u) ** 2 / (2 * sigma))
            qg = grid[np.argmin(fq)]
            qn = lib.or_isaacs_dual_q(_dp_arr(oracle_mod, hp), _dp_arr(oracle_mod, gp), x, y, pn, qo, u, sigma,
                                     delta, first)
            assert abs(qn - qg) < 2e-5


def test_isaacs_hopf_and_lax_reach_the_same_value(oracle_mod):
    """Algorithm 4's saddle is Algorithm 3's with x_0 minimised and y_0
    maximised out through e* and h_* (the derivation of eq.
    discgenlaxhopfdghopf): the two iterations, which differ at node 0 and
    node 1, converge to the same value."""
    w = W.isaacs2(200)
    pb = oracle_mod.Problem(w.H, w.g, w.d, w.d_y, w.hp, w.gp)
    kw = dict(sigma=w.sigma, tau=w.tau, tol=1e-22, max_iter=60000, seed=w.init_seed, ids=w.ids)
    h = oracle_mod.solve(pb, w.x, w.t, w.N, hopf=True, **kw)
    l = oracle_mod.solve(pb, w.x, w.t, w.N, **kw)
    ok = (h.status == 0) & (l.status == 0)
    assert ok.mean() > 0.97
    assert np.max(np.abs(h.phi - l.phi)[ok]) < 1e-9


def _minmax_pq(f, lo=-20.0, hi=20.0):
    """min over q of max over p of f(p, q) for scalar p, q: dense grids, then
    bounded refinement around the grid optimum at each level.  The range
    covers the optimal costates of the grid (|p| <= a^2 |x| ~ 19)."""
    from scipy.optimize import minimize_scalar
    pg = np.linspace(lo, hi, 16001)

    def inner(q):
        k = int(np.argmax(f(pg, q)))
        a, b = pg[max(k - 1, 0)], pg[min(k + 1, len(pg) - 1)]
        r = minimize_scalar(lambda p: -f(p, q), bounds=(a, b), method="bounded", options={"xatol": 1e-12})
        return -r.fun
    qg = np.linspace(lo, hi, 1601)
    vals = np.array([inner(q) for q in qg])
    k = int(np.argmin(vals))
    r = minimize_scalar(inner, bounds=(qg[max(k - 1, 0)], qg[min(k + 1, len(qg) - 1)]), method="bounded",
                        options={"xatol": 1e-12})
    return r.fun


def test_isaacs_single_interval_matches_brute_force_min_max(oracle_mod):
    """N = 1: no free nodes, and the value is min over q of max over p of
    -e*(p) - h_*(-q) + p x - q y - delta H(x, y, p, -q), found here by nested
    scalar searches."""
    pb, hp, gp = _isaacs_pb(oracle_mod)
    c0, a, b = gp
    rng = _rng(102)
    for _ in range(6):
        x, y = rng.uniform(-2.5, 2.5, 2)
        t = float(rng.choice([0.025, 0.05, 0.1]))
        c = _isaacs_c(hp, x, y)
        f = lambda p, q: (-(p * p / (2 * a * a) + c0) + q * q / (2 * b * b) + p * x - q * y
                          - t * (c * q + 2 * np.abs(p) - np.sqrt(p * p + q * q) - 1))
        r = oracle_mod.solve(pb, np.array([[x, y]]), t, 1, sigma=2.0, tau=0.125, tol=1e-26, max_iter=60000, seed=3,
                             hopf=True)
        assert r.status[0] == 0
        assert abs(r.phi[0] - _minmax_pq(f)) < 1e-7, (x, y, t)


def test_isaacs_state_independent_speed_matches_the_hopf_formula(oracle_mod):
    """Constant speed (b1 = 0): stationarity in every free x_j and y_j makes
    all p_j and all q_j equal, so the discrete value is the game Hopf formula
    min_q max_p -e*(p) - h_*(-q) + p x - q y - t H(p, -q) for any N."""
    pb, hp, gp = _isaacs_pb(oracle_mod, hp=[2.0, 0.0, 4.0, 1.0, 1.0])
    c0, a, b = gp
    rng = _rng(103)
    for _ in range(4):
        x, y = rng.uniform(-2.5, 2.5, 2)
        t, N = 0.1, 10
        f = lambda p, q: (-(p * p / (2 * a * a) + c0) + q * q / (2 * b * b) + p * x - q * y
                          - t * (2.0 * q + 2 * np.abs(p) - np.sqrt(p * p + q * q) - 1))
        r = oracle_mod.solve(pb, np.array([[x, y]]), t, N, sigma=2.0, tau=0.125, tol=1e-26, max_iter=80000, seed=4,
                             hopf=True, traj=True)
        assert r.status[0] == 0
        assert abs(r.phi[0] - _minmax_pq(f)) < 1e-7
        assert np.ptp(r.p_traj[0, 1:, 0]) < 1e-9 and np.ptp(r.p_traj[0, 1:, 1]) < 1e-9


def _isaacs_lagrangian(xs, ys, ps, qs, x, y, hp, gp, delta):
    """Eq. discgenlaxhopfdghopf's objective, written here: nodes 1..N-1 free,
    costates 1..N."""
    c0, a, b = gp
    N = len(ps) - 1
    L = -(ps[1] ** 2 / (2 * a * a) + c0) + qs[1] ** 2 / (2 * b * b) + ps[N] * x - qs[N] * y
    for j in range(1, N):
        L += (ps[j] - ps[j + 1]) * xs[j] - (qs[j] - qs[j + 1]) * ys[j]
    for j in range(1, N + 1):
        c = _isaacs_c(hp, xs[j], ys[j])
        L -= delta * (c * qs[j] + 2 * abs(ps[j]) - np.hypot(ps[j], qs[j]) - 1)
    return L


def test_isaacs_fixed_point_is_stationary_for_independent_lagrangian(oracle_mod):
    """At convergence every free node and every q_j is a stationary point of
    the objective above, and every p_j either is (p_j != 0) or satisfies the
    subgradient condition of the 2 delta |p| kink (p_j = 0)."""
    pb, hp, gp = _isaacs_pb(oracle_mod)
    rng = _rng(104)
    N, t, h = 10, 0.05, 1e-6
    delta = t / N
    for _ in range(3):
        x, y = rng.uniform(-2.5, 2.5, 2)
        r = oracle_mod.solve(pb, np.array([[x, y]]), t, N, sigma=2.0, tau=0.125, tol=1e-28, max_iter=80000, seed=5,
                             hopf=True, traj=True)
        assert r.status[0] == 0
        xs, ys = r.x_traj[0, :, 0].copy(), r.x_traj[0, :, 1].copy()
        ps, qs = r.p_traj[0, :, 0].copy(), r.p_traj[0, :, 1].copy()
        assert xs[N] == x and ys[N] == y

        def d(arr, j):
            a0 = arr[j]
            arr[j] = a0 + h; fp = _isaacs_lagrangian(xs, ys, ps, qs, x, y, hp, gp, delta)
            arr[j] = a0 - h; fm = _isaacs_lagrangian(xs, ys, ps, qs, x, y, hp, gp, delta)
            arr[j] = a0
            return (fp - fm) / (2 * h)
        for j in range(1, N):
            assert abs(d(xs, j)) < 1e-7 and abs(d(ys, j)) < 1e-7
        for j in range(1, N + 1):
            assert abs(d(qs, j)) < 1e-7
            if abs(ps[j]) > 1e-6:
                assert abs(d(ps, j)) < 1e-7
            else:
                # the smooth part's slope lies inside the kink's subdifferential [-2 delta, 2 delta]
                p0 = ps[j]; ps[j] = 0.0
                smooth = d(ps, j)  # central difference across the kink cancels the |p| term
                ps[j] = p0
                assert abs(smooth) <= 2 * delta + 1e-7


def test_quadrotor_hopf_prox1_is_the_joint_argmin(oracle_mod):
    """Hopf formulation, quadrotor, shifted quadratic g (section 4.1 eq.
    dischopf; Algorithm 2): the node-1 step minimises g*(p) + delta H(x_1, p)
    + |p - v|^2/(2 sigma) with g*(p) = |p|^2/2 + <a,p> + c0.  Checked against a
    direct numerical minimisation of that objective (BFGS): the oracle's point
    is at least as low and within the minimiser's precision of BFGS's."""
    from scipy.optimize import minimize
    O = oracle_mod
    w = W.quadrotor12(8)
    rng = np.random.default_rng(5)
    gp = np.concatenate([[0.3], rng.uniform(-0.5, 0.5, 12)])
    pb = O.Problem(w.H, w.g, 12, 0, w.hp, gp)
    a = gp[1:]
    for sigma in (0.5, 2.0, 8.0):
        x1, v, delta = rng.uniform(-1, 1, 12), rng.normal(size=12), 0.05
        p = pb.hopf_prox1(x1, v, sigma, delta)
        f = lambda q: 0.5 * q @ q + a @ q + gp[0] + delta * pb.H_val(x1, q, delta) + np.sum((q - v) ** 2) / (2 * sigma)
        r = minimize(f, v, method="BFGS", options={"gtol": 1e-11, "maxiter": 10000})
        assert f(p) <= r.fun + 1e-11
        assert np.max(np.abs(p - r.x)) < 1e-6


def test_quadrotor_hopf_and_lax_reach_the_same_value(oracle_mod):
    """Both formulations are saddle points of one Lagrangian: minimising the
    Lax Lagrangian over x_0 turns g(x_0) - <p_1, x_0> into -g*(p_1), the Hopf
    objective.  Iterated to the same point, the two values agree (quadrotor,
    shifted quadratic g with a nonzero shift; 24 points, t = 0.3, N = 6,
    30,000 iterations)."""
    O = oracle_mod
    w = W.quadrotor12(64)
    rng = np.random.default_rng(7)
    gp = np.concatenate([[0.3], rng.uniform(-0.5, 0.5, 12)])
    pb = O.Problem(w.H, w.g, 12, 0, w.hp, gp)
    m = 24
    x, t, N = w.x[:m], np.full(m, 0.3), np.full(m, 6, np.int32)
    kw = dict(sigma=w.sigma, tau=w.tau, tol=1e-20, max_iter=30000, seed=3, N_max=6, threads=4)
    lax = O.solve(pb, x, t, N, **kw)
    hopf = O.solve(pb, x, t, N, hopf=True, **kw)
    d = np.abs(lax.phi - hopf.phi) / np.maximum(np.abs(lax.phi), 1.0)
    assert np.all(np.isfinite(hopf.phi))
    assert np.median(d) < 1e-7 and d.max() < 1e-5
