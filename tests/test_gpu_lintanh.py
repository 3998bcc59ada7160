"""Linear-tanh family (dense d, matrix-core path) and its reverse mode.

Forward: GPU values and trajectories after K fixed iterations against the FP64
oracle run for the same K (FP32 bar: 1e-4 relative, |a-b| <= 1e-4 max(|b|,1)).
Reverse: d phi/d x, d phi/d A, d phi/d Q and d phi/d eps from hjpd_value_grad
against FP64 central differences of the oracle's fixed-K value, taken as
directional derivatives (phi(b + hV) - phi(b - hV)) / 2h along random unit
directions V, h = 1e-6 max(1, |b|).
"""
import numpy as np
import pytest

import workloads as W
from helpers import rel_err, traj_err

pytestmark = pytest.mark.gpu


def _small_workload(d=16, n=6, N=12, K=100, seed=5):
    r = np.random.default_rng(seed)
    A = r.standard_normal((d, d)) / np.sqrt(d)
    Mq = r.standard_normal((d, d))
    Q = Mq @ Mq.T / d + 0.5 * np.eye(d)
    w = W.lintanh100(8)
    w.d, w.n, w.N_max, w.max_iter = d, n, N, K
    w.x = r.standard_normal((n, d))
    w.t = np.full(n, 1.0)
    w.N = np.full(n, N, np.int32)
    w.hp = np.concatenate([[0.1], A.ravel()])
    w.gp = Q.ravel().copy()
    w.extra = {"A": A, "Q": Q, "ids": np.arange(n)}
    return w


def _f32(a):
    return np.asarray(a, np.float64).astype(np.float32).astype(np.float64)


def _gpu_lt(w, K, E, grad_phi, traj=False):
    import torch

    from paper_1803_01215_amd.autograd import LinearTanhValue
    lt = LinearTanhValue(w.d, w.N_max, w.sigma, w.tau, K, ckpt_every=E, seed=w.init_seed)
    dev = "cuda"
    x = torch.tensor(w.x, dtype=torch.float32, device=dev)
    t = torch.tensor(w.t, dtype=torch.float32, device=dev)
    N = torch.tensor(w.N, dtype=torch.int32, device=dev)
    hp = torch.tensor(w.hp, dtype=torch.float32, device=dev)
    Q = torch.tensor(w.gp, dtype=torch.float32, device=dev)
    gphi = torch.tensor(grad_phi, dtype=torch.float32, device=dev)
    out = lt.solver.solve(x, t, N, hp, Q, traj=traj)
    phi, dx, dh, dg = lt.value_grad(x, t, N, hp, Q, gphi)
    torch.cuda.synchronize()
    res = dict(phi_solve=out.phi.cpu().numpy().astype(np.float64), status=out.status.cpu().numpy(),
               iters=out.iters.cpu().numpy(), phi=phi.cpu().numpy().astype(np.float64),
               dx=dx.cpu().numpy().astype(np.float64), dh=dh.cpu().numpy().astype(np.float64),
               dg=dg.cpu().numpy().astype(np.float64))
    if traj:
        res["x_traj"] = out.x_traj.cpu().numpy().astype(np.float64)
        res["p_traj"] = out.p_traj.cpu().numpy().astype(np.float64)
    lt.close()
    return res


def _oracle_phi(O, w, K, x=None, hp=None, gp=None, idx=None, traj=False):
    idx = np.arange(w.n) if idx is None else np.asarray(idx)
    x = _f32(w.x) if x is None else x
    hp = _f32(w.hp) if hp is None else hp
    gp = _f32(w.gp) if gp is None else gp
    pb = O.Problem(w.H, w.g, w.d, 0, hp, gp)
    return O.solve(pb, x[idx], _f32(w.t)[idx], w.N[idx], sigma=float(_f32(w.sigma)), tau=float(_f32(w.tau)),
                   tol=1e-30, max_iter=K, fixed_iters=True, seed=w.init_seed, N_max=w.N_max, ids=idx, traj=traj)


def test_lintanh100_forward_matches_oracle(oracle_mod):
    w = W.lintanh100().subset(np.arange(20))
    K = w.max_iter
    g = _gpu_lt(w, K, 50, np.ones(w.n), traj=True)
    assert np.all(g["iters"] == K)
    o = _oracle_phi(oracle_mod, w, K, traj=True)
    e = rel_err(g["phi_solve"], o.phi)
    print("lintanh100 phi rel err max %.3g" % e.max())
    assert e.max() <= 1e-4
    assert rel_err(g["phi"], o.phi).max() <= 1e-4  # value returned by value_grad
    ex = traj_err(g["x_traj"], o.x_traj, w.N)
    ep = traj_err(g["p_traj"], o.p_traj, w.N)
    print("traj rel err x %.3g p %.3g" % (ex.max(), ep.max()))
    assert ex.max() <= 1e-4 and ep.max() <= 1e-4


def _fd_dir(O, w, K, which, V, wts, h_rel=1e-6):
    """Central difference of sum_i wts_i phi_i along V for x (per point), A, Q or eps."""
    base = {"x": _f32(w.x), "hp": _f32(w.hp), "gp": _f32(w.gp)}
    if which == "x":
        h = h_rel * max(1.0, np.abs(base["x"]).max())
        vals = []
        for s in (1, -1):
            vals.append(_oracle_phi(O, w, K, x=base["x"] + s * h * V).phi)
        return (vals[0] - vals[1]) / (2 * h)
    key = "gp" if which == "Q" else "hp"
    vec = np.zeros_like(base[key])
    if which == "A":
        vec[1:] = V.ravel()
    elif which == "eps":
        vec[0] = 1.0
    else:
        vec[:] = V.ravel()
    h = h_rel * max(1.0, np.abs(base[key]).max())
    vals = []
    for s in (1, -1):
        kw = {key: base[key] + s * h * vec}
        vals.append(np.dot(wts, _oracle_phi(O, w, K, **kw).phi))
    return (vals[0] - vals[1]) / (2 * h)


def _check_grads(O, w, K, E, n_dirs=2, seed=0):
    rng = np.random.default_rng(seed)
    wts = rng.uniform(0.5, 1.5, w.n)
    g = _gpu_lt(w, K, E, wts)
    d = w.d
    # d phi / d x per point, along random unit directions
    errs = []
    for _ in range(n_dirs):
        V = rng.standard_normal((w.n, d))
        V /= np.linalg.norm(V, axis=1, keepdims=True)
        fd = _fd_dir(O, w, K, "x", V, wts)  # per point, unweighted
        an = np.sum(g["dx"] * V, axis=1) / wts
        errs.append(np.max(np.abs(an - fd) / np.maximum(np.abs(fd), 1)))
    for which in ("A", "Q"):
        for _ in range(n_dirs):
            V = rng.standard_normal((d, d))
            V /= np.linalg.norm(V)
            fd = _fd_dir(O, w, K, which, V, wts)
            an = np.sum((g["dh"][1:] if which == "A" else g["dg"]) * V.ravel())
            errs.append(abs(an - fd) / max(abs(fd), 1))
    fd = _fd_dir(O, w, K, "eps", None, wts)
    errs.append(abs(g["dh"][0] - fd) / max(abs(fd), 1))
    print("gradient rel errors:", np.array(errs))
    return np.array(errs), g


def test_lintanh_small_gradients_match_central_differences(oracle_mod):
    w = _small_workload()
    errs, _ = _check_grads(oracle_mod, w, K=100, E=25)
    assert errs.max() <= 1e-4


@pytest.mark.parametrize("d", [32, 128])
def test_lintanh_other_sizes_values_and_gradients(oracle_mod, d):
    """d = 32 leaves six waves without a row tile of their own, and the reverse
    step forms node 0's adjoint product on them; d = 128 leaves none, and every
    wave sums a quarter of each row's terms."""
    w = _small_workload(d=d, n=3, N=12, K=60, seed=11)
    errs, g = _check_grads(oracle_mod, w, K=60, E=20, n_dirs=1)
    assert errs.max() <= 1e-4
    o = _oracle_phi(oracle_mod, w, 60)
    assert rel_err(g["phi"], o.phi).max() <= 1e-4


def test_lintanh100_gradients_match_central_differences(oracle_mod):
    w = W.lintanh100().subset(np.arange(3))
    errs, _ = _check_grads(oracle_mod, w, K=w.max_iter, E=50, n_dirs=1)
    assert errs.max() <= 1e-4


def test_checkpoint_interval_does_not_change_gradients():
    w = _small_workload(n=4, K=60)
    wts = np.ones(w.n)
    a = _gpu_lt(w, 60, 60, wts)
    b = _gpu_lt(w, 60, 7, wts)
    for k in ("dx", "dh", "dg", "phi"):
        assert np.allclose(a[k], b[k], rtol=1e-6, atol=1e-7), k


def test_envelope_identity_on_gpu_gradient():
    """At a converged iterate d phi/d x = p_N - delta grad_x H(x, p_N)
    (the value is the Lagrangian at a stationary point; x enters as x_N)."""
    w = _small_workload(n=4, K=400, N=10)
    g = _gpu_lt(w, 400, 50, np.ones(w.n), traj=True)
    A = w.extra["A"]
    delta = w.t[0] / w.N[0]
    for i in range(w.n):
        x = w.x[i]
        pN = g["p_traj"][i, w.N[i]]
        th = np.tanh(x)
        env = pN + delta * (A.T @ pN + 0.1 * (1 - th * th) * pN)
        assert np.max(np.abs(env - g["dx"][i])) < 1e-3 * max(1, np.abs(env).max())


def test_autograd_function_matches_value_grad():
    import torch

    from paper_1803_01215_amd.autograd import LinearTanhValue, hj_value
    w = _small_workload(n=5, K=80)
    lt = LinearTanhValue(w.d, w.N_max, w.sigma, w.tau, 80, ckpt_every=20, seed=w.init_seed)
    dev = "cuda"
    x = torch.tensor(w.x, dtype=torch.float32, device=dev, requires_grad=True)
    t = torch.tensor(w.t, dtype=torch.float32, device=dev)
    N = torch.tensor(w.N, dtype=torch.int32, device=dev)
    eps = torch.tensor(0.1, dtype=torch.float32, device=dev, requires_grad=True)
    A = torch.tensor(w.extra["A"], dtype=torch.float32, device=dev, requires_grad=True)
    Q = torch.tensor(w.extra["Q"], dtype=torch.float32, device=dev, requires_grad=True)
    wts = torch.linspace(0.5, 1.5, w.n, device=dev)
    phi = hj_value(x, t, N, eps, A, Q, lt)
    (phi * wts).sum().backward()
    hp = torch.cat([eps.detach().reshape(1), A.detach().reshape(-1)])
    _, dx, dh, dg = lt.value_grad(x.detach(), t, N, hp, Q.detach().reshape(-1), wts)
    torch.cuda.synchronize()
    assert torch.allclose(x.grad, dx)
    assert torch.allclose(A.grad.reshape(-1), dh[1:])
    assert torch.allclose(eps.grad.reshape(1), dh[:1])
    assert torch.allclose(Q.grad.reshape(-1), dg)
    lt.close()
