"""Parity at the full workload sizes, in the launch configuration the
benchmark times: the whole batch in one hipGraph-replayed solve with the
benchmark's tile and iteration cap.  The oracle cannot rerun every point, so
it reruns a seeded sample: random points plus the slowest ones (the last to
leave the persistent queue), each for exactly the GPU's stop iteration, and
the sample is compared element by element at the usual bar (FP64 1e-9, FP32
1e-4 relative; where a point amplifies rounding, at ten times its rounding
floor, as in the small-size tests; nothing is screened out).  Every point of
the full batch is also checked for a valid status and count.
"""
import numpy as np
import pytest

import workloads as W
from helpers import check_against_oracle, oracle_fixed, rel_err, traj_err

pytestmark = pytest.mark.gpu


def _graph_solve(w, dtype, *, traj=False, max_iter=None, lanes_per_point=0, nodes_per_lane=0, **kw):
    """Capture the solve in a hipGraph (first call) and replay it (second
    call); the replay must reproduce the captured launch bit for bit."""
    import torch

    from paper_1803_01215_amd.solver import Solver
    td = torch.float64 if dtype == "f64" else torch.float32
    s = Solver(d=w.d, d_y=w.d_y, H=w.H, g=w.g, N_max=w.N_max, sigma=w.sigma, tau=w.tau, theta=w.theta, tol=w.tol,
               max_iter=w.max_iter if max_iter is None else max_iter, seed=w.init_seed, dtype=td, graph=True,
               lanes_per_point=lanes_per_point, nodes_per_lane=nodes_per_lane, **kw)
    dev = "cuda"
    args = [torch.tensor(w.x, dtype=td, device=dev), torch.tensor(w.t, dtype=td, device=dev),
            torch.tensor(w.N, dtype=torch.int32, device=dev), torch.tensor(w.hp, dtype=td, device=dev),
            torch.tensor(w.gp, dtype=td, device=dev)]
    runs = []
    for _ in range(2):
        out = s.solve(*args, traj=traj)
        torch.cuda.synchronize()
        r = {"phi": out.phi.cpu().numpy().astype(np.float64), "iters": out.iters.cpu().numpy().astype(np.int32),
             "status": out.status.cpu().numpy().astype(np.int32)}
        if traj:
            r["x_traj"] = out.x_traj.cpu().numpy().astype(np.float64)
            r["p_traj"] = out.p_traj.cpu().numpy().astype(np.float64)
        runs.append(r)
        del out
    s.close()
    for k in runs[0]:
        assert np.array_equal(runs[0][k], runs[1][k], equal_nan=True), k
    return runs[1]


def _sample(g, n, n_rand, n_slow, seed):
    rng = np.random.default_rng(seed)
    slow = np.argsort(-g["iters"], kind="stable")[:n_slow]
    rand = rng.choice(n, n_rand, replace=False)
    return np.unique(np.concatenate([slow, rand]))


def _check_sampled(O, w, g, idx, dtype, *, traj=False, hopf=False, disc="be", max_iter=None, max_above=0.0,
                   max_undetermined=0.0):
    # whole batch: every point written, counts within the cap
    cap = w.max_iter if max_iter is None else max_iter
    assert np.all(np.isin(g["status"], [0, 1, 2])), np.bincount(g["status"][g["status"] >= 0])
    assert np.all((g["iters"] >= 1) & (g["iters"] <= cap))
    ws = w.subset(idx)
    if max_iter is not None:
        ws.max_iter = max_iter
    gs = {k: v[idx] for k, v in g.items()}
    o = oracle_fixed(O, ws, gs["iters"], traj=traj, inputs_dtype=dtype, hopf=hopf, disc=disc)
    print("[%s %s n=%d sample=%d] status=%s, sample status=%s" % (
        w.name, dtype, w.n, len(idx), np.bincount(g["status"], minlength=3), np.bincount(gs["status"], minlength=3)),
        flush=True)
    r = check_against_oracle(O, ws, gs, o, dtype, traj=traj, hopf=hopf, disc=disc, max_undetermined=max_undetermined)
    assert np.mean(r["above"]) <= max_above, np.mean(r["above"])
    return r


HEADLINE_CAP = 5000  # the benchmark's iteration cap for cnorm10


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_fullsize_cnorm10_headline(oracle_mod, dtype):
    """65,536 points, N = 32, tol 1e-6, cap 5,000, 16 x 2 tile, hipGraph."""
    w = W.cnorm10()
    g = _graph_solve(w, dtype, max_iter=HEADLINE_CAP, lanes_per_point=16, nodes_per_lane=2)
    assert np.mean(g["status"] == 0) > 0.99
    idx = _sample(g, w.n, 160, 32, seed=11)
    _check_sampled(oracle_mod, w, g, idx, dtype, max_iter=HEADLINE_CAP)


@pytest.mark.parametrize("variant", [dict(hopf=True), dict(disc="fe"), dict(disc="trap")])
def test_fullsize_cnorm10_variants_f32(oracle_mod, variant):
    """The Hopf formulation and the forward-Euler / trapezoid discretisations
    on the full headline batch, same tile, cap and graph."""
    w = W.cnorm10()
    g = _graph_solve(w, "f32", max_iter=HEADLINE_CAP, lanes_per_point=16, nodes_per_lane=2, **variant)
    assert np.mean(g["status"] == 0) > 0.99
    idx = _sample(g, w.n, 96, 32, seed=12)
    _check_sampled(oracle_mod, w, g, idx, "f32", max_iter=HEADLINE_CAP, **variant)


def test_fullsize_quadrotor12_with_trajectories(oracle_mod):
    """131,072 points, N = ceil(t/0.05) in 10..60, trajectories written, FP32,
    cap 20,000, default tiles per N class.  The sample is compared as the
    small-size quadrotor test does: every sampled point, converged or at the
    cap, at the plain bar or at its rounding floor."""
    w = W.quadrotor12()
    g = _graph_solve(w, "f32", traj=True, max_iter=20000)
    idx = _sample(g, w.n, 64, 16, seed=13)
    _check_sampled(oracle_mod, w, g, idx, "f32", traj=True, max_iter=20000, max_above=0.25, max_undetermined=0.08)


def test_fullsize_quadrotor12_hopf_with_trajectories(oracle_mod):
    """The same full set in the Hopf formulation (the paper's method for its
    quadcopter): graph-captured and replayed, sampled points against the
    oracle's Hopf path as in the Lax test above."""
    w = W.quadrotor12()
    g = _graph_solve(w, "f32", traj=True, max_iter=20000, hopf=True)
    idx = _sample(g, w.n, 64, 16, seed=17)
    _check_sampled(oracle_mod, w, g, idx, "f32", traj=True, hopf=True, max_iter=20000, max_above=0.25,
                   max_undetermined=0.08)


def test_fullsize_pursuit12_uneven_N(oracle_mod):
    """262,144 points, N in 16..96 across several tile classes in one graph,
    cap 20,000.  About 6 % of the points are still moving at the cap; after
    20,000 FP32 iterations such an iterate has drifted from the FP64 one by
    more than the FP32 bar, as far as the oracle's own binary32 builds drift:
    those are compared at their rounding floor, every other sampled point at
    the plain bar, converged or not."""
    w = W.pursuit12()
    g = _graph_solve(w, "f32", max_iter=20000)
    assert len(np.unique(w.N)) > 40
    idx = _sample(g, w.n, 64, 16, seed=14)
    r = _check_sampled(oracle_mod, w, g, idx, "f32", max_iter=20000, max_above=0.25, max_undetermined=0.25)
    # the bar is out of the oracle's own reach, or no digit is determined, only where the iterate was
    # still moving at the cap
    assert np.all(g["status"][idx][r["above"] | ~r["det"]] == 1)


def test_fullsize_lintanh100_forward_and_reverse(oracle_mod):
    """16,384 points, d = 100, N = 50, 500 fixed iterations, checkpoints every
    50: the benchmark's configuration.  Forward: values and trajectories of
    sampled points against the oracle at the same 500 iterations.  Reverse:
    with output weights one-hot at a sampled point, the batch gradient is that
    point's gradient, checked against oracle central differences along random
    directions in x, A and Q; and the full-batch gradients are linear in the
    output weights, d(w1) + d(w2) = d(w1 + w2), which covers the reduction
    over all 16,384 points."""
    from test_gpu_lintanh import _f32, _gpu_lt, _oracle_phi
    w = W.lintanh100()
    K, E = w.max_iter, 50
    rng = np.random.default_rng(15)
    idx = np.sort(rng.choice(w.n, 5, replace=False))
    i0 = int(idx[0])
    onehot = np.zeros(w.n)
    onehot[i0] = 1.0
    g = _gpu_lt(w, K, E, onehot, traj=True)
    assert np.all(g["iters"] == K)
    o = _oracle_phi(oracle_mod, w, K, idx=idx, traj=True)
    assert rel_err(g["phi_solve"][idx], o.phi).max() <= 1e-4
    assert rel_err(g["phi"][idx], o.phi).max() <= 1e-4
    assert traj_err(g["x_traj"][idx], o.x_traj, w.N[idx]).max() <= 1e-4
    assert traj_err(g["p_traj"][idx], o.p_traj, w.N[idx]).max() <= 1e-4
    # one point's gradient through the full-batch reverse pass
    base = {"x": _f32(w.x), "hp": _f32(w.hp), "gp": _f32(w.gp)}
    d = w.d
    errs = []
    V = rng.standard_normal(d)
    V /= np.linalg.norm(V)
    h = 1e-6 * max(1.0, np.abs(base["x"][i0]).max())
    xs = [base["x"].copy(), base["x"].copy()]
    xs[0][i0] += h * V
    xs[1][i0] -= h * V
    fd = (_oracle_phi(oracle_mod, w, K, x=xs[0], idx=[i0]).phi[0] - _oracle_phi(oracle_mod, w, K, x=xs[1], idx=[i0]).phi[0]) / (2 * h)
    errs.append(abs(g["dx"][i0] @ V - fd) / max(abs(fd), 1))
    assert np.all(g["dx"][np.arange(w.n) != i0] == 0)
    for key, which in (("hp", "A"), ("gp", "Q")):
        M = rng.standard_normal((d, d))
        M /= np.linalg.norm(M)
        vec = np.zeros_like(base[key])
        if which == "A":
            vec[1:] = M.ravel()
        else:
            vec[:] = M.ravel()
        h = 1e-6 * max(1.0, np.abs(base[key]).max())
        ph = [_oracle_phi(oracle_mod, w, K, idx=[i0], **{key: base[key] + s * h * vec}).phi[0] for s in (1, -1)]
        fd = (ph[0] - ph[1]) / (2 * h)
        an = np.sum((g["dh"][1:] if which == "A" else g["dg"]) * M.ravel())
        errs.append(abs(an - fd) / max(abs(fd), 1))
    print("one-point gradient rel errors at full size:", errs, flush=True)
    assert max(errs) <= 1e-4
    # linearity of the full-batch gradients in the output weights
    w1 = rng.uniform(0.5, 1.5, w.n)
    w2 = rng.uniform(-1.0, 1.0, w.n)
    a, b, c = (_gpu_lt(w, K, E, wt) for wt in (w1, w2, w1 + w2))
    for k in ("dx", "dh", "dg"):
        scale = max(np.abs(c[k]).max(), 1.0)
        assert np.max(np.abs(a[k] + b[k] - c[k])) <= 1e-4 * scale, k


@pytest.mark.parametrize("hopf", [True, False])
def test_fullsize_isaacs2_game(oracle_mod, hopf):
    """Isaacs' game, the section's whole 73 x 73 grid at its four times
    (21,316 points, N = 5..20), FP32, cap 20,000: the game Hopf formulation
    (Algorithm 4) and Algorithm 3."""
    w = W.isaacs2()
    g = _graph_solve(w, "f32", max_iter=20000, hopf=hopf)
    assert np.mean(g["status"] == 0) > 0.97
    idx = _sample(g, w.n, 96, 32, seed=16)
    _check_sampled(oracle_mod, w, g, idx, "f32", max_iter=20000, hopf=hopf)
