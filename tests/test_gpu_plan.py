"""Schedule of the persistent path: capacity classes and tiles (hjpd_set_plan,
hjpd_get_plan), the autotuner and its on-disk cache, per-launch timing, the
work queue's integrity (every valid point popped exactly once) and the
no-refill ablation.  The plan and refill change only which lane group takes
which point and when, never a point's arithmetic, so results must be bitwise
equal across plans; the tiles added for finer classes (8 x 3, 16 x 3) are
also checked against the oracle.
"""
import os

import numpy as np
import pytest

import workloads as W
from helpers import check_against_oracle, gpu_solve, oracle_fixed

pytestmark = pytest.mark.gpu


def _inputs(w, td):
    import torch
    dev = "cuda"
    return (torch.tensor(w.x, dtype=td, device=dev), torch.tensor(w.t, dtype=td, device=dev),
            torch.tensor(w.N, dtype=torch.int32, device=dev), torch.tensor(w.hp, dtype=td, device=dev),
            torch.tensor(w.gp, dtype=td, device=dev))


def _solver(w, td, **kw):
    from paper_1803_01215_amd.solver import Solver
    return Solver(d=w.d, d_y=w.d_y, H=w.H, g=w.g, N_max=w.N_max, sigma=w.sigma, tau=w.tau, theta=w.theta, tol=w.tol,
                  max_iter=w.max_iter, seed=w.init_seed, dtype=td, **kw)


def _run(s, inp, traj=False):
    import torch
    out = s.solve(*inp, traj=traj)
    torch.cuda.synchronize()
    r = {"phi": out.phi.cpu().numpy(), "iters": out.iters.cpu().numpy(), "status": out.status.cpu().numpy()}
    if traj:
        r["x_traj"] = out.x_traj.cpu().numpy()
        r["p_traj"] = out.p_traj.cpu().numpy()
    return r


def _equal(a, b):
    for k in a:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


FINE = [(8, 8, 1), (16, 16, 1), (24, 8, 3), (32, 16, 2), (48, 16, 3), (64, 32, 2), (96, 32, 3)]


def test_class_boundaries_change_schedule_only():
    """Splitting the default plan's classes without changing any point's tile
    (N in 17..24 and 25..32 both on 16 x 2, 33..48 and 49..64 both on 32 x 2)
    changes only which launch serves which point: values, iterations,
    statuses and trajectories are bitwise equal."""
    import torch
    w = W.pursuit12().subset(np.arange(3000))
    w.max_iter = 1500
    inp = _inputs(w, torch.float32)
    a = _solver(w, torch.float32)
    b = _solver(w, torch.float32)
    split = [(8, 8, 1), (16, 16, 1), (24, 16, 2), (32, 16, 2), (48, 32, 2), (64, 32, 2), (96, 32, 3)]
    b.set_plan(split)
    plan, cached = b.plan()
    assert plan == split and not cached
    assert a.plan()[0] == [(8, 8, 1), (16, 16, 1), (32, 16, 2), (64, 32, 2), (96, 32, 3)]
    _equal(_run(a, inp, traj=True), _run(b, inp, traj=True))
    a.close(); b.close()


def test_finest_plan_matches_oracle(oracle_mod):
    """The finest partition, with the 8 x 3 and 16 x 3 tiles in its classes,
    on the pursuit-evasion game (N 16..96): a tile fixes the summation order
    of a point's residuals, so results are compared with the oracle at the
    FP32 bar rather than bitwise with another plan."""
    import torch
    w = W.pursuit12().subset(np.arange(200))
    w.max_iter = 2500
    inp = _inputs(w, torch.float32)
    s = _solver(w, torch.float32)
    s.set_plan(FINE)
    g = {k: v.astype(np.float64) if k in ("phi", "x_traj", "p_traj") else v for k, v in _run(s, inp, traj=True).items()}
    s.close()
    o = oracle_fixed(oracle_mod, w, g["iters"], traj=True, inputs_dtype="f32")
    check_against_oracle(oracle_mod, w, g, o, "f32", traj=True)


@pytest.mark.parametrize("tile", [(8, 3), (16, 3)])
@pytest.mark.parametrize("name", ["quadrotor12", "pursuit12", "cnorm10"])
def test_new_tiles_match_oracle(oracle_mod, tile, name):
    """The three-node tiles on every kernel family they serve (general control
    kernel, game kernel, shifted-layout kernel): FP64, fixed 400 iterations,
    N up to the tile's capacity with ragged values, values and trajectories
    against the oracle at 1e-9 (the quadrotor at its rounding floor where its
    flat attitude directions amplify rounding)."""
    L, K = tile
    cap = L * K
    w = W.get(name, 24)
    w.N = np.array([1, 2, 3, cap // 2, cap - 1, cap] * 4, dtype=np.int32)
    w.N_max = cap
    w.t = (0.05 if name == "quadrotor12" else 0.03) * w.N
    w.fixed_iters = True
    w.max_iter = 400
    g = gpu_solve(w, dtype="f64", lanes_per_point=L, nodes_per_lane=K, traj=True)
    assert np.all(g["iters"] == 400)
    o = oracle_fixed(oracle_mod, w, g["iters"], traj=True)
    quad = name == "quadrotor12"
    r = check_against_oracle(oracle_mod, w, g, o, "f64", traj=True, max_undetermined=0.08 if quad else 0.0)
    assert r["above"].mean() <= (0.25 if quad else 0.0)


def test_set_plan_rejects_bad_plans():
    import torch

    from paper_1803_01215_amd import hjpd as C
    w = W.pursuit12().subset(np.arange(64))
    s = _solver(w, torch.float32)
    before = s.plan()[0]
    for bad in ([(64, 32, 2), (32, 16, 2)],          # bounds do not ascend
                [(32, 16, 2), (96, 16, 4)],          # capacity 64 below the class's N = 96
                [(16, 16, 1), (64, 32, 2)],          # does not reach N_max = 96
                [(96, 4, 24)]):                      # tile not built
        with pytest.raises(C.HjpdError) as e:
            s.set_plan(bad)
        assert e.value.code in (C.HJPD_EINVAL, C.HJPD_EUNSUPPORTED)
        assert s.plan()[0] == before
    s.close()


def test_autotune_writes_the_cache_and_create_reads_it(tmp_path, monkeypatch):
    """hjpd_autotune appends its plan to $HJPD_TUNE_CACHE; a second context for
    the same problem starts from that plan without tuning (get_plan reports it
    came from the cache), a context for another problem does not, and the
    cached plan gives bitwise the same results as the tuned one."""
    import torch
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("HJPD_TUNE_CACHE", str(cache))
    w = W.pursuit12().subset(np.arange(4096))
    w.max_iter = 600
    inp = _inputs(w, torch.float32)
    a = _solver(w, torch.float32)
    assert not a.plan()[1]
    a.autotune(*inp, probe_iters=40)
    tuned = a.plan()[0]
    text = cache.read_text()
    assert text.count("plan=") == 1 and "arch=gfx950" in text
    b = _solver(w, torch.float32)
    plan_b, cached = b.plan()
    assert cached and plan_b == tuned
    _equal(_run(a, inp), _run(b, inp))
    w2 = W.pursuit12().subset(np.arange(64))
    w2.N_max = 90
    w2.N = np.minimum(w2.N, 90)
    c = _solver(w2, torch.float32)
    assert not c.plan()[1]
    # every class's tile covers its top N
    prev = 0
    for hi, L, K in tuned:
        assert hi > prev and L * K >= hi
        prev = hi
    assert prev == w.N_max
    a.close(); b.close(); c.close()
    monkeypatch.delenv("HJPD_TUNE_CACHE")


def test_launch_timing_per_class():
    import torch
    w = W.pursuit12().subset(np.arange(4096))
    w.max_iter = 500
    inp = _inputs(w, torch.float32)
    s = _solver(w, torch.float32, timing=True)
    _run(s, inp)
    total, nl = s.timing()
    lts = s.launch_timings()
    assert nl == len(s.plan()[0]) == len(lts) == 5
    assert sorted((a["N_lo"], a["N_hi"]) for a in lts) == [(1, 8), (9, 16), (17, 32), (33, 64), (65, 96)]
    for a in lts:
        assert 0 < a["ms"] <= total * 1.001
    s.close()


@pytest.mark.parametrize("refill", [True, False])
def test_queue_pops_every_valid_point_exactly_once(refill):
    """Pop counter per point id: every valid point is popped exactly once,
    bad-input points never, over several capacity classes and a ragged
    batch; also without refill."""
    import torch
    w = W.pursuit12().subset(np.arange(5003))
    w.max_iter = 300
    t = w.t.copy()
    N = w.N.copy()
    t[[5, 77, 4000]] = [0.0, -1.0, np.nan]
    N[[9, 1234]] = [0, 97]
    w.t, w.N = t, N
    inp = _inputs(w, torch.float32)
    s = _solver(w, torch.float32, refill=refill)
    pops = torch.zeros(w.n, dtype=torch.int32, device="cuda")
    s.set_pop_counter(pops)
    r = _run(s, inp)
    bad = np.zeros(w.n, bool)
    bad[[5, 77, 4000, 9, 1234]] = True
    pc = pops.cpu().numpy()
    assert np.all(pc[~bad] == 1), np.unique(pc[~bad], return_counts=True)
    assert np.all(pc[bad] == 0)
    assert np.all(r["status"][bad] == 3) and np.all(r["iters"][~bad] >= 1)
    # a second solve on the same counter adds exactly one more pop per valid point
    _run(s, inp)
    assert np.all(pops.cpu().numpy()[~bad] == 2)
    s.set_pop_counter(None)
    s.close()


def test_no_refill_changes_schedule_only():
    """Without refill (one point per lane group, a group for every point) the
    results equal the refill path's bit for bit."""
    import torch
    w = W.quadrotor12().subset(np.arange(2000))
    w.max_iter = 2000
    inp = _inputs(w, torch.float32)
    a = _solver(w, torch.float32)
    b = _solver(w, torch.float32, refill=False)
    _equal(_run(a, inp, traj=True), _run(b, inp, traj=True))
    a.close(); b.close()
