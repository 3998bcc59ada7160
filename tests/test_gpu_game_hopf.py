"""GPU parity of the game Hopf formulation (section 4.2, eq.
discgenlaxhopfdghopf, Algorithm 4) on Isaacs' game of section 6.3 against the
oracle's game Hopf path, with the protocol of the Lax parity tests: the oracle
is rerun for exactly the GPU's stop iteration per point and compared element
by element (FP64 1e-9, FP32 1e-4 relative)."""
import numpy as np
import pytest

import workloads as W
from helpers import gpu_solve
from test_gpu_parity import _check

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_isaacs_game_hopf_matches_oracle(oracle_mod, dtype):
    """A seeded 600-point sample of the section's grid at its four times
    (N = 5, 10, 15, 20: three capacity classes in one solve)."""
    w = W.isaacs2(600)
    # FP32: the few points still moving at the 20,000 cap are oscillating
    # iterates that amplify rounding; they are compared at their rounding floor
    g = _check(oracle_mod, w, dtype, hopf=True, check_kstop=(dtype == "f64"), max_above=0.02 if dtype == "f32" else 0.0)
    assert np.mean(g["status"] == 0) > 0.97
    assert np.all(g["x_traj"][:, 0, :] == 0) and np.all(g["p_traj"][:, 0, :] == 0)
    assert np.array_equal(g["x_traj"][np.arange(w.n), w.N], w.x.astype(np.float32).astype(np.float64)
                          if dtype == "f32" else w.x)


@pytest.mark.parametrize("tile", [(8, 4), (32, 1), (64, 1), (16, 2)])
def test_isaacs_game_hopf_tiles_match_oracle(oracle_mod, tile):
    w = W.isaacs2(200)
    _check(oracle_mod, w, "f32", lanes_per_point=tile[0], nodes_per_lane=tile[1], check_kstop=False, hopf=True)


def test_isaacs_small_and_ragged_N(oracle_mod):
    """N = 1 (node 1 is node N: both conjugates and the target meet in one
    node), 2, 3 and N filling a 16-lane group exactly."""
    w = W.isaacs2(96)
    w.N = np.array([1, 2, 3, 7, 16, 20] * 16, dtype=np.int32)
    w.t = 0.005 * w.N
    w.N_max = 20
    _check(oracle_mod, w, "f64", check_kstop=False, hopf=True)


def test_isaacs_game_hopf_reaches_the_game_lax_value(oracle_mod):
    """The GPU's Algorithm 4 value equals the oracle's Algorithm 3 value (a
    different iteration, with node 0 and the initial cost itself) at
    converged points: the two saddles coincide once x_0 and y_0 are
    optimised out through e* and h_*."""
    w = W.isaacs2(300)
    g = gpu_solve(w, dtype="f64", traj=False, tol=1e-20, max_iter=60000, hopf=True)
    pb = oracle_mod.Problem(w.H, w.g, w.d, w.d_y, w.hp, w.gp)
    lax = oracle_mod.solve(pb, w.x, w.t, w.N, sigma=w.sigma, tau=w.tau, tol=1e-20, max_iter=60000, seed=w.init_seed,
                           ids=w.ids)
    ok = (g["status"] == 0) & (lax.status == 0)
    assert ok.mean() > 0.95
    assert np.max(np.abs(g["phi"] - lax.phi)[ok]) < 1e-8


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_isaacs_game_lax_matches_oracle(oracle_mod, dtype):
    """Algorithm 3 on Isaacs' game (node 0 by the closed-form proxes of e and
    of -h, value g(x_0, y_0) + ...): the same 600-point sample against the
    oracle's Algorithm 3 path, values and both trajectories, node 0 included."""
    w = W.isaacs2(600)
    g = _check(oracle_mod, w, dtype, hopf=False, check_kstop=(dtype == "f64"), max_above=0.02 if dtype == "f32" else 0.0)
    assert np.mean(g["status"] == 0) > 0.97
    # node 0 moves (x_0 = e*'(p_1), y_0 = -h_*'(-q_1) at the saddle), costate 0 stays zero
    assert np.mean(np.abs(g["x_traj"][:, 0, :]).sum(axis=1) > 0) > 0.9
    assert np.all(g["p_traj"][:, 0, :] == 0)


@pytest.mark.parametrize("tile", [(8, 4), (64, 1), (16, 2)])
def test_isaacs_game_lax_tiles_and_ragged_N(oracle_mod, tile):
    """Node 0 in the group's first lane with N = 1 (node 1 is node N), 2, 3,
    a group boundary and the tile's capacity; FP64, fixed 400 iterations."""
    L, K = tile
    cap = L * K
    w = W.isaacs2(96)
    w.N = np.array([1, 2, 3, K, K + 1, cap] * 16, dtype=np.int32)
    w.t = 0.005 * w.N
    w.N_max = cap
    w.fixed_iters = True
    _check(oracle_mod, w, "f64", lanes_per_point=L, nodes_per_lane=K, max_iter=400, check_kstop=False, hopf=False)


def test_isaacs_game_lax_and_hopf_agree(oracle_mod):
    """The GPU's Algorithm 3 and Algorithm 4 values coincide at points both
    converge on (x_0 and y_0 optimised out through e* and h_*)."""
    w = W.isaacs2(300)
    a = gpu_solve(w, dtype="f64", traj=False, tol=1e-20, max_iter=60000, hopf=False)
    b = gpu_solve(w, dtype="f64", traj=False, tol=1e-20, max_iter=60000, hopf=True)
    ok = (a["status"] == 0) & (b["status"] == 0)
    assert ok.mean() > 0.95
    assert np.max(np.abs(a["phi"] - b["phi"])[ok]) < 1e-8
