"""GPU parity of the Hopf formulation (section 4.1 eq. dischopf, Algorithm 2)
against the oracle's Hopf path, with the same protocol as the Lax parity
tests: the oracle is rerun for exactly the GPU's stop iteration per point and
compared element by element (FP64 1e-9, FP32 1e-4 relative)."""
import numpy as np
import pytest

import workloads as W
from helpers import gpu_solve
from test_gpu_parity import _check

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("plain", [False, True])
def test_hopf_eikonal2d_f64_matches_oracle_and_closed_form(oracle_mod, plain):
    w = W.eikonal2d()
    g = _check(oracle_mod, w, "f64", plain=plain, hopf=True)
    assert np.all(g["status"] == 0)
    exact = np.maximum(np.linalg.norm(w.x, axis=1) - w.t, 0) - 1
    assert np.max(np.abs(g["phi"] - exact)) < 1e-6
    assert np.all(g["x_traj"][:, 0, :] == 0) and np.all(g["p_traj"][:, 0, :] == 0)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("plain", [False, True])
def test_hopf_cnorm10_matches_oracle(oracle_mod, dtype, plain):
    w = W.cnorm10(300)
    _check(oracle_mod, w, dtype, plain=plain, hopf=True)


@pytest.mark.parametrize("tile", [(8, 4), (32, 1), (64, 1)])
def test_hopf_cnorm10_tiles_match_oracle(oracle_mod, tile):
    w = W.cnorm10(130)
    _check(oracle_mod, w, "f32", lanes_per_point=tile[0], nodes_per_lane=tile[1], check_kstop=False, hopf=True)


def test_hopf_small_and_ragged_N(oracle_mod):
    w = W.cnorm10(64)
    w.N = np.array([1, 2, 3, 17, 31, 32] * 10 + [32] * 4, dtype=np.int32)
    _check(oracle_mod, w, "f64", check_kstop=False, hopf=True)


def test_hopf_and_lax_reach_the_same_value():
    """Both formulations solve the same discrete saddle (x_0 minimised out
    analytically in Hopf), so converged values agree to the tolerance's scale."""
    w = W.cnorm10(256)
    a = gpu_solve(w, dtype="f64", traj=False, tol=1e-14, max_iter=20000)
    b = gpu_solve(w, dtype="f64", traj=False, tol=1e-14, max_iter=20000, hopf=True)
    ok = (a["status"] == 0) & (b["status"] == 0)
    assert ok.mean() > 0.95
    assert np.max(np.abs(a["phi"] - b["phi"])[ok]) < 1e-6


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_hopf_quadrotor12_matches_oracle(oracle_mod, dtype):
    """The Hopf formulation on the quadrotor (general control kernel; node 1's
    step is the family's p-prox with step sigma delta/(1 + sigma) at (v -
    sigma a)/(1 + sigma)), with the settings of the Lax quadrotor test: every
    point at the 20,000 cap, values and trajectories, at the plain bar or at
    the point's rounding floor where the flat attitude directions amplify
    rounding."""
    w = W.quadrotor12().subset(np.arange(97))
    _check(oracle_mod, w, dtype, max_iter=20000, check_kstop=False, max_undetermined=0.08, max_above=0.25,
           hopf=True)


def test_hopf_quadrotor12_largest_tiles_f64(oracle_mod):
    """N = 256 and 255 (64 x 4 tile) and 129 (64 x 3): FP64, 300 fixed
    iterations, trajectories compared (node 0 reported as zero)."""
    w = W.quadrotor12().subset(np.arange(9))
    w.N = np.array([256, 255, 129] * 3, dtype=np.int32)
    w.N_max = 256
    w.t = np.full(w.n, 3.0)
    w.fixed_iters = True
    g = _check(oracle_mod, w, "f64", max_iter=300, check_kstop=False, hopf=True)
    assert np.all(g["iters"] == 300)


@pytest.mark.parametrize("hopf", [False, True])
def test_quadrotor12_small_and_ragged_N_f64(oracle_mod, hopf):
    """N = 1 (the only dual is p_1, the Hopf joint prox; no interior node
    moves), 2, 3 and N at and below the tile edges, Lax and Hopf, FP64 at a
    1500-iteration cap.  t = 0.05 N keeps the workload's step delta = 0.05
    (the step sizes sigma, tau are set for it)."""
    w = W.quadrotor12().subset(np.arange(40))
    w.N = np.array([1, 2, 3, 15, 16, 17, 31, 32] * 5, dtype=np.int32)
    w.t = 0.05 * w.N
    _check(oracle_mod, w, "f64", max_iter=1500, check_kstop=False, hopf=hopf)
