"""The frozen per-workload parameter files (workloads/configs/*.json) restate
what the seeded generators in workloads/ produce: step sizes sigma and tau
(tau = 0.25/sigma, sigma from an oracle sweep), extrapolation, tolerance, cap,
sizes and seeds.  They must not drift apart."""
import json
import os

import pytest

import workloads as W

HERE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "workloads", "configs")


@pytest.mark.parametrize("name", sorted(W.ALL))
def test_config_file_matches_generator(name):
    rec = json.load(open(os.path.join(HERE, name + ".json")))
    w = W.get(name)
    for key in ("H", "g", "d", "d_y", "n", "N_max", "dtype", "sigma", "tau", "theta", "tol", "max_iter",
                "fixed_iters", "init_seed"):
        assert rec[key] == getattr(w, key), key
    assert rec["seed"] == W.SEED_BASE + w.index
    assert abs(rec["tau"] * rec["sigma"] - 0.25) < 1e-12  # tau = 0.25 / sigma, sigma tau ||D||^2 < 1
    if isinstance(rec["h_params"], list):
        assert rec["h_params"] == [float(v) for v in w.hp]
    if isinstance(rec["g_params"], list):
        assert rec["g_params"] == [float(v) for v in w.gp]
