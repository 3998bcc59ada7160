"""The launch schedule never changes a point's arithmetic.

A persistent launch takes the full-occupancy grid when its batch is many times
what that grid holds at once, at most two blocks per CU otherwise, and never
more blocks than the batch fills.  Queue order, grid size and wave priority
decide only which lane group runs which point and when.  Each point's start
noise depends on its index in the batch, so a prefix of a batch solved alone
must give bitwise the same value, stop iteration and status as the same points
inside the whole batch, whatever grid either launch took.
"""
import numpy as np
import pytest

import workloads as W
from helpers import gpu_solve

pytestmark = pytest.mark.gpu


def _same(full, part, m):
    for k in ("phi", "iters", "status"):
        a, b = full[k][:m], part[k]
        same = (a == b) | (np.isnan(a) & np.isnan(b)) if k == "phi" else (a == b)
        bad = np.where(~same)[0]
        if len(bad):
            print("%s differs at %d points, e.g. %s" % (k, len(bad), [(int(i), a[i], b[i], int(full["status"][i]),
                                                                      int(part["status"][i])) for i in bad[:5]]), flush=True)
        assert len(bad) == 0, k


def test_cnorm10_prefix_matches_whole_batch():
    # 65,536 points: two blocks per CU; 512 points: 32 blocks (fill limit)
    w = W.cnorm10()
    full = gpu_solve(w, dtype="f32", traj=False, max_iter=5000)
    m = 512
    part = gpu_solve(w.subset(np.arange(m)), dtype="f32", traj=False, max_iter=5000)
    print("[cnorm10 f32] full n=%d, prefix m=%d, converged %d / %d" % (
        w.n, m, int((full["status"] == 0).sum()), int((part["status"] == 0).sum())), flush=True)
    _same(full, part, m)


def test_quadrotor_prefix_matches_whole_batch():
    # 131,072 points: full occupancy for the classes the batch overfills;
    # 2,048 points: two blocks per CU, fill-limited for the smaller classes
    w = W.quadrotor12()
    full = gpu_solve(w, dtype="f32", traj=False)
    m = 2048
    part = gpu_solve(w.subset(np.arange(m)), dtype="f32", traj=False)
    print("[quadrotor12 f32] full n=%d, prefix m=%d, converged %d / %d" % (
        w.n, m, int((full["status"] == 0).sum()), int((part["status"] == 0).sum())), flush=True)
    _same(full, part, m)


def test_pursuit_prefix_matches_whole_batch():
    # the game kernel with four capacity classes on parallel branches:
    # 16,384 points (two blocks per CU) against 1,024 (fill limit)
    w = W.pursuit12().subset(np.arange(16384))
    full = gpu_solve(w, dtype="f32", traj=False, max_iter=3000)
    m = 1024
    part = gpu_solve(w.subset(np.arange(m)), dtype="f32", traj=False, max_iter=3000)
    print("[pursuit12 f32] n=%d, prefix m=%d, converged %d / %d" % (
        w.n, m, int((full["status"] == 0).sum()), int((part["status"] == 0).sum())), flush=True)
    _same(full, part, m)
