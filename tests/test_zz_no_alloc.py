"""The allocation-free entry point against hjpd_solve_batch, through the C ABI.

hjpd_solve_batch_noalloc runs the same queue builder and persistent kernels
as hjpd_solve_batch, with the queue and its counters in the library's static
per-GPU scratch instead of the context's workspace, so its outputs must equal
hjpd_solve_batch's bit for bit (each point is solved on its own; the queue
order does not change results).  Two calls in a row, the second on a smaller
batch, check that nothing left in the shared scratch by one call leaks into
the next.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _ctx(w, dtype, max_iter, flags=0):
    from paper_1803_01215_amd import hjpd as C
    desc = C.hjpd_desc(d=w.d, d_y=w.d_y, H=w.H, g=w.g, dtype=C.HJPD_F64 if dtype == "f64" else C.HJPD_F32,
                       N_max=w.N_max, sigma=w.sigma, tau=w.tau, theta=w.theta, tol=w.tol, max_iter=max_iter,
                       seed=w.init_seed, flags=flags)
    return C.hjpd_create(desc)


def _run(fn, ctx, w, m, dtype, traj):
    import torch
    td = torch.float64 if dtype == "f64" else torch.float32
    dev = "cuda"
    x = torch.tensor(w.x[:m], dtype=td, device=dev).contiguous()
    t = torch.tensor(w.t[:m], dtype=td, device=dev)
    N = torch.tensor(w.N[:m], dtype=torch.int32, device=dev)
    hp = torch.tensor(w.hp, dtype=td, device=dev)
    gp = torch.tensor(w.gp, dtype=td, device=dev)
    phi = torch.full((m,), float("nan"), dtype=td, device=dev)
    it = torch.full((m,), -7, dtype=torch.int32, device=dev)
    st = torch.full((m,), -7, dtype=torch.int32, device=dev)
    xt = torch.zeros(m, w.N_max + 1, w.d, dtype=td, device=dev) if traj else None
    pt = torch.zeros(m, w.N_max + 1, w.d, dtype=td, device=dev) if traj else None
    fn(ctx, m, x, t, N, hp, gp, phi, xt, pt, it, st, torch.cuda.current_stream())
    torch.cuda.synchronize()
    out = {"phi": phi.cpu().numpy(), "iters": it.cpu().numpy(), "status": st.cpu().numpy()}
    if traj:
        out["x_traj"] = xt.cpu().numpy()
        out["p_traj"] = pt.cpu().numpy()
    return out


@pytest.mark.parametrize("name,dtype,max_iter,sizes,traj", [
    ("pursuit12", "f32", 1500, (3001, 1100), False),   # four capacity classes on parallel branches
    ("quadrotor12", "f32", 1500, (2048, 777), True),   # three classes, trajectories written
    ("cnorm10", "f64", 2000, (1500, 257), False),      # one class, FP64
])
def test_noalloc_matches_solve_batch(name, dtype, max_iter, sizes, traj):
    from paper_1803_01215_amd import hjpd as C
    w = W.get(name, max(sizes))
    ctx = _ctx(w, dtype, max_iter)
    try:
        for m in sizes:
            print("[noalloc] %s %s n=%d" % (name, dtype, m), flush=True)
            ref = _run(C.hjpd_solve_batch, ctx, w, m, dtype, traj)
            got = _run(C.hjpd_solve_batch_noalloc, ctx, w, m, dtype, traj)
            assert np.all(ref["status"] >= 0) and np.all(ref["iters"] >= 1)
            for k in ref:
                np.testing.assert_array_equal(got[k], ref[k], err_msg="%s %s n=%d" % (name, k, m))
    finally:
        C.hjpd_destroy(ctx)


def test_noalloc_rejects_what_it_cannot_hold():
    import torch

    from paper_1803_01215_amd import hjpd as C
    w = W.cnorm10(8)
    ctx = _ctx(w, "f32", 10)
    try:
        z = torch.zeros(8, device="cuda")
        with pytest.raises(C.HjpdError) as e:
            C.hjpd_solve_batch_noalloc(ctx, (1 << 20) + 1, z, z, z, z, z, z, None, None, z, z)
        assert e.value.code == C.HJPD_EINVAL
    finally:
        C.hjpd_destroy(ctx)
    ctx = _ctx(w, "f32", 10, flags=C.HJPD_PLAIN)
    try:
        z = torch.zeros(8, device="cuda")
        with pytest.raises(C.HjpdError) as e:
            C.hjpd_solve_batch_noalloc(ctx, 8, z, z, z, z, z, z, None, None, z, z)
        assert e.value.code == C.HJPD_EUNSUPPORTED
    finally:
        C.hjpd_destroy(ctx)
