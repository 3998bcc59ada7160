"""Shared helpers for the GPU parity tests: run a workload through the C ABI
and through the oracle on the same seeded inputs."""
from __future__ import annotations

import numpy as np

import workloads as W


def rel_err(a, b):
    """|a - b| / max(|b|, 1), elementwise."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.abs(a - b) / np.maximum(np.abs(b), 1.0)


def traj_err(a, b, N):
    """Per point: max over nodes 0..N and coordinates of |a - b|, divided by
    max(||b||_inf, 1) over the same entries."""
    out = np.zeros(len(N))
    for i, Ni in enumerate(N):
        aa = a[i, : Ni + 1]
        bb = b[i, : Ni + 1]
        out[i] = np.max(np.abs(aa - bb)) / max(np.max(np.abs(bb)), 1.0)
    return out


def gpu_solve(w: W.Workload, *, dtype="f32", plain=False, fixed_iters=None, max_iter=None, tol=None, traj=True,
              graph=False, lanes_per_point=0, nodes_per_lane=0, x=None, t=None, N=None, timing=False, hopf=False,
              disc="be"):
    import torch

    from paper_1803_01215_amd.solver import Solver

    td = torch.float64 if dtype == "f64" else torch.float32
    s = Solver(d=w.d, d_y=w.d_y, H=w.H, g=w.g, N_max=w.N_max, sigma=w.sigma, tau=w.tau, theta=w.theta,
               tol=w.tol if tol is None else tol, max_iter=w.max_iter if max_iter is None else max_iter,
               seed=w.init_seed, dtype=td, plain=plain,
               fixed_iters=w.fixed_iters if fixed_iters is None else fixed_iters, graph=graph,
               lanes_per_point=lanes_per_point, nodes_per_lane=nodes_per_lane, timing=timing, hopf=hopf, disc=disc)
    dev = "cuda"
    xs = torch.tensor(w.x if x is None else x, dtype=td, device=dev).contiguous()
    ts = torch.tensor(w.t if t is None else t, dtype=td, device=dev).contiguous()
    Ns = torch.tensor(w.N if N is None else N, dtype=torch.int32, device=dev).contiguous()
    hp = torch.tensor(w.hp, dtype=td, device=dev)
    gp = torch.tensor(w.gp, dtype=td, device=dev)
    out = s.solve(xs, ts, Ns, hp, gp, traj=traj)
    torch.cuda.synchronize()
    res = {k: (None if getattr(out, k) is None else getattr(out, k).cpu().numpy().astype(
        np.float64 if k in ("phi", "x_traj", "p_traj") else np.int32)) for k in ("phi", "iters", "status", "x_traj",
                                                                               "p_traj")}
    s.close()
    return res


def oracle_fixed(O, w: W.Workload, iters, *, traj=True, inputs_dtype="f64", threads=0, x_scale=None, hopf=False,
                 disc="be"):
    """Oracle run with exactly iters[i] iterations at point i (points grouped
    by count).  Inputs are first rounded to the GPU run's precision so both
    sides see the same numbers; x_scale (optional) then multiplies x, for the
    conditioning screen."""
    pb = O.Problem(w.H, w.g, w.d, w.d_y, _round(w.hp, inputs_dtype), _round(w.gp, inputs_dtype))
    x, t = _round(w.x, inputs_dtype), _round(w.t, inputs_dtype)
    if x_scale is not None:
        x = x * x_scale
    n = w.n
    phi = np.zeros(n); status = np.zeros(n, np.int32); it = np.zeros(n, np.int32)
    xt = np.zeros((n, w.N_max + 1, w.d)) if traj else None
    pt = np.zeros((n, w.N_max + 1, w.d)) if traj else None
    ids = w.ids
    for K in np.unique(iters):
        sel = np.nonzero(iters == K)[0]
        if K < 1:
            continue
        r = O.solve(pb, x[sel], t[sel], w.N[sel], sigma=float(_round(w.sigma, inputs_dtype)),
                    tau=float(_round(w.tau, inputs_dtype)), theta=w.theta, tol=float(_round(w.tol, inputs_dtype)),
                    max_iter=int(K), fixed_iters=True, seed=w.init_seed, N_max=w.N_max, ids=ids[sel], traj=traj,
                    threads=threads, hopf=hopf, disc=disc)
        phi[sel] = r.phi; status[sel] = r.status; it[sel] = r.iters
        if traj:
            xt[sel] = r.x_traj; pt[sel] = r.p_traj
    return {"phi": phi, "iters": it, "status": status, "x_traj": xt, "p_traj": pt}


def oracle_tol(O, w: W.Workload, *, inputs_dtype="f64", threads=0, traj=False, hopf=False, disc="be"):
    pb = O.Problem(w.H, w.g, w.d, w.d_y, _round(w.hp, inputs_dtype), _round(w.gp, inputs_dtype))
    r = O.solve(pb, _round(w.x, inputs_dtype), _round(w.t, inputs_dtype), w.N,
                sigma=float(_round(w.sigma, inputs_dtype)), tau=float(_round(w.tau, inputs_dtype)), theta=w.theta,
                tol=float(_round(w.tol, inputs_dtype)), max_iter=w.max_iter, fixed_iters=w.fixed_iters,
                seed=w.init_seed, N_max=w.N_max, ids=w.ids, traj=traj, threads=threads, hopf=hopf, disc=disc)
    return {"phi": r.phi, "iters": r.iters, "status": r.status, "x_traj": r.x_traj, "p_traj": r.p_traj}


def _round(a, dt):
    a = np.asarray(a, np.float64)
    return a.astype(np.float32).astype(np.float64) if dt == "f32" else a


def well_conditioned(O, w: W.Workload, iters, base, dtype, tol, hopf=False, disc="be"):
    """Points whose oracle result is stable under a rounding-sized change of
    the inputs: relative 1e-15 for FP64 runs; 1e-6 for FP32 runs (FP32 unit
    roundoff 6e-8 accumulated over thousands of iterations), both signs.  A
    point is kept when the oracle's own value and trajectories move by at
    most tol/10.  Elsewhere the iteration amplifies rounding differences (a
    non-contractive, oscillating iterate), so two implementations with
    different rounding order cannot agree elementwise; such points are
    screened out and counted.  `base` is the unperturbed oracle result."""
    eps = 1e-15 if dtype == "f64" else 1e-6
    traj = base.get("x_traj") is not None
    ok = np.ones(w.n, bool)
    for sgn in (1.0, -1.0):
        r = oracle_fixed(O, w, iters, traj=traj, inputs_dtype=dtype, x_scale=1.0 + sgn * eps, hopf=hopf, disc=disc)
        ok &= rel_err(r["phi"], base["phi"]) <= tol / 10
        if traj:
            ok &= traj_err(r["x_traj"], base["x_traj"], w.N) <= tol / 10
            ok &= traj_err(r["p_traj"], base["p_traj"], w.N) <= tol / 10
    return ok
