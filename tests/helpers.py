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
              disc="be", **kw):
    import torch

    from paper_1803_01215_amd.solver import Solver

    td = torch.float64 if dtype == "f64" else torch.float32
    s = Solver(d=w.d, d_y=w.d_y, H=w.H, g=w.g, N_max=w.N_max, sigma=w.sigma, tau=w.tau, theta=w.theta,
               tol=w.tol if tol is None else tol, max_iter=w.max_iter if max_iter is None else max_iter,
               seed=w.init_seed, dtype=td, plain=plain,
               fixed_iters=w.fixed_iters if fixed_iters is None else fixed_iters, graph=graph,
               lanes_per_point=lanes_per_point, nodes_per_lane=nodes_per_lane, timing=timing, hopf=hopf, disc=disc,
               **kw)
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


TOL = {"f64": 1e-9, "f32": 1e-4}

# A point's comparison bound is max(TOL, FLOOR_FACTOR * its rounding floor).
# Measured on 512 quadrotor and 1,024 pursuit-evasion points (FP32, 20,000
# iterations) and 97 quadrotor points (FP64, 2,500 and 20,000 iterations):
# the GPU's distance from the oracle is at most 5.7 times the floor below
# (FP32 quadrotor values; 3.8 for its trajectories, 3.0 for pursuit-evasion)
# wherever the floor is not far below the bar.
FLOOR_FACTOR = 10.0
# A floor this large (relative) means the rounding sequences of the oracle
# itself agree on no digit: the point's result is not determined by the
# arithmetic (an iterate still oscillating at the cap, a transient blow-up).
UNDETERMINED_FLOOR = 0.1


def variant_fixed(O, variant, w: W.Workload, iters, *, traj=True, inputs_dtype="f64", x_scale=None, hopf=False,
                  disc="be"):
    """oracle_fixed in one of the oracle's rounding variants ("f64" is the
    oracle itself)."""
    pb = O.Problem(w.H, w.g, w.d, w.d_y, _round(w.hp, inputs_dtype), _round(w.gp, inputs_dtype))
    x, t = _round(w.x, inputs_dtype), _round(w.t, inputs_dtype)
    if x_scale is not None:
        x = x * x_scale
    n = w.n
    phi = np.full(n, np.nan); status = np.zeros(n, np.int32); it = np.zeros(n, np.int32)
    xt = np.zeros((n, w.N_max + 1, w.d)) if traj else None
    pt = np.zeros((n, w.N_max + 1, w.d)) if traj else None
    for K in np.unique(iters):
        sel = np.nonzero(iters == K)[0]
        if K < 1:
            continue
        r = O.solve_variant(variant, pb, x[sel], t[sel], w.N[sel], sigma=float(_round(w.sigma, inputs_dtype)),
                            tau=float(_round(w.tau, inputs_dtype)), theta=w.theta,
                            tol=float(_round(w.tol, inputs_dtype)), max_iter=int(K), fixed_iters=True,
                            seed=w.init_seed, N_max=w.N_max, ids=w.ids[sel], traj=traj, hopf=hopf, disc=disc)
        phi[sel] = r.phi; status[sel] = r.status; it[sel] = r.iters
        if traj:
            xt[sel] = r.x_traj; pt[sel] = r.p_traj
    return {"phi": phi, "iters": it, "status": status, "x_traj": xt, "p_traj": pt}


def _finite_pt(r, N, traj):
    """Per point: value (and trajectory entries 0..N) all finite."""
    ok = np.isfinite(r["phi"])
    if traj:
        for i, Ni in enumerate(N):
            ok[i] &= np.all(np.isfinite(r["x_traj"][i, : Ni + 1])) and np.all(np.isfinite(r["p_traj"][i, : Ni + 1]))
    return ok


def point_errors(a, b, N, traj):
    """Per point: (value error, trajectory error) of a against b, relative as
    in rel_err / traj_err (x and p together); 0 where both are non-finite,
    inf where exactly one is."""
    fa, fb = _finite_pt(a, N, traj), _finite_pt(b, N, traj)
    both = fa & fb
    ev = np.where(both, 0.0, np.where(fa == fb, 0.0, np.inf))
    et = ev.copy()
    idx = np.nonzero(both)[0]
    ev[idx] = rel_err(a["phi"][idx], b["phi"][idx])
    if traj and len(idx):
        et[idx] = np.maximum(traj_err(a["x_traj"][idx], b["x_traj"][idx], N[idx]),
                             traj_err(a["p_traj"][idx], b["p_traj"][idx], N[idx]))
    return ev, (et if traj else np.zeros_like(ev))


def rounding_floor(O, w: W.Workload, iters, dtype, base, *, traj, hopf=False, disc="be"):
    """Per point, how far other rounding sequences of the same iteration land
    from the oracle (`base`) after the same number of iterations:
      FP32 runs: the binary32 builds of the oracle, without and with FMA
                 contraction (inputs rounded to binary32, as on the GPU), and
                 the first on x moved by one binary32 ulp (x (1 +- 2^-23));
      FP64 runs: the binary64 build with FMA contraction, and the oracle on
                 inputs moved by one unit in the last place (x (1 +- 2^-52)).
    Where the iteration amplifies rounding (nearly flat directions of the
    saddle, iterates still oscillating at the cap) the floor is large;
    elsewhere it is far below the bar.  Returns (value floor, trajectory
    floor), inf where a variant and the oracle disagree on whether the point
    stays finite."""
    runs = []
    if dtype == "f32":
        for v in ("f32", "f32fma"):
            runs.append(variant_fixed(O, v, w, iters, traj=traj, inputs_dtype="f32", hopf=hopf, disc=disc))
        for sgn in (1.0, -1.0):
            runs.append(variant_fixed(O, "f32", w, iters, traj=traj, inputs_dtype="f32",
                                      x_scale=1.0 + sgn * 2.0 ** -23, hopf=hopf, disc=disc))
    else:
        runs.append(variant_fixed(O, "f64fma", w, iters, traj=traj, hopf=hopf, disc=disc))
        for sgn in (1.0, -1.0):
            runs.append(variant_fixed(O, "f64", w, iters, traj=traj, x_scale=1.0 + sgn * 2.0 ** -52, hopf=hopf,
                                      disc=disc))
    fv = np.zeros(w.n)
    ft = np.zeros(w.n)
    for r in runs:
        ev, et = point_errors(r, base, w.N, traj)
        fv = np.maximum(fv, ev)
        ft = np.maximum(ft, et)
    return fv, ft


def check_against_oracle(O, w: W.Workload, g, o, dtype, *, traj, hopf=False, disc="be", max_undetermined=0.0,
                         label=""):
    """Compare GPU results g with the oracle o (run for the GPU's iteration
    counts) at every point: value and trajectories within
    max(TOL, FLOOR_FACTOR * rounding floor).  Points whose floor reaches
    UNDETERMINED_FLOOR (the oracle's own rounding sequences agree on no digit,
    or one of them leaves the finite range where another does not) have no
    determined result; they are counted and allowed up to max_undetermined (a
    fraction).  NONFINITE statuses must agree at every other point."""
    tol = TOL[dtype]
    fv, ft = rounding_floor(O, w, g["iters"], dtype, o, traj=traj, hopf=hopf, disc=disc)
    ev, et = point_errors(g, o, w.N, traj)
    det = (fv < UNDETERMINED_FLOOR) & (ft < UNDETERMINED_FLOOR)
    bv = np.maximum(tol, FLOOR_FACTOR * fv)
    bt = np.maximum(tol, FLOOR_FACTOR * ft)
    # where a rounding sequence of the oracle itself misses the bar
    above = det & ((fv > tol) | (ft > tol))
    plain = det & (bv == tol) & (bt == tol)
    print("  %s %d of %d points determined (%d undetermined); the oracle's own rounding sequences miss the "
          "bar %.0e at %d of them; bound = bar at %d, max bound value %.2e traj %.2e" % (
              label, det.sum(), w.n, (~det).sum(), tol, above.sum(), plain.sum(),
              bv[det].max() if det.any() else 0, bt[det].max() if det.any() else 0), flush=True)
    if det.any():
        i = np.nonzero(det)[0]
        print("  value err max %.3g (where the bound is the bar: %.3g); traj err max %.3g (%.3g)" % (
            ev[i].max(), ev[plain].max() if plain.any() else 0, et[i].max(), et[plain].max() if plain.any() else 0),
            flush=True)
    bad = det & ((ev > bv) | (et > bt))
    if bad.any():
        j = np.nonzero(bad)[0][:10]
        print("  failing points %s: value err %s bound %s traj err %s bound %s status %s iters %s" % (
            j, ev[j], bv[j], et[j], bt[j], g["status"][j], g["iters"][j]), flush=True)
    assert not bad.any()
    assert np.mean(~det) <= max_undetermined, (np.nonzero(~det)[0], g["status"][~det], g["iters"][~det])
    assert np.all((g["status"][det] == 2) == (o["status"][det] == 2))
    return {"det": det, "above": above, "fv": fv, "ft": ft, "ev": ev, "et": et}
