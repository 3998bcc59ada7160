"""Throughput benchmark: converged (x,t) solves per second at PDHG residual 1e-6.

One step = one full solve of the workload (every point runs the primal-dual
iteration of section 5.1, Algorithm 1, until both squared residuals are below
1e-6 or the cap is hit) with all inputs resident in HBM.

Default workload (cnorm10): d = 10, H = c(x)||p||, c = 1 + 0.5 sin(x1) cos(x2),
g = ||x - a||^2/2 - 1, 65,536 points x ~ N(0, I), t ~ U[0.2, 1], N = 32, FP32.
The batched path is the persistent lane-group kernel replayed from a hipGraph;
the plain path (one point per lane, state in HBM) is timed beside it.

Prints one JSON line (rank 0, one GPU).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp32_vector": 157.3e12, "fp64_vector": 78.6e12, "fp32_matrix": 157.3e12}


def flops_per_iter_cnorm(N: int, d: int) -> int:
    """Algorithmic flops of one iteration of one point for H = c(x)||p|| with
    g = ||x-a||^2/2 - c0 (FMA = 2 flops; transcendentals not counted):
      dual step,   nodes 1..N:   9d + 12  (stencil 3d, c(x) 3, ||v||^2 2d,
                                           shrink 5, scale d, residual 3d,
                                           grad c 4)
      primal step, nodes 1..N-1: 8d + 6   (grad 2, update 3d + 4, difference
                                           d, residual 2d, extrapolation 2d)
      node 0:                    9d       (prox 4d, residual 3d, extrap. 2d)
    plus per dual node 2 sin/cos pairs and 1 rsqrt."""
    return N * (9 * d + 12) + (N - 1) * (8 * d + 6) + 9 * d


# Sources of the persistent kernel: HBM traffic measured by rocprofv3 counters
# is reported only while these files are unchanged since the measurement.
KERNEL_SOURCES = ["paper_1803_01215_amd/csrc/hjpd_kernels.hpp", "paper_1803_01215_amd/csrc/hjpd_families.hpp",
                  "paper_1803_01215_amd/csrc/hjpd_device.hpp", "paper_1803_01215_amd/csrc/hjpd_api.hip"]
TRAFFIC_FILE = "profiles/traffic_cnorm10_f32_group16x2.json"


def kernel_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None when the summary is absent, names another kernel, or the kernel
    sources changed after the counters were taken."""
    path = os.path.join(ROOT, TRAFFIC_FILE)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel") != kernel or rec.get("sources_sha256") != kernel_sources_sha256():
        return None
    return float(rec["bytes_per_launch"])


def mfma_flops_per_iter_lintanh(N: int, d: int) -> int:
    """Matrix-core flops of one iteration of one point for the linear-tanh
    family: A x_j for the dual step at j = 1..N and A^T p_j for the primal
    step at j = 1..N-1, each a d x d by d product (FMA = 2 flops)."""
    return 2 * d * d * (2 * N - 1)


def oracle_sample(w, m):
    """The FP64 oracle on the first m points of a workload (FP32-rounded
    parameters, the GPU's stopping rule), OpenMP over points on the host's
    cores: converged solves/s of the sample (fixed-iteration workloads count
    every finished point), with the sample and thread count stated."""
    from oracle import oracle as O
    O.build()
    m = min(m, w.n)
    sub = w.subset(np.arange(m))
    pb = O.Problem(sub.H, sub.g, sub.d, sub.d_y, sub.hp.astype(np.float32).astype(np.float64),
                   sub.gp.astype(np.float32).astype(np.float64))
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    r = O.solve(pb, sub.x, sub.t, sub.N, sigma=sub.sigma, tau=sub.tau, theta=sub.theta, tol=sub.tol,
                max_iter=sub.max_iter, seed=sub.init_seed, N_max=sub.N_max, ids=sub.ids, threads=threads,
                fixed_iters=sub.fixed_iters)
    dt = time.perf_counter() - t0
    done = m if sub.fixed_iters else int((r.status == 0).sum())
    return {"value": done / dt, "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": "first %d of the %d points, FP64 C oracle, OpenMP over points, %.1f s wall, %d %s" % (
                m, w.n, dt, done, "finished" if sub.fixed_iters else "converged")}


def bench_lintanh(torch, dev, steps, cpu=False):
    """Forward solves/s and MFMA throughput at K = 500 fixed iterations, and
    the reverse-mode call (forward with checkpoints every 50 + backward +
    reductions) on the same 16,384 points."""
    import workloads as W
    from paper_1803_01215_amd.autograd import LinearTanhValue
    from paper_1803_01215_amd.solver import Solver

    w = W.lintanh100()
    K = w.max_iter
    f32 = torch.float32
    x = torch.tensor(w.x, dtype=f32, device=dev)
    t = torch.tensor(w.t, dtype=f32, device=dev)
    N = torch.tensor(w.N, dtype=torch.int32, device=dev)
    hp = torch.tensor(w.hp, dtype=f32, device=dev)
    Q = torch.tensor(w.gp, dtype=f32, device=dev)
    s = Solver(d=w.d, H=w.H, g=w.g, N_max=w.N_max, sigma=w.sigma, tau=w.tau, tol=w.tol, max_iter=K,
               seed=w.init_seed, dtype=f32, fixed_iters=True, timing=True)
    out = s.alloc(w.n)
    s.solve(x, t, N, hp, Q, out=out)
    torch.cuda.synchronize()
    kms = []
    for _ in range(max(1, steps // 2)):
        s.solve(x, t, N, hp, Q, out=out)
        ms, nl = s.timing()
        kms.append(ms)
    fwd_ms = float(np.mean(kms))
    s.close()
    flops = float(w.n) * K * mfma_flops_per_iter_lintanh(w.N_max, w.d)
    lt = LinearTanhValue(w.d, w.N_max, w.sigma, w.tau, K, ckpt_every=50, seed=w.init_seed)
    gphi = torch.ones(w.n, dtype=f32, device=dev)
    lt.value_grad(x, t, N, hp, Q, gphi)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = max(1, steps // 5)
    e0.record()
    for _ in range(reps):
        lt.value_grad(x, t, N, hp, Q, gphi)
    e1.record()
    torch.cuda.synchronize()
    vg_ms = e0.elapsed_time(e1) / reps
    lt.close()
    return {"workload": "lintanh100: d=100, H=-<p,Ax+0.1 tanh x>+|p|^2/2, g=x^T Q x/2, 16,384 points, N=50, "
                        "K=500 fixed iterations, FP32",
            "forward_kernel_ms": fwd_ms, "forward_solves_per_s": w.n / (fwd_ms * 1e-3),
            "mfma": {"bound": "mfma", "achieved": flops / (fwd_ms * 1e-3) / 1e12, "peak": PEAK["fp32_matrix"] / 1e12,
                     "unit": "TFLOP/s", "frac": flops / (fwd_ms * 1e-3) / PEAK["fp32_matrix"],
                     "kernel": "k_lt_forward<100>", "flops_per_launch": flops},
            "value_grad_ms": vg_ms, "value_grad_points_per_s": w.n / (vg_ms * 1e-3), "ckpt_every": 50,
            "cpu_oracle": oracle_sample(w, 64) if cpu else None}


def bench_full_sets(torch, dev):
    """The batched path (persistent, default tiles, hipGraph) on the full
    quadrotor set with both trajectories written (Lax, and the Hopf
    formulation the paper uses for its quadcopter) and on the full
    pursuit-evasion set: one warm-up, then the median of two solves."""
    import workloads as W
    from paper_1803_01215_amd.solver import Solver

    out = {}
    for key, name, traj, hopf in (("quadrotor12", "quadrotor12", True, False),
                                  ("quadrotor12_hopf", "quadrotor12", True, True),
                                  ("pursuit12", "pursuit12", False, False)):
        w = W.get(name)
        td = torch.float32
        inp = (torch.tensor(w.x, dtype=td, device=dev), torch.tensor(w.t, dtype=td, device=dev),
               torch.tensor(w.N, dtype=torch.int32, device=dev), torch.tensor(w.hp, dtype=td, device=dev),
               torch.tensor(w.gp, dtype=td, device=dev))
        s = Solver(d=w.d, d_y=w.d_y, H=w.H, g=w.g, N_max=w.N_max, sigma=w.sigma, tau=w.tau, theta=w.theta,
                   tol=w.tol, max_iter=w.max_iter, seed=w.init_seed, dtype=td, graph=True, hopf=hopf)
        o = s.alloc(w.n, traj=traj)
        s.solve(*inp, out=o, traj=traj)
        torch.cuda.synchronize()
        times = []
        for _ in range(2):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            s.solve(*inp, out=o, traj=traj)
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        ms = float(np.median(times))
        conv = int((o.status == 0).sum())
        out[key] = {"points": w.n, "dtype": "f32", "max_iter": w.max_iter, "trajectories": traj,
                    "formulation": "Hopf (Algorithm 2)" if hopf else "Lax (Algorithm 1)", "ms": ms,
                     "converged": conv, "solves_per_s": conv / (ms * 1e-3),
                     "iterations": int(o.iters.to(torch.int64).sum())}
        s.close()
        del o, inp
    return out


def bench_configs(torch, dev, subset, cpu=False):
    """Batched (persistent, default tiles, hipGraph) against plain (one point
    per lane) on the other workloads: the eikonal set in full (FP64), the
    quadrotor and pursuit-evasion sets on their first `subset` points (FP32,
    20,000-iteration cap; the plain kernel streams each point's state through
    HBM every iteration, so a full-size plain run would take minutes)."""
    import workloads as W
    from paper_1803_01215_amd.solver import Solver

    out = {}
    for name, td, m in (("eikonal2d", torch.float64, None), ("quadrotor12", torch.float32, subset),
                        ("pursuit12", torch.float32, subset)):
        w = W.get(name)
        if m is not None and m < w.n:
            w = w.subset(np.arange(m))
        inp = (torch.tensor(w.x, dtype=td, device=dev), torch.tensor(w.t, dtype=td, device=dev),
               torch.tensor(w.N, dtype=torch.int32, device=dev), torch.tensor(w.hp, dtype=td, device=dev),
               torch.tensor(w.gp, dtype=td, device=dev))
        rec = {"points": w.n, "dtype": "f64" if td == torch.float64 else "f32", "max_iter": w.max_iter}
        for label, kw in (("batched", dict(graph=True)), ("plain", dict(plain=True))):
            s = Solver(d=w.d, d_y=w.d_y, H=w.H, g=w.g, N_max=w.N_max, sigma=w.sigma, tau=w.tau, theta=w.theta,
                       tol=w.tol, max_iter=w.max_iter, seed=w.init_seed, dtype=td, **kw)
            o = s.alloc(w.n)
            s.solve(*inp, out=o)
            torch.cuda.synchronize()
            times = []
            for _ in range(3 if label == "batched" else 1):  # median of 3: one launch can be an outlier
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                s.solve(*inp, out=o)
                e1.record()
                torch.cuda.synchronize()
                times.append(e0.elapsed_time(e1))
            ms = float(np.median(times))
            conv = int((o.status == 0).sum())
            rec[label] = {"ms": ms, "converged": conv, "solves_per_s": conv / (ms * 1e-3)}
            s.close()
        rec["speedup"] = rec["batched"]["solves_per_s"] / max(rec["plain"]["solves_per_s"], 1e-30)
        if cpu:
            rec["cpu_oracle"] = oracle_sample(w, {"eikonal2d": 256, "quadrotor12": 512, "pursuit12": 1024}[name])
        out[name] = rec
        if name == "quadrotor12":
            # robustness recipes (section 6): cap 5,000, then up to three more
            # phases, stopping also on a stalled value (rel. change <= 1e-7)
            rw = w.subset(np.arange(w.n))
            rw.max_iter = 5000
            s = Solver(d=rw.d, d_y=rw.d_y, H=rw.H, g=rw.g, N_max=rw.N_max, sigma=rw.sigma, tau=rw.tau,
                       theta=rw.theta, tol=rw.tol, max_iter=rw.max_iter, seed=rw.init_seed, dtype=td, graph=True,
                       restarts=3, sigma_inc=0.0, value_tol=1e-7)
            o = s.alloc(rw.n)
            s.solve(*inp, out=o)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            s.solve(*inp, out=o)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            st = np.bincount(o.status.cpu().numpy(), minlength=5)
            out["quadrotor12_recipes"] = {
                "points": rw.n, "recipe": "max_iter 5000, restarts 3, sigma_inc 0, value_tol 1e-7", "ms": ms,
                "converged": int(st[0]), "value_stalled": int(st[4]), "max_iter": int(st[1]),
                "solves_per_s": float(st[0] + st[4]) / (ms * 1e-3)}
            s.close()
        print("[configs] %s: batched %.1f ms, plain %.1f ms" % (name, rec["batched"]["ms"], rec["plain"]["ms"]),
              file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 run")
    ap.add_argument("--cpu-sample", type=int, default=65536)
    ap.add_argument("--max-iter", type=int, default=5000,
                    help="iteration cap of the headline run (points above it count as not converged)")
    ap.add_argument("--no-c5", action="store_true", help="skip the linear-tanh (d=100) forward/reverse timing")
    ap.add_argument("--configs", type=int, default=0, metavar="M",
                    help="also time batched vs plain on the eikonal, quadrotor and pursuit-evasion workloads "
                         "(the last two on their first M points)")
    ap.add_argument("--full-sets", action="store_true",
                    help="also time the batched path on the full quadrotor set (131,072 points, trajectories "
                         "written; Lax and Hopf) and the full pursuit-evasion set (262,144 points)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run one 256 MiB device copy (counter calibration for rocprofv3 --pmc)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU (the query points are independent; several GPUs would each take a "
              "share of them): run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads as W
    from paper_1803_01215_amd.solver import Solver

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    w = W.cnorm10()
    n = w.n
    cap_default = w.max_iter
    w.max_iter = args.max_iter

    def tensors(td):
        return (torch.tensor(w.x, dtype=td, device=dev), torch.tensor(w.t, dtype=td, device=dev),
                torch.tensor(w.N, dtype=torch.int32, device=dev), torch.tensor(w.hp, dtype=td, device=dev),
                torch.tensor(w.gp, dtype=td, device=dev))

    def make(td, **kw):
        return Solver(d=w.d, H=w.H, g=w.g, N_max=w.N_max, sigma=w.sigma, tau=w.tau, theta=w.theta, tol=w.tol,
                      max_iter=w.max_iter, seed=w.init_seed, dtype=td, **kw)

    def timed_steps(solver, inp, out, steps, warmup):
        for _ in range(warmup):
            solver.solve(*inp, out=out)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            solver.solve(*inp, out=out)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    # ---- batched FP32 (the headline) ------------------------------------------------
    td = torch.float32
    inp = tensors(td)
    batched = make(td, graph=True, lanes_per_point=16, nodes_per_lane=2)
    out = batched.alloc(n)
    ms_step = timed_steps(batched, inp, out, args.steps, args.warmup)
    status = out.status.cpu().numpy()
    iters = out.iters.cpu().numpy().astype(np.int64)
    conv = int((status == 0).sum())
    value = conv / (ms_step * 1e-3)

    # dominant kernel: per-launch device time from the library's HIP events on
    # the same stream, over the same number of steps (no graph, one launch)
    probe = make(td, timing=True, lanes_per_point=16, nodes_per_lane=2)
    out2 = probe.alloc(n)
    probe.solve(*inp, out=out2)
    torch.cuda.synchronize()
    kms = []
    for _ in range(args.steps):
        probe.solve(*inp, out=out2)
        ms, nl = probe.timing()
        assert nl == 1
        kms.append(ms)
    kern_ms = float(np.mean(kms))
    flops = float(sum(iters * flops_per_iter_cnorm(w.N_max, w.d)))
    achieved = flops / (kern_ms * 1e-3)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK["fp32_vector"] / 1e12, "unit": "TFLOP/s",
                "frac": achieved / PEAK["fp32_vector"],
                "traffic": measured_traffic("k_group_control_shift<float, CNorm<10>, 16, 2, false>"),
                "kernel": "k_group_control_shift<float, CNorm<10>, 16, 2, false>", "kernel_ms": kern_ms,
                "flops_per_launch": flops}

    # ---- the same with the long iteration cap (20000) -----------------------------
    w.max_iter = cap_default
    long = make(td, graph=True, lanes_per_point=16, nodes_per_lane=2)
    outl = long.alloc(n)
    ms_long = timed_steps(long, inp, outl, max(1, args.steps // 2), 1)
    conv_long = int((outl.status.cpu().numpy() == 0).sum())
    long_rec = {"max_iter": cap_default, "value": conv_long / (ms_long * 1e-3), "ms_per_step": ms_long,
                "converged": conv_long}
    long.close()
    w.max_iter = args.max_iter

    if args.copy_calib:
        src = torch.empty(64 << 20, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # ---- Hopf formulation (Algorithm 2) on the same workload, same tile and cap ---------
    hopf = make(td, graph=True, lanes_per_point=16, nodes_per_lane=2, hopf=True)
    outh = hopf.alloc(n)
    ms_hopf = timed_steps(hopf, inp, outh, max(1, args.steps // 2), 1)
    conv_hopf = int((outh.status.cpu().numpy() == 0).sum())
    hopf_rec = {"value": conv_hopf / (ms_hopf * 1e-3), "ms_per_step": ms_hopf, "converged": conv_hopf,
                "iters_p50": float(np.median(outh.iters.cpu().numpy()))}
    hopf.close()

    # ---- forward-Euler and trapezoidal discretisations, same workload, tile and cap --------
    disc_rec = {}
    for disc in ("fe", "trap"):
        sd = make(td, graph=True, lanes_per_point=16, nodes_per_lane=2, disc=disc)
        outd = sd.alloc(n)
        ms_d = timed_steps(sd, inp, outd, max(1, args.steps // 2), 1)
        conv_d = int((outd.status.cpu().numpy() == 0).sum())
        disc_rec[disc] = {"value": conv_d / (ms_d * 1e-3), "ms_per_step": ms_d, "converged": conv_d,
                          "iters_p50": float(np.median(outd.iters.cpu().numpy()))}
        sd.close()

    # ---- game Hopf formulation (Algorithm 4): Isaacs' game on the section's full grid -------
    wi = W.isaacs2()
    si = Solver(d=wi.d, d_y=wi.d_y, H=wi.H, g=wi.g, N_max=wi.N_max, sigma=wi.sigma, tau=wi.tau, theta=wi.theta,
                tol=wi.tol, max_iter=wi.max_iter, seed=wi.init_seed, dtype=td, graph=True, hopf=True)
    inp_i = (torch.tensor(wi.x, dtype=td, device=dev), torch.tensor(wi.t, dtype=td, device=dev),
             torch.tensor(wi.N, dtype=torch.int32, device=dev), torch.tensor(wi.hp, dtype=td, device=dev),
             torch.tensor(wi.gp, dtype=td, device=dev))
    outi = si.alloc(wi.n)
    ms_i = timed_steps(si, inp_i, outi, max(1, args.steps // 2), 1)
    st_i = outi.status.cpu().numpy()
    conv_i = int((st_i == 0).sum())
    isaacs_rec = {"workload": "isaacs2: Isaacs' game, H=-c(x,y)q+2|p|-sqrt(p^2+q^2)-1, g=(2.5x)^2/2-1/2-y^2/2, "
                              "73x73 grid on [-3,3]^2 x t in {0.025,0.05,0.075,0.1}, delta=0.005, game Hopf",
                  "points": wi.n, "tol": wi.tol, "max_iter": wi.max_iter, "value": conv_i / (ms_i * 1e-3),
                  "unit": "converged solves/s", "ms_per_step": ms_i, "converged": conv_i,
                  "iters_p50": float(np.median(outi.iters.cpu().numpy()))}
    si.close()

    # ---- plain FP32 -------------------------------------------------------------------
    plain = make(td, plain=True)
    outp = plain.alloc(n)
    ms_plain = timed_steps(plain, inp, outp, max(1, args.plain_steps), 1)
    conv_plain = int((outp.status.cpu().numpy() == 0).sum())
    plain_rec = {"value": conv_plain / (ms_plain * 1e-3), "ms_per_step": ms_plain, "converged": conv_plain}
    batched.close(); probe.close(); plain.close()

    # ---- batched FP64 --------------------------------------------------------------------
    fp64_rec = None
    if not args.no_fp64:
        inp64 = tensors(torch.float64)
        b64 = make(torch.float64, graph=True, lanes_per_point=16, nodes_per_lane=2)
        o64 = b64.alloc(n)
        ms64 = timed_steps(b64, inp64, o64, max(1, args.steps // 2), 1)
        c64 = int((o64.status.cpu().numpy() == 0).sum())
        it64 = o64.iters.cpu().numpy().astype(np.int64)
        b64.close()
        # the FP64 kernel's own time (library HIP events, one launch per solve)
        p64 = make(torch.float64, timing=True, lanes_per_point=16, nodes_per_lane=2)
        q64 = p64.alloc(n)
        p64.solve(*inp64, out=q64)
        k64 = []
        for _ in range(max(1, args.steps // 2)):
            p64.solve(*inp64, out=q64)
            k64.append(p64.timing()[0])
        p64.close()
        kms64 = float(np.mean(k64))
        fl64 = float(sum(it64 * flops_per_iter_cnorm(w.N_max, w.d)))
        fp64_rec = {"value": c64 / (ms64 * 1e-3), "ms_per_step": ms64, "converged": c64,
                    "roofline": {"bound": "alu", "achieved": fl64 / (kms64 * 1e-3) / 1e12,
                                 "peak": PEAK["fp64_vector"] / 1e12, "unit": "TFLOP/s",
                                 "frac": fl64 / (kms64 * 1e-3) / PEAK["fp64_vector"],
                                 "kernel": "k_group_control_shift<double, CNorm<10>, 16, 2, false>",
                                 "kernel_ms": kms64, "flops_per_launch": fl64}}

    # ---- matrix-core path (linear-tanh, d = 100): forward and reverse mode ------------------
    c5_rec = None
    if not args.no_c5:
        c5_rec = bench_lintanh(torch, dev, args.steps, cpu=not args.no_cpu)

    cfg_rec = bench_configs(torch, dev, args.configs, cpu=not args.no_cpu) if args.configs > 0 else None
    full_rec = bench_full_sets(torch, dev) if args.full_sets else None

    # ---- CPU oracle baseline on a bounded sample ------------------------------------------
    cpu_rec = oracle_sample(w, args.cpu_sample) if not args.no_cpu else None

    rec = {
        "metric": "converged (x,t) solves/sec at PDHG residual 1e-6, batched vs plain kernel",
        "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "cnorm10: d=10 state-dependent eikonal H=c(x)||p||, c=1+0.5 sin(x1)cos(x2), "
                               "g=||x-a||^2/2-1, 65,536 points x~N(0,I), t~U[0.2,1], N=32, tol 1e-6",
                   "points": n, "N": w.N_max, "d": w.d, "sigma": w.sigma, "tau": w.tau, "tile": "16 lanes x 2 nodes", "max_iter": args.max_iter,
                   "converged": conv, "iters_p50": float(np.median(iters)), "iters_p95": float(np.percentile(iters, 95)),
                   "iters_max": int(iters.max())},
        "roofline": roofline,
        "cpu_baseline": cpu_rec,
        "plain": plain_rec,
        "speedup_vs_plain": value / plain_rec["value"] if plain_rec["value"] > 0 else None,
        "fp64": fp64_rec,
        "long_cap": long_rec,
        "hopf": hopf_rec,
        "forward_euler": disc_rec["fe"],
        "trapezoid": disc_rec["trap"],
        "isaacs2_game_hopf": isaacs_rec,
        "lintanh100": c5_rec,
        "configs": cfg_rec,
        "full_sets": full_rec,
    }
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
