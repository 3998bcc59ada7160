"""Throughput benchmark: converged (x,t) solves per second at PDHG residual 1e-6.

One step = one full solve of the headline workload (every point runs the
primal-dual iteration of section 5.1 until both squared residuals are below
1e-6, or the iteration cap) with all inputs resident in HBM.

Headline workload (pursuit12): the pursuit-evasion game of two 3-D point
masses with drag, d = 12 (6 + 6), solved by Algorithm 3 (section 4.2),
262,144 points with t ~ U[0.5, 4] and N = clamp(ceil(24 t), 16, 96), so the
uneven N spans four capacity classes in one hipGraph-captured solve, FP32,
cap 20,000.  The batched path (persistent lane-group kernels with a device
queue, retire/refill, classes on parallel branches) is timed over the whole
set; the plain path (one point per lane, state in HBM, no refill) and the FP64
CPU oracle on seeded samples beside it.  The other workloads (the 2-D eikonal,
cnorm10, the quadrotor with trajectories, linear-tanh forward and reverse)
follow as extra keys, each with its own roofline and CPU baseline.

Prints one JSON line (one GPU).
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp32_vector": 157.3e12, "fp64_vector": 78.6e12, "fp32_matrix": 157.3e12}


# ---------------------------------------------------------------------------
# Algorithmic flops per point-iteration (FMA = 2 flops, a product or a sum 1;
# square roots, reciprocals, rsqrt and sin/cos are not counted; constants of a
# point, such as sigma delta or 1/(1 + sigma delta w), are counted once per
# point, not per iteration).  Counted from the kernels' source, node by node.
# ---------------------------------------------------------------------------

def flops_per_iter_cnorm(N: int, d: int) -> int:
    """H = c(x)||p||, g = ||x-a||^2/2 - c0 (also used for the norm g, whose
    node-0 shrink costs about the same):
      dual step,   nodes 1..N:   9d + 12  (stencil 3d, c(x) 3, ||v||^2 2d,
                                           shrink 5, scale d, residual 3d,
                                           grad c 4)
      primal step, nodes 1..N-1: 8d + 6   (grad 2, update 3d + 4, difference
                                           d, residual 2d, extrapolation 2d)
      node 0:                    9d       (prox 4d, residual 3d, extrap. 2d)
    plus per dual node 2 sin/cos pairs and 1 rsqrt."""
    return N * (9 * d + 12) + (N - 1) * (8 * d + 6) + 9 * d


def flops_per_iter_quad(N: int) -> int:
    """Quadrotor, d = 12 (k_group_control with the Quad family):
      dual step, nodes 1..N: 182
        stencil 36 (3 per coordinate);
        geometry at x_j 59: b = R e3/m 12, its Jacobian db 30, W and tan/sec
          products 5, dW/droll 4, sec^2 and sec tan 4, dW/dpitch 4;
        prox 51: position costate 6, angle costate W omega 6 + 5 + 5, gravity
          1, b.w 5, |b|^2 5, coefficient 4, rank-one correction 6, body-rate
          scaling 3, b.p 5;
        residual 36 (3 per coordinate);
      primal step, nodes 1..N-1: 153
        grad_x H 51: roll and pitch terms of -W^T p 14 + 9, thrust terms
          7 + 7 + 4, body-rate rows of -W^T p 5 + 5;
        update 102: positions (no gradient) 3 x (2 + 5), others 9 x (4 + 5),
          where 5 = residual 2, extrapolation 2, step 1;
      node 0: 96 (affine prox increment 3, residual 2, extrapolation 2, step 1,
        per coordinate).
    Plus 3 sin/cos pairs and a reciprocal per dual node (not counted)."""
    return N * 182 + (N - 1) * 153 + 96


def flops_per_iter_pursuit(N: int) -> int:
    """Pursuit-evasion game, 6 + 6 (k_group_game with the Pursuit family):
      dual steps (p and q blocks), nodes 1..N: 2 x 58
        stencil 18, speed |v| 5, kappa |v| 1, position costate 6, velocity
        costate 10, residual 18;
      primal steps (x descent, y ascent), nodes 1..N-1: 2 x 69
        J_F^T pi 21 (v.pi 5, ratio 1, three rows of 5), update 48 (positions
        3 x 7 with no gradient, velocities 3 x 9);
      node 0 (prox of g(., y_0) for x_0, stretch of -g for y_0): 2 x 59.
    Plus one square root per block and node and two rsqrt at node 0."""
    return N * 116 + (N - 1) * 138 + 118


def mfma_flops_per_iter_lintanh(N: int, d: int) -> int:
    """Matrix-core flops of one forward iteration of one point for the
    linear-tanh family: A x_j for the dual step at j = 1..N and A^T p_j for the
    primal step at j = 1..N-1, each a d x d by d product (FMA = 2 flops)."""
    return 2 * d * d * (2 * N - 1)


def mfma_flops_per_iter_lintanh_backward(N: int, d: int) -> int:
    """Flops of one reverse-sweep iteration of one point (k_lt_backward): the
    segment recompute of the forward products 2d^2(2N-1); the vector-Jacobian
    products A xbar_j (j < N) and A^T vbar_j (j <= N), 2d^2(2N-1); the
    outer products of dA over the same nodes, 2d^2(2N-1); and at node 0 the
    product M xbar_0 and the rank-one dM update, 4d^2."""
    return 3 * 2 * d * d * (2 * N - 1) + 4 * d * d


# ---------------------------------------------------------------------------
# Counter traffic (rocprofv3 FETCH_SIZE / WRITE_SIZE, scaled by a copy
# calibration), reported only while the kernel sources match the measurement.
# ---------------------------------------------------------------------------

KERNEL_SOURCES = ["paper_1803_01215_amd/csrc/hjpd_kernels.hpp", "paper_1803_01215_amd/csrc/hjpd_families.hpp",
                  "paper_1803_01215_amd/csrc/hjpd_device.hpp", "paper_1803_01215_amd/csrc/hjpd_api.hip"]
TRAFFIC_FILES = ["profiles/traffic_pursuit12_f32.json", "profiles/traffic_cnorm10_f32_group16x2.json"]


def kernel_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from a committed counter summary, or
    None when no summary names it or the kernel sources changed after the
    counters were taken."""
    for name in TRAFFIC_FILES:
        path = os.path.join(ROOT, name)
        if not os.path.exists(path):
            continue
        with open(path) as fh:
            rec = json.load(fh)
        if rec.get("kernel") == kernel and rec.get("sources_sha256") == kernel_sources_sha256():
            return float(rec["bytes_per_launch"])
    return None


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def iteration_histogram(iters) -> dict:
    """Counts of points per iteration range (edges 1, 10, 30, 100, ..., 30000)."""
    edges = [1, 10, 30, 100, 300, 1000, 3000, 10000, 20000, 30000]
    h, _ = np.histogram(np.asarray(iters), bins=edges)
    return {"edges": edges, "counts": [int(c) for c in h]}


def oracle_sample(w, m, threads=None):
    """The FP64 oracle on the first m points of a workload (FP32-rounded
    parameters, the GPU's stopping rule and cap), OpenMP over points on the
    host's cores: converged solves/s of the sample (fixed-iteration workloads
    count every finished point), with the sample, thread count and CPU model
    stated."""
    from oracle import oracle as O
    O.build()
    m = min(m, w.n)
    sub = w.subset(np.arange(m))
    pb = O.Problem(sub.H, sub.g, sub.d, sub.d_y, sub.hp.astype(np.float32).astype(np.float64),
                   sub.gp.astype(np.float32).astype(np.float64))
    threads = threads or int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    r = O.solve(pb, sub.x, sub.t, sub.N, sigma=sub.sigma, tau=sub.tau, theta=sub.theta, tol=sub.tol,
                max_iter=sub.max_iter, seed=sub.init_seed, N_max=sub.N_max, ids=sub.ids, threads=threads,
                fixed_iters=sub.fixed_iters)
    dt = time.perf_counter() - t0
    done = m if sub.fixed_iters else int((r.status == 0).sum())
    return {"value": done / dt, "unit": "solves/s", "cores": threads, "kind": "oracle", "cpu": cpu_model(),
            "sample": "first %d of the %d points, FP64 C oracle, cap %d, OpenMP over points, %.1f s wall, %d %s" % (
                m, w.n, sub.max_iter, dt, done, "finished" if sub.fixed_iters else "converged")}


# Tuner probe length for the quadrotor workload.  At 100 iterations per probe the
# 49..60-node class picked 32x2 or 16x4 from run to run (657 vs 621 ms per solve);
# at 400 and 1,000 it picked 16x4 in each of the four runs measured; 1,000 costs
# about 5 s of tuning.
QUAD_PROBE_ITERS = 1000


class Bench:
    def __init__(self, torch, dev):
        self.torch, self.dev = torch, dev

    def tensors(self, w, td):
        t = self.torch
        return (t.tensor(w.x, dtype=td, device=self.dev), t.tensor(w.t, dtype=td, device=self.dev),
                t.tensor(w.N, dtype=t.int32, device=self.dev), t.tensor(w.hp, dtype=td, device=self.dev),
                t.tensor(w.gp, dtype=td, device=self.dev))

    def solver(self, w, td, **kw):
        from paper_1803_01215_amd.solver import Solver
        return Solver(d=w.d, d_y=w.d_y, H=w.H, g=w.g, N_max=w.N_max, sigma=w.sigma, tau=w.tau, theta=w.theta,
                      tol=w.tol, max_iter=w.max_iter, seed=w.init_seed, dtype=td, **kw)

    def timed(self, s, inp, out, steps, warmup, traj=False):
        """Mean ms per solve over `steps` solves after `warmup` solves, HIP
        events on the solve's stream (torch's current stream)."""
        torch = self.torch
        for _ in range(warmup):
            s.solve(*inp, out=out, traj=traj)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            s.solve(*inp, out=out, traj=traj)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / max(steps, 1)

    def batched(self, w, td, steps, warmup, traj=False, plan=None, **kw):
        """The batched path, graph-replayed: ms per solve, statuses, iterations."""
        s = self.solver(w, td, graph=True, **kw)
        if plan is not None:
            s.set_plan(plan)
        inp = self.tensors(w, td)
        out = s.alloc(w.n, traj=traj)
        ms = self.timed(s, inp, out, steps, warmup, traj=traj)
        st = out.status.cpu().numpy()
        it = out.iters.cpu().numpy().astype(np.int64)
        s.close()
        del out, inp
        conv = int((st == 0).sum())
        return {"ms": ms, "converged": conv, "solves_per_s": conv / (ms * 1e-3), "status": st, "iters": it}

    def launches(self, w, td, flops_fn, peak, traj=False, reps=3, plan=None, **kw):
        """Per capacity class of the plan: one eager solve of just the class's
        points (same plan and tile), timed by the library with HIP events on
        the class launch's own stream (mean over reps), so no other class
        shares the GPU or a hardware queue with it.  Returns per class the
        launch's ms, N range, tile, its points' algorithmic flops (their
        iterations times the count at their N) and the resulting rate."""
        s = self.solver(w, td, timing=True, **kw)
        if plan is not None:
            s.set_plan(plan)
        classes = s.plan()[0]
        s.close()
        N = np.asarray(w.N)
        out = []
        lo = 1
        for hi, L, K in classes:
            sel = np.nonzero((N >= lo) & (N <= hi))[0]
            rec = {"N_lo": lo, "N_hi": hi, "L": L, "K": K, "points": int(len(sel)), "ms": 0.0, "flops": 0.0,
                   "tflops": 0.0, "frac": 0.0}
            lo = hi + 1
            if len(sel) == 0:
                out.append(rec)
                continue
            sub = w.subset(sel)
            s = self.solver(sub, td, timing=True, **kw)
            s.set_plan(classes)
            inp = self.tensors(sub, td)
            o = s.alloc(sub.n, traj=traj)
            s.solve(*inp, out=o, traj=traj)
            self.torch.cuda.synchronize()
            ms = []
            for _ in range(reps):
                s.solve(*inp, out=o, traj=traj)
                lt = [a for a in s.launch_timings() if a["N_lo"] == rec["N_lo"]]
                ms.append(lt[0]["ms"])
            it = o.iters.cpu().numpy().astype(np.int64)
            st = o.status.cpu().numpy()
            s.close()
            del o, inp
            fl = np.array([flops_fn(int(n)) for n in sub.N], dtype=np.float64)
            ok = st != 3
            rec["ms"] = float(np.mean(ms))
            rec["flops"] = float(np.sum(it[ok] * fl[ok]))
            rec["tflops"] = rec["flops"] / (rec["ms"] * 1e-3) / 1e12
            rec["frac"] = rec["flops"] / (rec["ms"] * 1e-3) / peak
            out.append(rec)
        return out

    def tune(self, w, td, probe_iters=100, **kw):
        """The library's autotuner on the whole workload: the chosen plan
        [(hi, L, K), ...] and the seconds tuning took (0 when the plan came
        from the tuning cache named by $HJPD_TUNE_CACHE)."""
        s = self.solver(w, td, **kw)
        plan, cached = s.plan()
        if cached:
            s.close()
            return plan, 0.0
        inp = self.tensors(w, td)
        t0 = time.perf_counter()
        s.autotune(*inp, probe_iters=probe_iters)
        self.torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        plan = s.plan()[0]
        s.close()
        return plan, dt

    def plain(self, w, td, steps=1):
        s = self.solver(w, td, plain=True)
        inp = self.tensors(w, td)
        out = s.alloc(w.n)
        ms = self.timed(s, inp, out, steps, 1)
        conv = int((out.status.cpu().numpy() == 0).sum())
        s.close()
        return {"ms": ms, "converged": conv, "solves_per_s": conv / (ms * 1e-3)}


def copy_calibration(torch, dev):
    """One device copy of 256 MiB (read 256 MiB, write 256 MiB): the scale of
    rocprofv3's FETCH_SIZE and WRITE_SIZE counters for known traffic."""
    src = torch.empty(64 << 20, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def fma_calibration(rounds=5000):
    """What the vector ALUs sustain for single (not packed) FMAs, the form
    every solver kernel is compiled to: the library's calibration kernel over
    independent chains per lane x resident waves per SIMD, FP32 and FP64.
    TFLOP/s from exact flop counts and HIP-event launch times."""
    from paper_1803_01215_amd import hjpd as C
    out = {}
    for name, dt, grid in (("fp32", C.HJPD_F32, [(c, w) for c in (1, 2, 4, 8, 16) for w in (1, 2, 4, 8)]),
                           ("fp64", C.HJPD_F64, [(c, w) for c in (1, 4, 8) for w in (1, 2, 8)])):
        rows = []
        for c, w in grid:
            r = C.hjpd_calibrate_fma(dt, c, w, rounds)
            rows.append({"chains": c, "waves_per_simd": w, "ms": r["ms"],
                         "tflops": r["flops"] / (r["ms"] * 1e-3) / 1e12})
        out[name] = rows
        out[name + "_best_tflops"] = max(r["tflops"] for r in rows)
    return out


def roofline_of(launches, kernel_fmt, dtype_name, peak, bound="alu"):
    """The dominant launch (the class with the longest kernel time) and every class's figures."""
    dom = max(launches, key=lambda a: a["ms"])
    kernel = kernel_fmt % (dtype_name, dom["L"], dom["K"])
    return {"bound": bound, "achieved": dom["tflops"], "peak": peak / 1e12, "unit": "TFLOP/s", "frac": dom["frac"],
            "traffic": measured_traffic(kernel), "kernel": kernel, "kernel_ms": dom["ms"],
            "flops_per_launch": dom["flops"], "class_N": [dom["N_lo"], dom["N_hi"]],
            "launches": [{k: a[k] for k in ("N_lo", "N_hi", "L", "K", "ms", "points", "tflops", "frac")}
                         for a in launches]}


def bench_c5(B, steps, cpu):
    """Linear-tanh, d = 100: forward solves/s and matrix-core throughput at
    K = 500 fixed iterations, and hjpd_value_grad (forward with checkpoints
    every 50 + reverse sweep + reductions), with the reverse-sweep kernel
    timed on its own."""
    import workloads as W
    from paper_1803_01215_amd.autograd import LinearTanhValue
    torch = B.torch
    w = W.lintanh100()
    K = w.max_iter
    f32 = torch.float32
    x, t, N, hp, Q = B.tensors(w, f32)
    s = B.solver(w, f32, fixed_iters=True, timing=True)
    out = s.alloc(w.n)
    s.solve(x, t, N, hp, Q, out=out)
    torch.cuda.synchronize()
    kms = []
    for _ in range(max(1, steps // 2)):
        s.solve(x, t, N, hp, Q, out=out)
        kms.append(s.timing()[0])
    fwd_ms = float(np.mean(kms))
    s.close()
    flops = float(w.n) * K * mfma_flops_per_iter_lintanh(w.N_max, w.d)
    lt = LinearTanhValue(w.d, w.N_max, w.sigma, w.tau, K, ckpt_every=50, seed=w.init_seed, timing=True)
    gphi = torch.ones(w.n, dtype=f32, device=B.dev)
    lt.value_grad(x, t, N, hp, Q, gphi)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = max(1, steps // 5)
    bms = []
    e0.record()
    for _ in range(reps):
        lt.value_grad(x, t, N, hp, Q, gphi)
        bms.append(lt.solver.timing()[0])
    e1.record()
    torch.cuda.synchronize()
    vg_ms = e0.elapsed_time(e1) / reps
    bwd_ms = float(np.mean(bms))
    lt.close()
    bflops = float(w.n) * K * mfma_flops_per_iter_lintanh_backward(w.N_max, w.d)
    return {"workload": "lintanh100: d=100, H=-<p,Ax+0.1 tanh x>+|p|^2/2, g=x^T Q x/2, 16,384 points, N=50, "
                        "K=500 fixed iterations, FP32",
            "forward_kernel_ms": fwd_ms, "forward_solves_per_s": w.n / (fwd_ms * 1e-3),
            "roofline": {"bound": "mfma", "achieved": flops / (fwd_ms * 1e-3) / 1e12, "peak": PEAK["fp32_matrix"] / 1e12,
                         "unit": "TFLOP/s", "frac": flops / (fwd_ms * 1e-3) / PEAK["fp32_matrix"],
                         "kernel": "k_lt_forward<100>", "flops_per_launch": flops, "traffic": None},
            "value_grad_ms": vg_ms, "value_grad_points_per_s": w.n / (vg_ms * 1e-3), "ckpt_every": 50,
            "backward_kernel_ms": bwd_ms,
            "backward_roofline": {"bound": "mfma", "achieved": bflops / (bwd_ms * 1e-3) / 1e12,
                                  "peak": PEAK["fp32_matrix"] / 1e12, "unit": "TFLOP/s",
                                  "frac": bflops / (bwd_ms * 1e-3) / PEAK["fp32_matrix"],
                                  "kernel": "k_lt_backward<100>", "flops_per_launch": bflops, "traffic": None},
            "cpu_baseline": oracle_sample(w, 256) if cpu else None}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baselines")
    ap.add_argument("--no-extra", action="store_true", help="headline workload only")
    ap.add_argument("--plain-sample", type=int, default=4096,
                    help="points of the seeded sample the plain kernel (and the batched path beside it) solves")
    ap.add_argument("--cpu-sample", type=int, default=6144,
                    help="headline points the CPU oracle solves (about 10 s on 16 host threads)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run one 256 MiB device copy (counter calibration for rocprofv3 --pmc)")
    ap.add_argument("--tune-cache", metavar="FILE",
                    help="tuning cache: the headline's plan is read from FILE if recorded there, else tuned and "
                         "recorded (so a profiled run can repeat the measured plan without tuning)")
    ap.add_argument("--calibrate", action="store_true",
                    help="only the FMA calibration sweep (for hardware-counter runs), one JSON line")
    ap.add_argument("--profile", nargs="?", const="pursuit12",
                    choices=["pursuit12", "cnorm10", "quadrotor12", "lintanh100"],
                    help="one workload's solves only, for rocprofv3: pursuit12 (the headline; plan from "
                         "--tune-cache or tuned), cnorm10 (FP32, cap 5,000), quadrotor12 (plan from --tune-cache "
                         "or tuned, trajectories written) or lintanh100 (forward and value_grad)")
    args = ap.parse_args()
    if args.tune_cache:
        os.environ["HJPD_TUNE_CACHE"] = os.path.abspath(args.tune_cache)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU (the query points are independent; several GPUs would each take a "
              "share of them): run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    B = Bench(torch, torch.device("cuda:0"))
    f32, f64 = torch.float32, torch.float64
    cpu = not args.no_cpu

    def log(msg):
        print("[bench] " + msg, file=sys.stderr, flush=True)

    if args.calibrate:
        print(json.dumps({"fma_calibration": fma_calibration()}))
        return

    if args.profile == "lintanh100":
        r = bench_c5(B, args.steps, False)
        print(json.dumps({"profile": "lintanh100 forward and value_grad", "steps": args.steps,
                          "forward_kernel_ms": r["forward_kernel_ms"], "backward_kernel_ms": r["backward_kernel_ms"],
                          "value_grad_ms": r["value_grad_ms"]}))
        return

    if args.profile == "quadrotor12":
        wq = W.quadrotor12()
        qplan, _ = B.tune(wq, f32, probe_iters=QUAD_PROBE_ITERS)
        q = B.batched(wq, f32, args.steps, args.warmup, traj=True, plan=qplan)
        cls, lo = [], 1
        for hi, L, K in qplan:
            m = (wq.N >= lo) & (wq.N <= hi)
            cls.append({"N_lo": lo, "N_hi": hi, "L": L, "K": K, "points": int(m.sum()),
                        "iters_sum": int(q["iters"][m].sum())})
            lo = hi + 1
        print(json.dumps({"profile": "quadrotor12 solves", "plan": qplan, "steps": args.steps,
                          "warmup": args.warmup, "ms_per_step": q["ms"], "converged": q["converged"],
                          "classes": cls}))
        return

    if args.profile == "cnorm10":
        wc = W.cnorm10()
        wc.max_iter = 5000
        c = B.batched(wc, f32, args.steps, args.warmup)
        if args.copy_calib:
            copy_calibration(torch, B.dev)
        print(json.dumps({"profile": "cnorm10 FP32 solves", "steps": args.steps, "warmup": args.warmup,
                          "ms_per_step": c["ms"], "converged": c["converged"], "points": wc.n,
                          "iters_sum": int(c["iters"].sum())}))
        return

    # ---- headline: pursuit-evasion, full set, one graph ------------------------------------
    w = W.pursuit12()
    plan, tune_s = B.tune(w, f32)
    log("pursuit12 tuned plan %s (%.1f s)" % (plan, tune_s))
    head = B.batched(w, f32, args.steps, args.warmup, plan=plan)
    log("pursuit12 batched %.1f ms, %d converged" % (head["ms"], head["converged"]))
    if args.profile:
        if args.copy_calib:
            copy_calibration(torch, B.dev)
        # per class: points and summed iterations of one solve (to put counters per wave-iteration)
        cls, lo = [], 1
        for hi, L, K in plan:
            m = (w.N >= lo) & (w.N <= hi)
            cls.append({"N_lo": lo, "N_hi": hi, "L": L, "K": K, "points": int(m.sum()),
                        "iters_sum": int(head["iters"][m].sum())})
            lo = hi + 1
        print(json.dumps({"profile": "pursuit12 headline solves", "plan": plan, "steps": args.steps,
                          "warmup": args.warmup, "ms_per_step": head["ms"], "converged": head["converged"],
                          "classes": cls}))
        return
    dflt = B.batched(w, f32, 3, 1)
    norefill = B.batched(w, f32, 2, 1, plan=plan, refill=False)
    log("pursuit12 default plan %.1f ms, no refill %.1f ms" % (dflt["ms"], norefill["ms"]))
    # the paper's recipe for games (section 6.2): sigma raised by 20 at each cap, continuing from the iterate
    wr = W.pursuit12()
    wr.max_iter = 5000
    rcp = B.batched(wr, f32, max(1, args.steps // 2), 1, plan=plan, restarts=3, sigma_inc=20.0)
    log("pursuit12 with the sigma recipe %.1f ms, %d converged" % (rcp["ms"], rcp["converged"]))
    lts = B.launches(w, f32, flops_per_iter_pursuit, PEAK["fp32_vector"], plan=plan)
    roofline = roofline_of(lts, "k_group_game<%s, Pursuit, %d, %d>", "float", PEAK["fp32_vector"])
    sub = w.subset(np.arange(min(args.plain_sample, w.n)))
    plain = B.plain(sub, f32)
    bsub = B.batched(sub, f32, 3, 1)
    bsub.pop("status"); bsub.pop("iters")
    log("pursuit12 sample: plain %.1f ms, batched %.1f ms" % (plain["ms"], bsub["ms"]))
    cpu_rec = oracle_sample(w, args.cpu_sample) if cpu else None
    it = head["iters"]
    st = head["status"]
    value = head["solves_per_s"]

    rec = {
        "metric": "converged (x,t) solves/sec at PDHG residual 1e-6, batched vs plain kernel",
        "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "pursuit12: pursuit-evasion game, two 3-D point masses with drag 0.1, d=12 (6+6), "
                               "H=<p,f0>-|B_p^T p|^2/2+|B_e^T p|^2/8 (paper convention: its negative), "
                               "g=|r_P-r_E|-0.5, 262,144 points, r~U[-2,2]^3, v~U[-0.5,0.5]^3, t~U[0.5,4], "
                               "N=clamp(ceil(24t),16,96), Algorithm 3, tol 1e-6, cap 20,000, one hipGraph",
                   "points": w.n, "N_range": [int(w.N.min()), int(w.N.max())], "d": w.d, "sigma": w.sigma,
                   "tau": w.tau, "max_iter": w.max_iter,
                   "plan": {"classes": [{"N_hi": hi, "lanes_per_point": L, "nodes_per_lane": K,
                                         "points_per_wavefront": 64 // L} for hi, L, K in plan],
                            "source": "hjpd_autotune on this workload (100 fixed probe iterations), %.1f s" % tune_s},
                   "converged": head["converged"], "status_counts": np.bincount(st, minlength=4).tolist(),
                   "iters_p50": float(np.median(it)), "iters_p95": float(np.percentile(it, 95)),
                   "iters_max": int(it.max()), "iters_hist": iteration_histogram(it)},
        "roofline": roofline,
        "cpu_baseline": cpu_rec,
        "plain": dict(plain, sample="first %d points" % sub.n),
        "batched_same_sample": dict(bsub, sample="first %d points" % sub.n),
        "speedup_vs_plain": bsub["solves_per_s"] / plain["solves_per_s"] if plain["solves_per_s"] > 0 else None,
        "default_plan": {"ms_per_step": dflt["ms"], "converged": dflt["converged"], "value": dflt["solves_per_s"]},
        "no_refill": {"ms_per_step": norefill["ms"], "converged": norefill["converged"],
                      "value": norefill["solves_per_s"],
                      "what": "same kernels, plan and queue order; one point per lane group, a group for every "
                              "point (a wave stays until its slowest point stops)"},
        "sigma_recipe": {"what": "section 6.2's recipe for games: cap 5,000 iterations, then sigma += 20 (tau = "
                                 "sigma0 tau0 / sigma) continuing from the iterate, at most 3 times; same plan",
                         "ms_per_step": rcp["ms"], "converged": rcp["converged"], "value": rcp["solves_per_s"],
                         "status_counts": [int(c) for c in np.bincount(rcp["status"], minlength=5)],
                         "iters_p50": float(np.median(rcp["iters"])),
                         "iters_hist": iteration_histogram(rcp["iters"])},
    }
    del head, dflt, norefill, rcp

    if not args.no_extra:
        # ---- C3: quadrotor, full set, both trajectories written --------------------------------
        wq = W.quadrotor12()
        qplan, qtune_s = B.tune(wq, f32, probe_iters=QUAD_PROBE_ITERS)
        q = B.batched(wq, f32, max(1, args.steps // 3), 1, traj=True, plan=qplan)
        log("quadrotor12 tuned plan %s; batched %.1f ms, %d converged" % (qplan, q["ms"], q["converged"]))
        qd = B.batched(wq, f32, 2, 1, traj=True)
        qn = B.batched(wq, f32, 2, 1, traj=True, plan=qplan, refill=False)
        qlts = B.launches(wq, f32, flops_per_iter_quad, PEAK["fp32_vector"], traj=True, reps=2, plan=qplan)
        qs = wq.subset(np.arange(min(args.plain_sample, wq.n)))
        qp = B.plain(qs, f32)
        qb = B.batched(qs, f32, 3, 1)
        qb.pop("status"); qb.pop("iters")
        # the Hopf formulation (Algorithm 2) and the weighted discretisations (forward Euler,
        # trapezoid), default plan
        qw = {}
        for key, kw in (("hopf", dict(hopf=True)), ("forward_euler", dict(disc="fe")), ("trapezoid", dict(disc="trap"))):
            r = B.batched(wq, f32, 1, 1, traj=True, **kw)
            qw[key] = {"ms_per_step": r["ms"], "converged": r["converged"], "value": r["solves_per_s"],
                       "status_counts": np.bincount(r["status"], minlength=4).tolist()}
        log("quadrotor12 Hopf %.1f ms, forward Euler %.1f ms, trapezoid %.1f ms" % (
            qw["hopf"]["ms_per_step"], qw["forward_euler"]["ms_per_step"], qw["trapezoid"]["ms_per_step"]))
        rec["quadrotor12"] = {
            "workload": "quadrotor12: 12-state quadrotor-like control, cost |u|^2/2, g=|x|^2/2, 131,072 points "
                        "x~U[-1,1]^12, t~U[0.5,3], N=ceil(t/0.05), Algorithm 1, tol 1e-6, cap 20,000, both "
                        "trajectories written, FP32, one hipGraph",
            "value": q["solves_per_s"], "unit": "converged solves/s", "ms_per_step": q["ms"],
            "converged": q["converged"], "status_counts": np.bincount(q["status"], minlength=4).tolist(),
            "iters_p50": float(np.median(q["iters"])), "iters_hist": iteration_histogram(q["iters"]),
            "roofline": roofline_of(qlts, "k_group_control<%s, Quad, %d, %d>", "float", PEAK["fp32_vector"]),
            "plan": [[hi, L, K] for hi, L, K in qplan],
            "default_plan": {"ms_per_step": qd["ms"], "converged": qd["converged"], "value": qd["solves_per_s"]},
            "no_refill": {"ms_per_step": qn["ms"], "converged": qn["converged"], "value": qn["solves_per_s"]},
            "plain": dict(qp, sample="first %d points" % qs.n),
            "batched_same_sample": dict(qb, sample="first %d points" % qs.n),
            "speedup_vs_plain": qb["solves_per_s"] / qp["solves_per_s"] if qp["solves_per_s"] > 0 else None,
            "cpu_baseline": oracle_sample(wq, 512) if cpu else None, **qw}
        del q

        # ---- C2: cnorm10 (state-dependent eikonal, d = 10), FP32 and FP64 ------------------------
        wc = W.cnorm10()
        wc.max_iter = 5000
        c = B.batched(wc, f32, args.steps, 1)
        clts = B.launches(wc, f32, lambda n: flops_per_iter_cnorm(n, wc.d), PEAK["fp32_vector"])
        cp = B.plain(wc, f32)
        c64 = B.batched(wc, f64, max(1, args.steps // 2), 1)
        c64lts = B.launches(wc, f64, lambda n: flops_per_iter_cnorm(n, wc.d), PEAK["fp64_vector"])
        extra = {}
        for key, kw in (("hopf", dict(hopf=True)), ("forward_euler", dict(disc="fe")), ("trapezoid", dict(disc="trap"))):
            r = B.batched(wc, f32, max(1, args.steps // 2), 1, **kw)
            extra[key] = {"ms_per_step": r["ms"], "converged": r["converged"], "value": r["solves_per_s"]}
        rec["cnorm10"] = {
            "workload": "cnorm10: d=10 state-dependent eikonal H=c(x)||p||, c=1+0.5 sin(x1)cos(x2), g=||x-a||^2/2-1, "
                        "65,536 points x~N(0,I), t~U[0.2,1], N=32, tol 1e-6, cap 5,000, FP32, one hipGraph",
            "value": c["solves_per_s"], "unit": "converged solves/s", "ms_per_step": c["ms"],
            "converged": c["converged"], "iters_p50": float(np.median(c["iters"])),
            "iters_hist": iteration_histogram(c["iters"]),
            "roofline": roofline_of(clts, "k_group_control_shift<%s, CNorm<10>, %d, %d, false>", "float",
                                    PEAK["fp32_vector"]),
            "plain": cp, "speedup_vs_plain": c["solves_per_s"] / cp["solves_per_s"] if cp["solves_per_s"] else None,
            "fp64": {"value": c64["solves_per_s"], "ms_per_step": c64["ms"], "converged": c64["converged"],
                     "roofline": roofline_of(c64lts, "k_group_control_shift<%s, CNorm<10>, %d, %d, false>", "double",
                                             PEAK["fp64_vector"])},
            "cpu_baseline": oracle_sample(wc, 16384) if cpu else None, **extra}
        log("cnorm10 batched %.2f ms" % c["ms"])

        # ---- C1: 2-D eikonal, FP64 ---------------------------------------------------------------
        we = W.eikonal2d()
        e = B.batched(we, f64, args.steps, 2)
        elts = B.launches(we, f64, lambda n: flops_per_iter_cnorm(n, we.d), PEAK["fp64_vector"])
        ep = B.plain(we, f64, steps=3)
        rec["eikonal2d"] = {
            "workload": "eikonal2d: H=||p||, g=||x||-1, 256 points x~U[-2,2]^2, t=1, N=16, tol 1e-8, cap 5,000, FP64",
            "value": e["solves_per_s"], "unit": "converged solves/s", "ms_per_step": e["ms"],
            "converged": e["converged"], "iters_hist": iteration_histogram(e["iters"]),
            "roofline": roofline_of(elts, "k_group_control_shift<%s, CNorm<2>, %d, %d, false>", "double",
                                    PEAK["fp64_vector"]),
            "plain": ep, "speedup_vs_plain": e["solves_per_s"] / ep["solves_per_s"] if ep["solves_per_s"] else None,
            "cpu_baseline": oracle_sample(we, 256) if cpu else None}

        # ---- C5: linear-tanh, d = 100, forward and reverse ----------------------------------------
        rec["lintanh100"] = bench_c5(B, args.steps, cpu)
        log("lintanh100 done")

        # ---- game Hopf formulation (Algorithm 4): Isaacs' game on the section's full grid ----------
        wi = W.isaacs2()
        i = B.batched(wi, f32, max(1, args.steps // 2), 1, hopf=True)
        rec["isaacs2_game_hopf"] = {
            "workload": "isaacs2: Isaacs' game, H=-c(x,y)q+2|p|-sqrt(p^2+q^2)-1, g=(2.5x)^2/2-1/2-y^2/2, 73x73 grid "
                        "on [-3,3]^2 x t in {0.025,0.05,0.075,0.1}, delta=0.005, game Hopf, tol 1e-8, FP32",
            "points": wi.n, "value": i["solves_per_s"], "unit": "converged solves/s", "ms_per_step": i["ms"],
            "converged": i["converged"], "iters_p50": float(np.median(i["iters"]))}
        # ---- Algorithm 3 on the same grid: node 0 by the proxes of e and -h --------------------------
        il = B.batched(wi, f32, max(1, args.steps // 2), 1)
        rec["isaacs2_game_lax"] = {
            "workload": "isaacs2 as above, Algorithm 3 (initial cost g(x_0, y_0) itself), tol 1e-8, FP32",
            "points": wi.n, "value": il["solves_per_s"], "unit": "converged solves/s", "ms_per_step": il["ms"],
            "converged": il["converged"], "iters_p50": float(np.median(il["iters"]))}

    # what single FMAs sustain on this GPU (context for the FP32 roofline fractions)
    rec["fma_calibration"] = fma_calibration()
    log("fma calibration: fp32 best %.1f TFLOP/s, fp64 best %.1f TFLOP/s" % (
        rec["fma_calibration"]["fp32_best_tflops"], rec["fma_calibration"]["fp64_best_tflops"]))

    if args.copy_calib:
        copy_calibration(torch, B.dev)

    print(json.dumps(rec))


if __name__ == "__main__":
    main()
