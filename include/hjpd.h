/*
 * hjpd — grid-free Hamilton-Jacobi solves on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the per-point primal-dual splitting method of Lin, Chow and Osher,
 * "Splitting methods for Hamilton-Jacobi equations arising in optimal control
 * and differential games" (arXiv 1803.01215).  For every query point (x, t)
 * the library solves the time-discretised generalized Lax saddle problem
 * (section 4.1, eq. disclaxBE; games: section 4.2, eq. discgenlaxhopfdg)
 *
 *   phi(x,t) ~ max_{p_1..p_N} min_{x_0..x_{N-1}} g(x_0)
 *              + sum_{j=1..N} <p_j, x_j - x_{j-1}> - delta sum_{j=1..N} H(x_j, p_j, s_j),
 *   x_N = x, delta = t/N, s_j = j delta,
 *
 * by the PDHG (Chambolle-Pock) type iteration of section 5.1, Algorithm 1
 * (step-by-step in Appendix A.1.1; games: Algorithm 3 / Appendix A.2.1),
 * and returns the value phi(x,t), the trajectory x_0..x_N and the
 * multipliers (costates) p_0..p_N.  Points are independent: the paper notes
 * the method is embarrassingly parallel over query points (section 7).
 *
 * Conventions shared by every entry point
 *  - Every array argument is caller-owned DEVICE memory (hipMalloc'd or a
 *    PyTorch CUDA tensor) unless stated otherwise.  The library never frees it.
 *  - Floating-point arrays use the context's dtype (float or double).
 *  - Layouts are row-major with the point index slowest:
 *      x        [n][d]               query states
 *      t        [n]                  horizons t > 0
 *      N        [n]  int32           time intervals per point, 1 <= N <= N_max
 *      phi      [n]                  values
 *      iters    [n]  int32           iterations performed
 *      status   [n]  int32           per-point HJPD_PT_* code
 *      x_traj   [n][N_max+1][d]      trajectory x_0..x_N (nodes > N untouched)
 *      p_traj   [n][N_max+1][d]      multipliers p_0..p_N (p_0 = 0)
 *    For games the d coordinates of a node are (x, y): pursuer/minimiser
 *    block first (d - d_y values), evader/maximiser block last (d_y); the
 *    multiplier arrays hold (p, q) in the same order, and the evader's
 *    costate is -q (section 4.2).
 *  - Calls are asynchronous: work is enqueued on `stream` (a hipStream_t; NULL
 *    means the default stream) and outputs are valid once the stream has
 *    completed.  A solve with several capacity classes runs up to three of
 *    them (those of largest N) on the context's own streams, forked from
 *    `stream` by an event after the work already on it and joined back to it
 *    before the call's work ends, and the others on `stream`, so ordering with
 *    respect to `stream` is as if everything ran on it.  Calls
 *    on one context must not overlap in time (the context's work queue, side
 *    streams and scratch are shared by its calls).
 *  - Return codes are HJPD_* below; on a non-OK return hjpd_last_error()
 *    gives a message (thread-local, valid until the next call on the thread).
 *    Non-convergence is not an error: it is reported per point in `status`.
 */
#ifndef HJPD_H
#define HJPD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hjpd_ctx hjpd_ctx; /* opaque; created and owned by the library */

/* Return codes. */
enum {
    HJPD_OK = 0,
    HJPD_EINVAL = 1,       /* invalid argument (checked before any device work) */
    HJPD_ENOMEM = 2,       /* device or host allocation failed */
    HJPD_EDEVICE = 3,      /* a HIP call failed (no device, launch failure, ...) */
    HJPD_EUNSUPPORTED = 4  /* valid but not supported (family pair, dimension, N_max) */
};

/* Per-point status written to status[i]. */
enum {
    HJPD_PT_CONVERGED = 0, /* ||x^{k+1}-x^k||^2 < tol and ||p^{k+1}-p^k||^2 < tol (games: also y, q) */
    HJPD_PT_MAXITER = 1,   /* max_iter iterations done without meeting the rule */
    HJPD_PT_NONFINITE = 2, /* a residual, the value or an output became Inf/NaN */
    HJPD_PT_BADINPUT = 3,  /* t <= 0 or not finite, N < 1 or N > N_max, or x not finite */
    HJPD_PT_VALUE_STALLED = 4 /* recipes: stopped by the value-change rule after the cap */
};

/*
 * Hamiltonian families.  H is given here in the paper's initial-value
 * convention H = max_u { <f(x,u), p> - L(x,u) } with time-reversed dynamics
 * (section 2.1).  Parameters are passed per call in `h_params` (device array
 * of the context's dtype):
 *
 *  HJPD_H_CNORM          H = c(x) ||p||_2, c(x) = 1 + alpha sin(x_1) cos(x_2)
 *                        (state-dependent eikonal, section 6.1; dynamics
 *                        f = c(x) u, ||u|| <= 1).  h_params = [alpha].
 *                        d in {2, 3, 4, 10}.
 *  HJPD_H_QUADROTOR      d = 12, state (r, v, eta, omega) = position, velocity,
 *                        Euler angles (roll, pitch, yaw), body rates.  Physical
 *                        dynamics r' = v, v' = (u_1/m) R(eta) e_3 - g_z e_3,
 *                        eta' = W(eta) omega, omega' = J^{-1} u_{2:4},
 *                        R = Rz(yaw) Ry(pitch) Rx(roll), cost |u|^2/2:
 *                        H = -<p, f0(x)> + ((b.p_v)^2 + sum_i (p_omega,i/J_i)^2)/2,
 *                        b = R e_3 / m; the pitch inside W is clamped to [-c, c].
 *                        h_params = [m, J_1, J_2, J_3, g_z, c].
 *  HJPD_H_PURSUIT_EVASION d = 12, d_y = 6: two 3-D point masses with drag,
 *                        (r, v)' = (v, -kappa |v| v + u); pursuer cost
 *                        |u_P|^2/2, evader reward |u_E|^2/(2 w_E).  In the game
 *                        variables H(x,y,p,q) = -<p,F(x)> + <q,F(y)>
 *                        + w_P |p_v|^2/2 - w_E |q_v|^2/2 (costate (p,-q)).
 *                        h_params = [kappa, w_P, w_E].
 *  HJPD_H_LINEAR_TANH    H = -<p, A x + eps tanh(x)> + |p|^2/2 (physical
 *                        dynamics A x + eps tanh x + u, cost |u|^2/2).
 *                        h_params = [eps, A (d*d, row-major)].  float32,
 *                        d in {16, 32, 100, 128}, N_max <= 64.
 *  HJPD_H_ISAACS         Isaacs' game of section 6.3, d = 2, d_y = 1 (scalar
 *                        players x and y): x' = 2 beta + sin(alpha),
 *                        y' = -c(x,y) + cos(alpha), running cost 1, so
 *                        H(x,y,p,q) = -c(x,y) q + 2|p| - sqrt(p^2 + q^2) - 1
 *                        (costate (p,-q) in the game formulation), bump speed
 *                        c = b0 (1 + b1 exp(-b2 |(x,y) - (cx,cy)|^2)).
 *                        h_params = [b0, b1, b2, cx, cy].  With
 *                        g = HJPD_G_SADDLE_QUAD, persistent kernel: the game
 *                        Hopf formulation (HJPD_HOPF, Algorithm 4), or
 *                        Algorithm 3 without it (node 0 by the proxes of e
 *                        and of -h, value g(x_0, y_0) + ...).
 */
enum { HJPD_H_CNORM = 0, HJPD_H_QUADROTOR = 1, HJPD_H_PURSUIT_EVASION = 2, HJPD_H_LINEAR_TANH = 3,
       HJPD_H_ISAACS = 4 };

/*
 * Initial-cost families g (g_params: device array of the context's dtype).
 *  HJPD_G_NORM        g = ||x||_2 - r.                    g_params = [r]
 *  HJPD_G_QUAD_SHIFT  g = ||x - a||^2/2 - c0.             g_params = [c0, a_1..a_d]
 *  HJPD_G_PAIR_DIST   g = ||r_P - r_E||_2 - r (games; positions are the first
 *                     three coordinates of each block).   g_params = [r]
 *  HJPD_G_QUAD_FORM   g = x^T Q_s x / 2, Q_s = (Q + Q^T)/2. g_params = [Q (d*d)]
 *  HJPD_G_SADDLE_QUAD g(x,y) = e(x) + h(y), e = (a x)^2/2 - c0 convex,
 *                     h = -(b y)^2/2 concave (games, scalar players); the
 *                     game Hopf formulation uses e*(p) = p^2/(2a^2) + c0 and
 *                     h_*(q) = -q^2/(2b^2).       g_params = [c0, a, b]
 * Supported pairs: CNORM with NORM or QUAD_SHIFT; QUADROTOR with QUAD_SHIFT;
 * PURSUIT_EVASION with PAIR_DIST; LINEAR_TANH with QUAD_FORM; ISAACS with
 * SADDLE_QUAD.
 */
enum { HJPD_G_NORM = 0, HJPD_G_QUAD_SHIFT = 1, HJPD_G_PAIR_DIST = 2, HJPD_G_QUAD_FORM = 3, HJPD_G_SADDLE_QUAD = 4 };

enum { HJPD_F32 = 0, HJPD_F64 = 1 };

/* desc.flags */
enum {
    HJPD_PERSISTENT = 0,        /* default: persistent lane-group kernel with a device work queue */
    HJPD_PLAIN = 1u << 0,       /* one point per lane, whole batch in one launch, no refill */
    HJPD_FIXED_ITERS = 1u << 1, /* run exactly max_iter iterations (no tolerance stop) */
    HJPD_GRAPH = 1u << 2,       /* capture the solve in a hipGraph and replay it on repeat calls */
    HJPD_TIMING = 1u << 3,      /* record HIP events around the main kernels (hjpd_get_timing) */
    HJPD_NO_ORDER_HINT = 1u << 4, /* queue points of one N in input order; by default points that start
                                    far from the minimiser of g are handed out first (order only,
                                    results are unchanged) */
    HJPD_HOPF = 1u << 5,         /* Hopf formulation (section 4.1 eq. dischopf, Algorithm 2) instead of
                                    Lax (Algorithm 1): nodes 1..N, no x_0; the dual step at j = 1 is the
                                    joint prox of g* + delta H(x_1,.) (Appendix A.1.2); the value is
                                    -g*(p_1) + <p_N,x> + sum_{j<N} <p_j - p_{j+1}, x_j> - delta sum H.
                                    Built for H = CNORM with g = NORM or QUAD_SHIFT (control path) and
                                    for H = QUADROTOR with g = QUAD_SHIFT (persistent kernel; node 1's
                                    step is the family's p-prox with step sigma delta/(1 + sigma) at
                                    (v - sigma a)/(1 + sigma));
                                    for H = ISAACS it selects the game Hopf formulation (section 4.2
                                    eq. discgenlaxhopfdghopf, Algorithm 4): value -e*(p_1) - h_*(-q_1)
                                    + <p_N,x> - <q_N,y> + sum_{j<N} (<p_j - p_{j+1}, x_j>
                                    - <q_j - q_{j+1}, y_j>) - delta sum H(x_j, y_j, p_j, -q_j)
                                    (without the flag, Algorithm 3 for the same game).
                                    Other pairs return HJPD_EUNSUPPORTED.  Trajectory node 0 is zero. */
    HJPD_FORWARD_EULER = 1u << 6, /* forward-Euler discretisation of the Lax saddle (section 4.1, eq.
                                    disclaxFE) instead of backward Euler.  With p_j the costate of the
                                    interval (j-1, j), j = 1..N (eq. disclaxFE's p_{j-1}), the saddle is
                                    g(x_0) + sum_j <p_j, x_j - x_{j-1}> - delta sum_j H(x_{j-1}, p_j):
                                    H meets g at x_0, which takes a proximal-gradient step
                                    prox_{tau g}(x_0 + tau p_1 + tau delta grad_x H(x_0, p_1)) (section 5.3).
                                    Trajectories keep the layout of the backward-Euler path (p_0 = 0). */
    HJPD_TRAPEZOID = 1u << 7      /* trapezoidal rule: the average of the backward- and forward-Euler
                                    Hamiltonian sums (the remark after Algorithm 1), i.e.
                                    - delta sum_j (H(x_{j-1}, p_j) + H(x_j, p_j)) / 2, second-order in
                                    delta where both Euler rules are first-order.  HJPD_FORWARD_EULER and
                                    HJPD_TRAPEZOID are built for H = CNORM with g = NORM or QUAD_SHIFT and
                                    for H = QUADROTOR with g = QUAD_SHIFT (FP64: tiles of at most two nodes
                                    per lane), on the persistent control path (not with HJPD_PLAIN,
                                    HJPD_HOPF or the recipes: HJPD_EUNSUPPORTED); setting both is
                                    HJPD_EINVAL. */,
    HJPD_NO_REFILL = 1u << 8      /* persistent kernels without retire and refill: every lane group solves
                                    exactly one point and the launch has a group for every point, so a wave
                                    stays resident until its slowest point stops (the same kernels, layout and
                                    queue order; for measuring what refill buys).  Not with HJPD_PLAIN. */
};

typedef struct {
    int d;           /* state dimension (games: both players together) */
    int d_y;         /* > 0 selects the game path (Algorithm 3); evader block size */
    int H, g;        /* HJPD_H_*, HJPD_G_* */
    int dtype;       /* HJPD_F32 or HJPD_F64 */
    int N_max;       /* largest N of any point; sizes the trajectory outputs */
    double sigma;    /* dual step (sigma > 0) */
    double tau;      /* primal step (tau > 0, sigma tau <= 1/4 since ||D||_2 < 2) */
    double theta;    /* extrapolation, 0 <= theta <= 1 (theta = 1 in the paper) */
    double tol;      /* tolerance on the squared residuals (> 0) */
    int max_iter;    /* iteration cap (>= 1); with HJPD_FIXED_ITERS the exact count */
    uint64_t seed;   /* random start: counter-based SplitMix64 stream */
    unsigned flags;  /* HJPD_PLAIN | HJPD_FIXED_ITERS | HJPD_GRAPH | HJPD_TIMING | HJPD_NO_ORDER_HINT | HJPD_HOPF
                        | HJPD_FORWARD_EULER | HJPD_TRAPEZOID | HJPD_NO_REFILL */
    int lanes_per_point; /* persistent tile override: lanes per point (8,16,32,64), 0 = tuned/default */
    int nodes_per_lane;  /* persistent tile override: time nodes per lane (1..4), 0 = tuned/default */
    /* Robustness recipes (section 6, remarks on slow points); all zero = plain
     * Algorithm 1 (3).  Persistent kernels, tolerance mode, Lax formulation
     * only: the control families, and the pursuit-evasion game with one start
     * (section 6.2 applies the sigma and value-change recipes to a game); else
     * HJPD_EUNSUPPORTED.
     *  starts:    random starts per point (seed, seed+1, ...); the reported
     *             point is the lowest value among the starts that met a
     *             stopping rule, else the lowest finite value, ties to the
     *             earlier start (0 or 1 = one start; control path only);
     *  restarts:  times the iteration may continue past the cap max_iter with
     *             sigma raised by sigma_inc and tau = sigma0 tau0 / sigma
     *             (sigma_inc = 0: continue with the same steps);
     *  value_tol: after the first cap, also stop (HJPD_PT_VALUE_STALLED) when
     *             the value changes by at most value_tol max(|value|, 1)
     *             between consecutive iterations (0 = off).
     * iters reports the chosen start's iterations over all its phases. */
    int starts;
    int restarts;
    double sigma_inc;
    double value_tol;
} hjpd_desc;

/*
 * Create a context for one problem (families, dimension, dtype, steps).
 * Validates the descriptor (EINVAL: d < 1, d_y < 0 or d_y >= d, sigma <= 0,
 * tau <= 0, sigma*tau > 1/4, theta outside [0,1], tol <= 0, max_iter < 1,
 * N_max < 1, unknown family or dtype, tile override out of range; EUNSUPPORTED:
 * family pair, dimension or N_max not built), selects a GPU kernel set, and
 * allocates the context's device workspace on the current device.
 * *out receives the context (NULL on failure).
 */
int hjpd_create(const hjpd_desc *desc, hjpd_ctx **out);

/*
 * Solve n independent points (Algorithm 1 / Algorithm 3 at every point).
 * x, t, N, h_params, g_params, phi, iters, status are required (non-NULL
 * when n > 0); x_traj and p_traj may be NULL.  n == 0 is a no-op.
 * The random start of point i (section 6 set-up) depends only on (seed, i,
 * array, node, coordinate), so results do not depend on batching or on the
 * kernel chosen, up to floating-point rounding order.
 * EINVAL: n < 0, a required pointer NULL.  Per-point input problems are
 * reported as HJPD_PT_BADINPUT (phi = NaN, iters = 0), not as return codes.
 */
int hjpd_solve_batch(hjpd_ctx *ctx, int64_t n, const void *x, const void *t, const int32_t *N,
                     const void *h_params, const void *g_params, void *phi, void *x_traj, void *p_traj,
                     int32_t *iters, int32_t *status, void *stream);

/*
 * hjpd_solve_batch without any allocation, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, kernels and results as
 * hjpd_solve_batch (bitwise: each point is solved on its own), for contexts
 * of the persistent kernels (not HJPD_PLAIN, not HJPD_H_LINEAR_TANH:
 * HJPD_EUNSUPPORTED).  Differences:
 *  - the work queue and its counters live in a static device array of the
 *    library, one copy per GPU (4.03 MiB, held until the process ends),
 *    instead of the context's workspace, so n is limited to 1,048,576 points
 *    (HJPD_EINVAL above);
 *  - the call never allocates or frees memory (device or host) and never
 *    builds a graph: with HJPD_GRAPH set it still enqueues the kernels
 *    directly on `stream`, so the caller may capture them into a graph of
 *    its own;
 *  - every call on a GPU shares that GPU's array: calls on one GPU whose
 *    work overlaps in time (from any context or thread, on different
 *    streams) race and give wrong results; serialise them (one stream, or
 *    events).  Each call clears what it needs before use.
 * The context's current device must be the current device (HJPD_EINVAL).
 */
int hjpd_solve_batch_noalloc(hjpd_ctx *ctx, int64_t n, const void *x, const void *t, const int32_t *N,
                             const void *h_params, const void *g_params, void *phi, void *x_traj, void *p_traj,
                             int32_t *iters, int32_t *status, void *stream);

/*
 * Value and reverse-mode gradients for HJPD_H_LINEAR_TANH with
 * HJPD_G_QUAD_FORM (float32): phi after exactly K_iters iterations
 * (fixed-iteration Algorithm 1), and, for upstream weights grad_phi [n],
 *   dphi_dx   [n][d]  = grad_phi[i] * d phi_i / d x_i
 *   dh_params [1+d*d] = sum_i grad_phi[i] * d phi_i / d (eps, A)
 *   dg_params [d*d]   = sum_i grad_phi[i] * d phi_i / d Q
 * by differentiating through the K_iters unrolled iterations, with the
 * forward iterate stored every ckpt_every iterations and each segment
 * recomputed during the reverse sweep.  dh_params / dg_params are
 * overwritten (not accumulated).  EINVAL: K_iters < 1, ckpt_every < 1,
 * required pointer NULL; EUNSUPPORTED: other families or float64.
 */
int hjpd_value_grad(hjpd_ctx *ctx, int64_t n, const void *x, const void *t, const int32_t *N,
                    const void *h_params, const void *g_params, const void *grad_phi, int K_iters,
                    int ckpt_every, void *phi, void *dphi_dx, void *dh_params, void *dg_params,
                    void *stream);

/*
 * Tune the persistent path on this batch: the capacity classes (which ranges
 * of N share one launch) and each class's tile, i.e. lanes per point L
 * (64/L points per wavefront) and nodes per lane K (the unroll of each lane's
 * loop over its time nodes), with L*K covering the class's largest N.  It
 * starts from a class boundary at every compiled capacity (8, 16, 24, 32, 48,
 * 64, 96, 128, 192, 256), picks each class's fastest tile among those of
 * capacity up to twice its top, then merges neighbouring classes while a
 * merge is at least 1 % faster.  Each candidate is timed as a whole solve of
 * exactly `probe_iters` iterations per point (default 200 if <= 0).  The
 * chosen plan is installed in the context and, when $HJPD_TUNE_CACHE names a
 * file, appended to it; hjpd_create reads that file and starts from the last
 * plan recorded for the same problem (family, g, d, d_y, dtype, N_max, kernel
 * variant, gfx950).  Synchronises `stream`.  Arguments as for
 * hjpd_solve_batch; phi, iters and status are scratch here.  EINVAL if the
 * descriptor fixes the tile; EUNSUPPORTED for HJPD_PLAIN or linear-tanh.
 */
int hjpd_autotune(hjpd_ctx *ctx, int64_t n, const void *x, const void *t, const int32_t *N,
                  const void *h_params, const void *g_params, void *phi, int32_t *iters, int32_t *status,
                  int probe_iters, void *stream);

/*
 * Queue-integrity hook: with a non-NULL `counts` (caller-owned device int32
 * array of at least n entries for the solves that follow, zeroed by the
 * caller), every pop of point i from the work queue adds 1 to counts[i]; a
 * correct queue pops every valid point exactly once and no bad-input point.
 * NULL turns counting off.  Persistent kernels only (EUNSUPPORTED otherwise).
 * Drops a captured graph.
 */
int hjpd_set_pop_counter(hjpd_ctx *ctx, int32_t *counts);

/*
 * Set the persistent path's capacity classes explicitly: class c serves the
 * points with hi[c-1] < N <= hi[c] (hi[-1] = 0) with the tile (L[c], K[c]).
 * hi ascending, the last one >= N_max (it is clamped to N_max), L[c]*K[c] >=
 * min(hi[c], N_max), 1..16 classes, tiles among the compiled ones (L in {8,
 * 16, 32, 64}, K in 1..4; capacities 8, 16, 24, 32, 48, 64, 96, 128, 192,
 * 256).  EINVAL / EUNSUPPORTED otherwise, with the previous plan kept.
 * A point's result depends on the tile that serves it (its lanes and nodes
 * per lane fix the summation order of its residuals, so a stop decision can
 * differ in the last bit) but not on the class boundaries, the other points
 * or the queue order.
 */
int hjpd_set_plan(hjpd_ctx *ctx, int n_classes, const int32_t *hi, const int32_t *L, const int32_t *K);

/*
 * The current plan: *n_classes classes, the first max_classes of them written
 * to hi, L, K (any may be NULL); *from_cache (may be NULL) is 1 when the plan
 * came from the tuning cache at hjpd_create.
 */
int hjpd_get_plan(hjpd_ctx *ctx, int max_classes, int32_t *hi, int32_t *L, int32_t *K, int *n_classes,
                  int *from_cache);

/*
 * With HJPD_TIMING: device milliseconds of the main solve kernel(s) of the
 * last completed hjpd_solve_batch (from the first launch's start to the
 * last one's end), measured with HIP events on the call's stream, or of the
 * reverse-sweep kernel of the last hjpd_value_grad; *launches receives the
 * number of those kernel launches.  Synchronises on those events.  EINVAL if timing is off or no
 * solve has run.
 */
int hjpd_get_timing(hjpd_ctx *ctx, double *ms, int *launches);

/*
 * With HJPD_TIMING, after an eager solve on the persistent kernels (not
 * HJPD_PLAIN, not HJPD_GRAPH, not HJPD_H_LINEAR_TANH): device milliseconds of
 * launch i (0 <= i < the launch count hjpd_get_timing reports) of the last
 * completed solve, measured with HIP events on the stream that launch ran on
 * (each capacity class is one persistent launch, section 7's per-point
 * independence lets the classes run side by side), and the launch's class:
 * the N range [*N_lo, *N_hi] it served and its tile (lanes per point, nodes
 * per lane).  Output pointers other than ms may be NULL.  Synchronises on
 * the launch's end event.  EINVAL if timing is off, no such solve has run,
 * or i is out of range.
 */
int hjpd_get_launch_timing(hjpd_ctx *ctx, int i, double *ms, int *N_lo, int *N_hi, int *lanes_per_point,
                           int *nodes_per_lane);

/*
 * Calibration of the FLOP accounting (no context; runs on the current
 * device): a kernel whose every lane runs `chains` independent chains of
 * fused multiply-adds a <- a b + c (chains in {1, 2, 4, 8, 16}), 32 per chain
 * and round, for `rounds` rounds (1 .. 2^30), in FP32 (single, not packed,
 * FMAs, as in every kernel of this library) or FP64 (dtype HJPD_F32 or
 * HJPD_F64), with `waves_per_simd` (1..8) blocks of four waves per compute
 * unit.  One warm-up launch, then one launch timed with HIP events on a
 * stream of its own: *ms receives its device milliseconds, *flops (if not
 * NULL) its exact flop count (2 per lane and FMA) and *wave_instructions (if
 * not NULL) its count of wave64 FMA instructions.  Allocates and frees a
 * small output buffer; synchronous.  EINVAL on a bad argument, EDEVICE on a
 * HIP error.
 */
int hjpd_calibrate_fma(int dtype, int chains, int waves_per_simd, int64_t rounds, double *ms, double *flops,
                       double *wave_instructions);

/* Release the context and its device workspace.  NULL is allowed. */
int hjpd_destroy(hjpd_ctx *ctx);

/* Message for the last non-OK return on this thread ("" if none). */
const char *hjpd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HJPD_H */
