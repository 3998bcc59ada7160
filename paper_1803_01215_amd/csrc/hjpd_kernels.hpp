// PDHG kernels for the per-point Lax saddle problem (section 5.1, Algorithm 1;
// games: Algorithm 3), run independently at every query point.
//
// Persistent lane-group kernel
//   A query point is owned by a group of L consecutive lanes of a wave64;
//   lane l holds time nodes j = l*K + 1 .. l*K + K (x_j, p_j, z_j in VGPRs),
//   lane 0 also holds node 0 (x_0, z_0; p_0 = 0).  Per iteration:
//     dual step   p_j <- prox_{sigma delta H(x_j,.)}(p_j + sigma (z_j - z_{j-1})), j = 1..N
//     node 0      x_0 <- prox_{tau g}(x_0 + tau p_1)
//     primal step x_j <- x_j - tau (p_j - p_{j+1}) + tau delta grad_x H(x_j, p_j), j = 1..N-1
//     extrapolate z = x_new + theta (x_new - x_old)
//     residuals   ||x^{k+1}-x^k||^2, ||p^{k+1}-p^k||^2 summed over the group.
//   z_{j-1} and p_{j+1} cross a lane boundary once per lane per iteration
//   (DPP wavefront shifts).  The eikonal family uses the same scheme with the
//   node layout shifted by one, so that node 0 is an ordinary slot
//   (k_group_control_shift).  Groups pop point ids from a device queue
//   (sorted by N, one segment per tile class); a group whose point meets the
//   stopping rule writes its outputs and immediately pops the next point
//   (retire and refill), so waves stay full until the queue drains.
//
// Plain kernel
//   One point per lane, the whole stacked state of the point in a global
//   workspace laid out [node][coord][lane] (coalesced across lanes), one
//   fused sweep over the nodes per iteration; a wave runs until all its
//   lanes have stopped (no refill).  This is the straightforward mapping of
//   the paper's per-point loop and serves as the baseline.
#pragma once

#include "hjpd_families.hpp"

namespace hjpd {

// Occupancy target of a persistent FP32 tile (waves per SIMD, the second
// __launch_bounds__ argument): the register state grows with K, so one node
// per lane keeps 4 waves, two keep 3, more keep 2.  FP64 state takes twice
// the registers; it is left to the compiler (1 = no constraint).
template <typename T, int K>
inline constexpr int kGroupWaves = sizeof(T) == 8 ? 1 : (K == 1 ? 4 : (K == 2 ? 3 : 2));

// The same per family: a family lists its FP32 waves per SIMD by K (its state
// and per-node cache decide how many registers a node takes), so that no
// tile spills registers to memory inside the iteration.
template <typename T, class F, int K>
inline constexpr int kFamWaves = sizeof(T) == 8 ? 1 : F::kWavesK[K];

// The shifted-layout kernel in FP64 with at most two nodes per lane is held
// to two waves per SIMD (256 VGPRs, a few spilled to scratch): unconstrained
// it takes 284 registers and one wave per SIMD, and the second wave hides more
// than the spills cost (cnorm10, 16x2: 17.1 -> 13.5 ms).
template <typename T, int K>
inline constexpr int kShiftWaves = (sizeof(T) == 8 && K <= 2) ? 2 : kGroupWaves<T, K>;

// Issue priority of a wave (s_setprio) from the iteration count of the
// oldest point it holds.  A point still iterating after a tenth, a fifth and
// two fifths of the iteration cap is in the slow tail of the batch: the few
// slowest points run their iterations one after another and end the
// persistent launch, so the SIMD arbiter is told to prefer their waves over
// waves of faster points from early on (levels 1, 2, 3).  Order of issue
// only; results are unchanged.
struct WavePrio {
  int t1, t2, t3;
  __device__ explicit WavePrio(int max_iter) {
    t1 = max_iter / 10 > 1 ? max_iter / 10 : 1;
    t2 = max_iter / 5 > t1 ? max_iter / 5 : t1 + 1;
    t3 = 2 * (max_iter / 5) > t2 ? 2 * (max_iter / 5) : t2 + 1;
  }
  __device__ bool step(int k) const { return k == t1 || k == t2 || k == t3; }
};
__device__ __forceinline__ void set_wave_priority(bool active, int k, const WavePrio& pr) {
  if (__any(active && k >= pr.t3)) __builtin_amdgcn_s_setprio(3);
  else if (__any(active && k >= pr.t2)) __builtin_amdgcn_s_setprio(2);
  else if (__any(active && k >= pr.t1)) __builtin_amdgcn_s_setprio(1);
  else __builtin_amdgcn_s_setprio(0);
}

template <typename T>
struct KArgs {
  const T* x;            // [n][d]
  const T* t;            // [n]
  const int32_t* N;      // [n]
  const T* hp;
  const T* gp;
  T* phi;                // [n]
  T* xtraj;              // [n][N_max+1][d] or null
  T* ptraj;
  int32_t* iters;
  int32_t* status;
  const int32_t* queue;      // point ids sorted by N (descending)
  const int32_t* cls_range;  // [2 * n_cls] begin/end of each class segment
  int32_t* heads;            // per-class pop counters (zeroed by the queue builder)
  T* work;                   // plain kernel workspace
  int64_t work_stride;       // lanes in the plain workspace
  int cls;
  T sigma, tau, theta, tol;
  int max_iter, fixed, N_max, d, gkind;
  int hopf;                  // 1: Hopf formulation (Algorithm 2), no node 0
  T wl, wr;                  // Hamiltonian weights at an interval's left / right node (weighted kernel only)
  uint64_t seed;
  int refill;                // 1: a group that finishes a point pops the next (retire and refill)
  int32_t* pops;             // optional [n] pop count per point id (queue integrity checks)
  // robustness recipes (kernels compiled with them only)
  int starts, restarts;
  T sigma_inc, value_tol;
};

template <typename T, int D>
__device__ __forceinline__ bool all_finite(const T (&v)[D]) {
  bool ok = true;
#pragma unroll
  for (int i = 0; i < D; i++) ok = ok && M<T>::finite(v[i]);
  return ok;
}

template <typename T>
__device__ __forceinline__ T init_x(T xt, uint64_t seed, int64_t pt, int arr, int j, int i) {
  return T(double(xt) + start_noise(seed, uint64_t(pt), arr, j, i));
}

// The per-node side data of the weighted discretisations (a placeholder for
// kernels compiled without them).
template <class F, typename T, bool W> struct SideOf { using type = int; };
template <class F, typename T> struct SideOf<F, T, true> { using type = typename F::template Side<T>; };

// ---------------------------------------------------------------------------
// Persistent lane-group kernel, optimal-control path (Algorithm 1), for the
// families whose dual step needs the whole neighbouring state (quadrotor).
// The eikonal family runs k_group_control_shift below.  kW: the weighted
// discretisations (forward Euler, trapezoid; KArgs::wl, wr), where interval
// j's dual step takes the Hamiltonians of x_{j-1} and x_j, x_j's gradient
// collects both intervals it bounds, and x_0 takes a proximal-gradient step.
// ---------------------------------------------------------------------------
template <typename T, class F, int L, int K, bool kW = false>
__global__ void __launch_bounds__(256, (kFamWaves<T, F, K>)) k_group_control(KArgs<T> a) {
  constexpr int D = F::D;
  const int lane = threadIdx.x & 63;
  const int l = lane & (L - 1);
  const int leader = lane - l;

  typename F::template Par<T> P;
  F::load(P, a.hp, a.gp, a.gkind, a.tau);
  const WavePrio prio(a.max_iter);
  const int beg = a.cls_range[2 * a.cls], end = a.cls_range[2 * a.cls + 1];
  int32_t* head = a.heads + a.cls;
  const T sigma = a.sigma, tau = a.tau, theta = a.theta;
  // Hopf formulation (Algorithm 2): no node 0 (x_0 = z_0 = 0, the Hopf
  // difference operator), node 1's dual step is the joint prox with g*, and
  // the value has -g*(p_1) in place of g(x_0).  A uniform switch.
  const bool hopf = F::kHopfGroup && a.hopf;
  const T wl = a.wl, wr = a.wr;  // kW: H weights at an interval's left / right node

  T x[K][D], p[K][D], z[K][D], x0[D], z0[D];
  T tj[K], tdj[K];  // per node: tau and tau*delta where the node takes a primal step, else 0
  T delta = T(0), sd = T(0), td = T(0);
  int Np = 0, k = 0;
  int64_t pt = -1;
  bool active = false;

  auto pop_and_init = [&]() {
    int idx = 0;
    // without refill a group serves the one point it popped first
    if (l == 0) idx = (a.refill || pt < 0) ? atomicAdd(head, 1) : (end - beg);
    idx = __shfl(idx, leader, 64);
    const int qi = beg + idx;
    active = qi < end;
    if (!active) return;
    pt = a.queue[qi];
    if (a.pops && l == 0) atomicAdd(a.pops + pt, 1);
    Np = a.N[pt];
    delta = a.t[pt] / T(Np);
    sd = sigma * delta;
    td = tau * delta;
    k = 0;
    T xt[D];
#pragma unroll
    for (int i = 0; i < D; i++) xt[i] = a.x[pt * a.d + i];
#pragma unroll
    for (int kk = 0; kk < K; kk++) {
      const int j = 1 + l * K + kk;
#pragma unroll
      for (int i = 0; i < D; i++) {
        x[kk][i] = (j < Np) ? init_x(xt[i], a.seed, pt, kArrX, j, i) : xt[i];
        p[kk][i] = (j <= Np) ? T(start_noise(a.seed, uint64_t(pt), kArrP, j, i)) : T(0);
        z[kk][i] = x[kk][i];
      }
    }
    // node 0 lives in the group's first lane; the other lanes keep x0 = z0 = 0
#pragma unroll
    for (int i = 0; i < D; i++) {
      x0[i] = (l == 0 && !hopf) ? init_x(xt[i], a.seed, pt, kArrX, 0, i) : T(0);
      z0[i] = x0[i];
    }
#pragma unroll
    for (int kk = 0; kk < K; kk++) {
      const int j = 1 + l * K + kk;
      tj[kk] = (j < Np) ? tau : T(0);
      tdj[kk] = (j < Np) ? td : T(0);
    }
  };

  pop_and_init();

  while (__any(active)) {
    // ---- dual step -------------------------------------------------------
    // z_{j-1} of the lane's first node: the previous lane's last node, or
    // z_0 in the group's first lane (z0 is zero in every other lane; the
    // Hopf difference operator has z_0 = 0).
    T zprev[D];
#pragma unroll
    for (int i = 0; i < D; i++) zprev[i] = group_prev_fill<L>(z[K - 1][i], l, z0[i]);
    typename F::template Cache<T> C[K];
    T rp = T(0), rx = T(0);
    // kW: every node's geometry first, then the side data of the node before
    // the lane's first (the previous lane's last node, or node 0 in the
    // group's first lane)
    typename SideOf<F, T, kW>::type Sp;
    if constexpr (kW) {
#pragma unroll
      for (int kk = 0; kk < K; kk++) F::geometry(P, x[kk], C[kk]);
      typename F::template Cache<T> C0;
      F::geometry(P, x0, C0);
      typename F::template Side<T> S0, Sl;
      F::side(x0, C0, S0);
      F::side(x[K - 1], C[K - 1], Sl);
      const T m0 = (l == 0) ? T(1) : T(0);  // fill is node 0's data in the first lane, 0 elsewhere
#pragma unroll
      for (int i = 0; i < 3; i++) {
        Sp.v[i] = group_prev_fill<L>(Sl.v[i], l, m0 * S0.v[i]);
        Sp.Ww[i] = group_prev_fill<L>(Sl.Ww[i], l, m0 * S0.Ww[i]);
        Sp.b[i] = group_prev_fill<L>(Sl.b[i], l, m0 * S0.b[i]);
      }
    }
    // Order of the lane's steps.  FP32 with four nodes per lane (Lax form):
    // dual(0), node 0, dual(1), primal(0), dual(2), primal(1), ...,
    // primal(K-1).  A node's primal step needs its own cache and the next
    // node's new dual, and must follow the next node's dual step (which reads
    // its old z), so this order keeps at most two nodes' caches live instead
    // of K: on the quadrotor the 16x4 tile spills 79 registers instead of 103
    // and runs 12 % faster.  Otherwise every dual step, node 0, then every
    // primal step (the 16x3 tile compiled from the interleaved form spills
    // less but ran 4-7 % slower; the weighted rules compute every cache
    // first anyway; FP64 keeps its measured code).  Both orders do the same
    // operations in the same order of the residual sums.
    if constexpr (K >= 4 && sizeof(T) == 4 && !kW) {
      T pnext[D];
#pragma unroll
      for (int kk = 0; kk <= K; kk++) {
        const int n = kk - 1;  // the primal step that follows dual(kk)
        if (kk < K) {
          // ---- dual step of node kk ------------------------------------------
          T v[D];
#pragma unroll
          for (int i = 0; i < D; i++) v[i] = p[kk][i] + sigma * (z[kk][i] - (kk == 0 ? zprev[i] : z[kk - 1][i]));
          T lam = sd;
          if constexpr (F::kHopfGroup) {
            if (kk == 0 && hopf) F::hopf1_in(P, v, lam, sigma, l == 0);  // node 1: with g*
          }
          if constexpr (kW) {
            typename F::template Side<T> Sa, Sb;
            if (kk == 0) Sa = Sp;
            else F::side(x[kk - 1], C[kk - 1], Sa);
            F::side(x[kk], C[kk], Sb);
            F::dual_w(P, Sa, Sb, v, lam, wl, wr);
          } else {
            F::dual(P, x[kk], v, lam, C[kk]);
          }
          if constexpr (!F::kZeroSafe) {
            // nodes past N keep p = 0
            const int j = 1 + l * K + kk;
#pragma unroll
            for (int i = 0; i < D; i++) v[i] = (j <= Np) ? v[i] : T(0);
          }
#pragma unroll
          for (int i = 0; i < D; i++) {
            const T dp = v[i] - p[kk][i];
            rp += dp * dp;
            p[kk][i] = v[i];
          }
        }
        if (kk == 0) {
          // ---- node 0 (after every lane's first dual step) -------------------
#pragma unroll
          for (int i = 0; i < D; i++) pnext[i] = group_next0<L>(p[0][i], l);
          if (l == 0 && !hopf) {
            T dx0[D];
            if constexpr (kW) {
              // proximal-gradient step: prox_{tau g}(x_0 + tau (p_1 + delta wl grad_x H(x_0, p_1)))
              typename F::template Cache<T> C0;
              F::geometry(P, x0, C0);
              T g0[D], p1[D];
              F::grad_w(P, x0, p[0], p[0], T(0), T(1), C0, g0);
#pragma unroll
              for (int i = 0; i < D; i++) p1[i] = p[0][i] + delta * wl * g0[i];
              F::step0(P, x0, p1, tau, dx0);
            } else {
              F::step0(P, x0, p[0], tau, dx0);
            }
#pragma unroll
            for (int i = 0; i < D; i++) {
              rx += dx0[i] * dx0[i];
              z0[i] = x0[i] + (T(1) + theta) * dx0[i];
              x0[i] += dx0[i];
            }
          }
        }
        if (n >= 0 && n < K) {
          // ---- primal step of node n -------------------------------------------
          // Nodes j >= N take no step: their tau and tau*delta are 0 (x_N = x
          // stays fixed, and past N nothing moves).
          T g[D];
          if constexpr (kW) {
            T pn[D];
#pragma unroll
            for (int i = 0; i < D; i++) pn[i] = (n == K - 1) ? pnext[i] : p[n + 1][i];
            F::grad_w(P, x[n], p[n], pn, wl, wr, C[n], g);
          } else {
            F::grad(P, x[n], p[n], C[n], g);
          }
#pragma unroll
          for (int i = 0; i < D; i++) {
            const T pp = (n == K - 1) ? pnext[i] : p[n + 1][i];
            const T dx = tdj[n] * g[i] - tj[n] * (p[n][i] - pp);
            rx += dx * dx;
            z[n][i] = x[n][i] + (T(1) + theta) * dx;
            x[n][i] += dx;
          }
        }
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < K; kk++) {
        T v[D];
#pragma unroll
        for (int i = 0; i < D; i++) v[i] = p[kk][i] + sigma * (z[kk][i] - (kk == 0 ? zprev[i] : z[kk - 1][i]));
        T lam = sd;
        if constexpr (F::kHopfGroup) {
          if (kk == 0 && hopf) F::hopf1_in(P, v, lam, sigma, l == 0);  // node 1: with g*
        }
        if constexpr (kW) {
          typename F::template Side<T> Sa, Sb;
          if (kk == 0) Sa = Sp;
          else F::side(x[kk - 1], C[kk - 1], Sa);
          F::side(x[kk], C[kk], Sb);
          F::dual_w(P, Sa, Sb, v, lam, wl, wr);
        } else {
          F::dual(P, x[kk], v, lam, C[kk]);
        }
        if constexpr (!F::kZeroSafe) {
          // nodes past N keep p = 0
          const int j = 1 + l * K + kk;
#pragma unroll
          for (int i = 0; i < D; i++) v[i] = (j <= Np) ? v[i] : T(0);
        }
#pragma unroll
        for (int i = 0; i < D; i++) {
          const T dp = v[i] - p[kk][i];
          rp += dp * dp;
          p[kk][i] = v[i];
        }
      }
      // ---- node 0 -----------------------------------------------------------
      T pnext[D];
#pragma unroll
      for (int i = 0; i < D; i++) pnext[i] = group_next0<L>(p[0][i], l);
      if (l == 0 && !hopf) {
        T dx0[D];
        if constexpr (kW) {
          // proximal-gradient step: prox_{tau g}(x_0 + tau (p_1 + delta wl grad_x H(x_0, p_1)))
          typename F::template Cache<T> C0;
          F::geometry(P, x0, C0);
          T g0[D], p1[D];
          F::grad_w(P, x0, p[0], p[0], T(0), T(1), C0, g0);
#pragma unroll
          for (int i = 0; i < D; i++) p1[i] = p[0][i] + delta * wl * g0[i];
          F::step0(P, x0, p1, tau, dx0);
        } else {
          F::step0(P, x0, p[0], tau, dx0);
        }
#pragma unroll
        for (int i = 0; i < D; i++) {
          rx += dx0[i] * dx0[i];
          z0[i] = x0[i] + (T(1) + theta) * dx0[i];
          x0[i] += dx0[i];
        }
      }
      // ---- primal step --------------------------------------------------------
      // Nodes j >= N take no step: their tau and tau*delta are 0 (x_N = x stays
      // fixed, and past N nothing moves).
#pragma unroll
      for (int kk = 0; kk < K; kk++) {
        T g[D];
        if constexpr (kW) {
          T pn[D];
#pragma unroll
          for (int i = 0; i < D; i++) pn[i] = (kk == K - 1) ? pnext[i] : p[kk + 1][i];
          F::grad_w(P, x[kk], p[kk], pn, wl, wr, C[kk], g);
        } else {
          F::grad(P, x[kk], p[kk], C[kk], g);
        }
#pragma unroll
        for (int i = 0; i < D; i++) {
          const T pp = (kk == K - 1) ? pnext[i] : p[kk + 1][i];
          const T dx = tdj[kk] * g[i] - tj[kk] * (p[kk][i] - pp);
          rx += dx * dx;
          z[kk][i] = x[kk][i] + (T(1) + theta) * dx;
          x[kk][i] += dx;
        }
      }
    }
    // ---- stopping rule (section 6 set-up) ------------------------------------
    k++;
    const T rxs = group_sum<L>(rx), rps = group_sum<L>(rp);
    const bool fin = M<T>::finite(rxs + rps);
    const bool small = (rxs < a.tol) && (rps < a.tol);
    const bool done = active && (!fin || (!a.fixed && small) || k >= a.max_iter);
    if (done) {
      // value: Lagrangian at the last iterate (Algorithm 1)
      T xprev[D];
#pragma unroll
      for (int i = 0; i < D; i++) xprev[i] = group_prev_fill<L>(x[K - 1][i], l, x0[i]);
      T acc = T(0);
      int bad = 0;
#pragma unroll
      for (int kk = 0; kk < K; kk++) {
        const int j = 1 + l * K + kk;
        if (j <= Np) {
          T s = T(0);
#pragma unroll
          for (int i = 0; i < D; i++) s += p[kk][i] * (x[kk][i] - (kk == 0 ? xprev[i] : x[kk - 1][i]));
          if constexpr (kW) {
            T xl[D];
#pragma unroll
            for (int i = 0; i < D; i++) xl[i] = (kk == 0) ? xprev[i] : x[kk - 1][i];
            acc += s - delta * (wl * F::H(P, xl, p[kk]) + wr * F::H(P, x[kk], p[kk]));
          } else {
            acc += s - delta * F::H(P, x[kk], p[kk]);
          }
          bad |= !(all_finite<T, D>(x[kk]) && all_finite<T, D>(p[kk]));
        }
      }
      if (l == 0) {
        if constexpr (F::kHopfGroup) {
          acc += hopf ? -F::gstar(P, p[0]) : F::g(P, x0);
        } else {
          acc += F::g(P, x0);
        }
        bad |= !all_finite<T, D>(x0);
      }
      acc = group_sum<L>(acc);
      bad = group_or<L>(bad);
      int st = !fin ? kNonFinite : (small ? kConverged : kMaxIter);
      if (bad || !M<T>::finite(acc)) st = kNonFinite;
      if (l == 0) {
        a.phi[pt] = acc;
        a.iters[pt] = k;
        a.status[pt] = st;
      }
      const int64_t base = pt * int64_t(a.N_max + 1) * a.d;
      if (a.xtraj) {
#pragma unroll
        for (int kk = 0; kk < K; kk++) {
          const int j = 1 + l * K + kk;
          if (j <= Np)
#pragma unroll
            for (int i = 0; i < D; i++) a.xtraj[base + j * D + i] = x[kk][i];
        }
        if (l == 0)
#pragma unroll
          for (int i = 0; i < D; i++) a.xtraj[base + i] = x0[i];
      }
      if (a.ptraj) {
#pragma unroll
        for (int kk = 0; kk < K; kk++) {
          const int j = 1 + l * K + kk;
          if (j <= Np)
#pragma unroll
            for (int i = 0; i < D; i++) a.ptraj[base + j * D + i] = p[kk][i];
        }
        if (l == 0)
#pragma unroll
          for (int i = 0; i < D; i++) a.ptraj[base + i] = T(0);
      }
      pop_and_init();
    }
    if (__any(done || (active && prio.step(k)))) set_wave_priority(active, k, prio);
  }
}

// ---------------------------------------------------------------------------
// Persistent lane-group kernel with the robustness recipes of section 6
// (several random starts, sigma raised at the iteration cap, value-change
// stop after the first cap), control path.  A separate kernel: the recipe
// state and the per-point step sizes would otherwise cost the plain kernel
// registers.  Launched with kRec = true; kRec = false reduces it to the plain
// iteration (the same arithmetic as k_group_control).
// ---------------------------------------------------------------------------
template <typename T, class F, int L, int K, bool kRec = true>
__global__ void __launch_bounds__(256, (kFamWaves<T, F, K>)) k_group_control_rec(KArgs<T> a) {
  constexpr int D = F::D;
  const int lane = threadIdx.x & 63;
  const int l = lane & (L - 1);
  const int leader = lane - l;

  typename F::template Par<T> P;
  F::load(P, a.hp, a.gp, a.gkind, a.tau);
  const WavePrio prio(a.max_iter);
  const int beg = a.cls_range[2 * a.cls], end = a.cls_range[2 * a.cls + 1];
  int32_t* head = a.heads + a.cls;
  const T theta = a.theta;
  // step sizes: kernel constants, or per point when the recipes may raise sigma
  T sigma = a.sigma, tau = a.tau;

  T x[K][D], p[K][D], z[K][D], x0[D], z0[D];
  T tj[K], tdj[K];  // per node: tau and tau*delta where the node takes a primal step, else 0
  T delta = T(0), sd = T(0), td = T(0);
  int Np = 0, k = 0;
  int64_t pt = -1;
  bool active = false;
  // recipe state (dead code without kRec)
  int start = 0, phase = 0, kp = 0, best_rank = 3;
  T prev_val = T(0), best_phi = T(0);
  bool have_prev = false;

  auto set_steps = [&]() __attribute__((always_inline)) {
    sd = sigma * delta;
    td = tau * delta;
#pragma unroll
    for (int kk = 0; kk < K; kk++) {
      const int j = 1 + l * K + kk;
      tj[kk] = (j < Np) ? tau : T(0);
      tdj[kk] = (j < Np) ? td : T(0);
    }
    if constexpr (kRec) F::set_tau(P, tau, a.gkind);
  };

  // random start number `s` of the current point (seed + s; s = 0 without recipes)
  auto init_start = [&](int s) __attribute__((always_inline)) {
    const uint64_t seed = a.seed + uint64_t(s);
    k = 0;
    if constexpr (kRec) {
      start = s;
      phase = 0;
      kp = 0;
      have_prev = false;
      sigma = a.sigma;
      tau = a.tau;
    }
    T xt[D];
#pragma unroll
    for (int i = 0; i < D; i++) xt[i] = a.x[pt * a.d + i];
#pragma unroll
    for (int kk = 0; kk < K; kk++) {
      const int j = 1 + l * K + kk;
#pragma unroll
      for (int i = 0; i < D; i++) {
        x[kk][i] = (j < Np) ? init_x(xt[i], seed, pt, kArrX, j, i) : xt[i];
        p[kk][i] = (j <= Np) ? T(start_noise(seed, uint64_t(pt), kArrP, j, i)) : T(0);
        z[kk][i] = x[kk][i];
      }
    }
    // node 0 lives in the group's first lane; the other lanes keep x0 = z0 = 0
#pragma unroll
    for (int i = 0; i < D; i++) {
      x0[i] = (l == 0) ? init_x(xt[i], seed, pt, kArrX, 0, i) : T(0);
      z0[i] = x0[i];
    }
    set_steps();
  };

  auto pop_and_init = [&]() __attribute__((always_inline)) {
    int idx = 0;
    // without refill a group serves the one point it popped first
    if (l == 0) idx = (a.refill || pt < 0) ? atomicAdd(head, 1) : (end - beg);
    idx = __shfl(idx, leader, 64);
    const int qi = beg + idx;
    active = qi < end;
    if (!active) return;
    pt = a.queue[qi];
    if (a.pops && l == 0) atomicAdd(a.pops + pt, 1);
    Np = a.N[pt];
    delta = a.t[pt] / T(Np);
    if constexpr (kRec) best_rank = 3;
    init_start(0);
  };

  // The value: the Lagrangian at the current iterate (Algorithm 1 fval; Hopf:
  // Algorithm 2 fval), summed over the group; `bad` flags a non-finite entry.
  auto lagrangian = [&](int& bad) __attribute__((always_inline)) {
    T xprev[D];
#pragma unroll
    for (int i = 0; i < D; i++) xprev[i] = group_prev_fill<L>(x[K - 1][i], l, x0[i]);
    T acc = T(0);
    bad = 0;
#pragma unroll
    for (int kk = 0; kk < K; kk++) {
      const int j = 1 + l * K + kk;
      if (j <= Np) {
        T s = T(0);
#pragma unroll
        for (int i = 0; i < D; i++) s += p[kk][i] * (x[kk][i] - (kk == 0 ? xprev[i] : x[kk - 1][i]));
        acc += s - delta * F::H(P, x[kk], p[kk]);
        bad |= !(all_finite<T, D>(x[kk]) && all_finite<T, D>(p[kk]));
      }
    }
    if (l == 0) {
      acc += F::g(P, x0);
      bad |= !all_finite<T, D>(x0);
    }
    bad = group_or<L>(bad);
    return group_sum<L>(acc);
  };

  pop_and_init();

  while (__any(active)) {
    // ---- dual step -------------------------------------------------------
    // z_{j-1} of the lane's first node: the previous lane's last node, or
    // z_0 in the group's first lane (z0 is zero in every other lane; the
    // Hopf difference operator has z_0 = 0).
    T zprev[D];
#pragma unroll
    for (int i = 0; i < D; i++) zprev[i] = group_prev_fill<L>(z[K - 1][i], l, z0[i]);
    typename F::template Cache<T> C[K];
    T rp = T(0), rx = T(0);
#pragma unroll
    for (int kk = 0; kk < K; kk++) {
      T v[D];
#pragma unroll
      for (int i = 0; i < D; i++) v[i] = p[kk][i] + sigma * (z[kk][i] - (kk == 0 ? zprev[i] : z[kk - 1][i]));
      F::dual(P, x[kk], v, sd, C[kk]);
      if constexpr (!F::kZeroSafe) {
        // nodes past N keep p = 0
        const int j = 1 + l * K + kk;
#pragma unroll
        for (int i = 0; i < D; i++) v[i] = (j <= Np) ? v[i] : T(0);
      }
#pragma unroll
      for (int i = 0; i < D; i++) {
        const T dp = v[i] - p[kk][i];
        rp += dp * dp;
        p[kk][i] = v[i];
      }
    }
    // ---- node 0 -----------------------------------------------------------
    T pnext[D];
#pragma unroll
    for (int i = 0; i < D; i++) pnext[i] = group_next0<L>(p[0][i], l);
    if (l == 0) {
      T dx0[D];
      F::step0(P, x0, p[0], tau, dx0);
#pragma unroll
      for (int i = 0; i < D; i++) {
        rx += dx0[i] * dx0[i];
        z0[i] = x0[i] + (T(1) + theta) * dx0[i];
        x0[i] += dx0[i];
      }
    }
    // ---- primal step --------------------------------------------------------
    // Nodes j >= N take no step: their tau and tau*delta are 0 (x_N = x stays
    // fixed, and past N nothing moves).
#pragma unroll
    for (int kk = 0; kk < K; kk++) {
      T g[D];
      F::grad(P, x[kk], p[kk], C[kk], g);
#pragma unroll
      for (int i = 0; i < D; i++) {
        const T pp = (kk == K - 1) ? pnext[i] : p[kk + 1][i];
        const T dx = tdj[kk] * g[i] - tj[kk] * (p[kk][i] - pp);
        rx += dx * dx;
        z[kk][i] = x[kk][i] + (T(1) + theta) * dx;
        x[kk][i] += dx;
      }
    }
    // ---- stopping rule (section 6 set-up) ------------------------------------
    k++;
    const T rxs = group_sum<L>(rx), rps = group_sum<L>(rp);
    const bool fin = M<T>::finite(rxs + rps);
    const bool small = (rxs < a.tol) && (rps < a.tol);
    bool done;
    int st = kMaxIter;
    if constexpr (!kRec) {
      done = active && (!fin || (!a.fixed && small) || k >= a.max_iter);
      st = !fin ? kNonFinite : (small ? kConverged : kMaxIter);
    } else {
      // recipes (tolerance mode only): cap -> raise sigma and continue, up to
      // a.restarts times; after the first cap also stop on a stalled value
      kp++;
      done = false;
      if (active) {
        if (!fin) {
          done = true;
          st = kNonFinite;
        } else if (small) {
          done = true;
          st = kConverged;
        } else {
          if (phase >= 1 && a.value_tol > T(0)) {
            int bad_v = 0;
            const T val = lagrangian(bad_v);
            if (have_prev && M<T>::fabs_(val - prev_val) <= a.value_tol * M<T>::fmax(M<T>::fabs_(val), T(1))) {
              done = true;
              st = kValueStalled;
            }
            prev_val = val;
            have_prev = true;
          }
          if (!done && kp >= a.max_iter) {
            if (phase < a.restarts) {
              phase++;
              kp = 0;
              have_prev = false;
              sigma += a.sigma_inc;
              tau = a.sigma * a.tau / sigma;
              set_steps();
            } else {
              done = true;
              st = kMaxIter;
            }
          }
        }
      }
    }
    if (done) {
      int bad = 0;
      const T acc = lagrangian(bad);
      if (bad || !M<T>::finite(acc)) st = kNonFinite;
      bool write = true;
      if constexpr (kRec) {
        // several starts: keep the lowest value among those that met a stopping
        // rule, else the lowest finite value; ties keep the earlier start
        const int rank = (st == kConverged || st == kValueStalled) ? 0 : (M<T>::finite(acc) ? 1 : 2);
        write = rank < best_rank || (rank == best_rank && rank < 2 && acc < best_phi);
        if (write) {
          best_rank = rank;
          best_phi = acc;
        }
      }
      if (write) {
        if (l == 0) {
          a.phi[pt] = acc;
          a.iters[pt] = k;
          a.status[pt] = st;
        }
        const int64_t base = pt * int64_t(a.N_max + 1) * a.d;
        if (a.xtraj) {
#pragma unroll
          for (int kk = 0; kk < K; kk++) {
            const int j = 1 + l * K + kk;
            if (j <= Np)
#pragma unroll
              for (int i = 0; i < D; i++) a.xtraj[base + j * D + i] = x[kk][i];
          }
          if (l == 0)
#pragma unroll
            for (int i = 0; i < D; i++) a.xtraj[base + i] = x0[i];
        }
        if (a.ptraj) {
#pragma unroll
          for (int kk = 0; kk < K; kk++) {
            const int j = 1 + l * K + kk;
            if (j <= Np)
#pragma unroll
              for (int i = 0; i < D; i++) a.ptraj[base + j * D + i] = p[kk][i];
          }
          if (l == 0)
#pragma unroll
            for (int i = 0; i < D; i++) a.ptraj[base + i] = T(0);
        }
      }
      if constexpr (kRec) {
        if (start + 1 < a.starts) init_start(start + 1);
        else pop_and_init();
      } else {
        pop_and_init();
      }
    }
    if (__any(done || (active && prio.step(k)))) set_wave_priority(active, k, prio);
  }
}

// ---------------------------------------------------------------------------
// Persistent lane-group kernel for the eikonal family, Lax formulation, with
// the node layout shifted by one: slot kk of lane l holds the primal node
// j = lK + kk (x_j, z_j) and the dual node j + 1 (p_{j+1}).  Node 0 is the
// first lane's slot 0, an ordinary primal slot whose step is followed by the
// prox of g (the first lane only); node L*K, when N fills the tile, is the
// query point, supplied by the group's last lane.  No lane carries a separate
// node-0 state.  Per iteration (Algorithm 1):
//   p_{j+1} <- shrink_2(p_{j+1} + sigma (z_{j+1} - z_j), sigma delta c(x_{j+1}))
//   x_j <- x_j - tau (p_j - p_{j+1}) + tau delta |p_j| grad c(x_j)
//   x_0 <- prox_{tau g}(that step)            (p_0 = 0)
// z_{j+1} and c(x_{j+1}) of a lane's last slot come from the next lane, p_j
// and |p_j| of its first slot from the previous lane: two D-wide and two
// scalar DPP row shifts.  Against k_group_control this removes the node-0
// block that every lane issued for one lane per group, and the x_0, z_0
// registers of every lane.
// The dual is held scaled by tau (registers ps = tau p): the shrink commutes
// with the scaling, so the dual step is unchanged in form, and the primal
// difference term becomes ps_{j+1} - ps_j with no multiply.  Slots that do not
// move (past N, and node 0 in the Hopf formulation) are masked where x and z
// are updated, by a 0/1 factor per slot, instead of in every coordinate of the
// step.  For the shifted quadratic g the node-0 prox is affine,
// m (x_0 + dx) + f, and is applied to the step as m dx + ((m - 1) x_0 + f).
// The p residual is tau^2 times the unscaled one and is tested against
// tau^2 tol; the value and p outputs are scaled back by 1/tau.  The p residual
// matters only once the x residual is below tol; in FP32 tiles with at most
// two nodes per lane it is formed only then.
// Hopf formulation (Algorithm 2, kHopf): node 0 does not exist; its slot
// keeps x_0 = z_0 = 0 (the Hopf difference operator) and takes no step, node
// 1's dual step is the joint prox with g*, and the value has -g*(p_1) in
// place of g(x_0).
// ---------------------------------------------------------------------------
// The family F marked for the weighted Euler rules (forward Euler, trapezoid)
// in k_group_control_shift: the saddle g(x_0) + sum_j <p_j, x_j - x_{j-1}> -
// delta sum_j (wl c(x_{j-1}) + wr c(x_j)) |p_j| (KArgs::wl, wr).  Slot kk's
// dual p_{j+1} shrinks by sigma delta (wl c(x_j) + wr c(x_{j+1})); x_j's
// gradient weight is tau delta (wr |p_j| + wl |p_{j+1}|), so node 0 takes the
// proximal-gradient step prox_{tau g}(x_0 + tau p_1 + tau delta wl |p_1|
// grad c(x_0)).
template <class F> struct Weighted : F {};
template <class F> struct IsWeighted { static constexpr bool value = false; };
template <class F> struct IsWeighted<Weighted<F>> { static constexpr bool value = true; };

template <typename T, class F, int L, int K, bool kHopf>
__global__ void __launch_bounds__(256, (kShiftWaves<T, K>)) k_group_control_shift(KArgs<T> a) {
  constexpr bool kMix = IsWeighted<F>::value;  // the weighted Euler rules (F = Weighted<...>, above)
  static_assert(!(kHopf && kMix), "weighted Euler rules are built for the Lax formulation only");
  constexpr int D = F::D;
  const int lane = threadIdx.x & 63;
  const int l = lane & (L - 1);
  const int leader = lane - l;
  const bool first = (l == 0), last = (l == L - 1);

  typename F::template Par<T> P;
  F::load(P, a.hp, a.gp, a.gkind, a.tau);
  const WavePrio prio(a.max_iter);
  const int beg = a.cls_range[2 * a.cls], end = a.cls_range[2 * a.cls + 1];
  int32_t* head = a.heads + a.cls;
  const T sigma = a.sigma, tau = a.tau, theta = a.theta;
  const T ts = tau * sigma, itau = T(1) / tau, tolp = a.tol * tau * tau;
  const T wl = a.wl, wr = a.wr;  // weighted rule (kMix): H weights at an interval's left / right node
  // node-0 prox as m v + f (first lane; identity elsewhere) when it is affine
  T m0, f0[D];
  const bool aff0 = F::prox0_affine(P, first, m0, f0);
  const T mm0 = m0 - T(1);
  // Lazy p residual (below) keeps the previous dual live through the primal
  // step: K*D more registers, taken only where the register budget is modest
  // (FP32, at most two nodes per lane).
  constexpr bool kLazyRp = sizeof(T) == 4 && K <= 2;

  T x[K][D], ps[K][D], z[K][D];
  T xe[D], ce;      // the query point x and c(x) in the group's last lane, 0 elsewhere
  T mv[K], mz[K];   // per primal slot: 1 and theta where the node moves, else 0
  T delta = T(0), tsd = T(0);
  int Np = 0, k = 0;
  int64_t pt = -1;
  bool active = false;

  auto pop_and_init = [&]() {
    int idx = 0;
    // without refill a group serves the one point it popped first
    if (l == 0) idx = (a.refill || pt < 0) ? atomicAdd(head, 1) : (end - beg);
    idx = __shfl(idx, leader, 64);
    const int qi = beg + idx;
    active = qi < end;
    if (!active) return;
    pt = a.queue[qi];
    if (a.pops && l == 0) atomicAdd(a.pops + pt, 1);
    Np = a.N[pt];
    delta = a.t[pt] / T(Np);
    tsd = ts * delta;
    k = 0;
    T xt[D];
#pragma unroll
    for (int i = 0; i < D; i++) xt[i] = a.x[pt * a.d + i];
#pragma unroll
    for (int kk = 0; kk < K; kk++) {
      const int j = l * K + kk;
      const bool moves = (j < Np) && !(kHopf && j == 0);  // Hopf: no node 0
#pragma unroll
      for (int i = 0; i < D; i++) {
        x[kk][i] = moves ? init_x(xt[i], a.seed, pt, kArrX, j, i) : ((j < Np) ? T(0) : xt[i]);
        ps[kk][i] = (j + 1 <= Np) ? tau * T(start_noise(a.seed, uint64_t(pt), kArrP, j + 1, i)) : T(0);
        z[kk][i] = x[kk][i];
      }
      mv[kk] = moves ? T(1) : T(0);
      mz[kk] = moves ? theta : T(0);
    }
    T cq, g0, g1;
    F::speed(P, xt, cq, g0, g1);
    ce = last ? cq : T(0);
#pragma unroll
    for (int i = 0; i < D; i++) xe[i] = last ? xt[i] : T(0);
  };

  pop_and_init();

  while (__any(active)) {
    // ---- speeds at the current iterate (own primal slots) --------------------
    T cj[K], gc0[K], gc1[K];
#pragma unroll
    for (int kk = 0; kk < K; kk++) F::speed(P, x[kk], cj[kk], gc0[kk], gc1[kk]);
    // right neighbour of the last slot: next lane's slot 0, or x in the last lane
    T znext[D];
#pragma unroll
    for (int i = 0; i < D; i++) znext[i] = group_next0<L>(z[0][i], l) + xe[i];
    const T cnext = group_next0<L>(cj[0], l) + ce;
    // ---- dual step: tau p_{j+1} in slot kk -------------------------------------
    T pn[K];  // tau |p_{j+1}|
    T pold[K][D];
    T rp = T(0), rx = T(0);
#pragma unroll
    for (int kk = 0; kk < K; kk++) {
      T v[D];
#pragma unroll
      for (int i = 0; i < D; i++) v[i] = ps[kk][i] + ts * ((kk == K - 1 ? znext[i] : z[kk + 1][i]) - z[kk][i]);
      // interval (j, j+1): speed of its right node; the weighted rule mixes
      // in its left node's (this slot's own primal node)
      const T cr = kMix ? wl * cj[kk] + wr * ((kk == K - 1) ? cnext : cj[kk + 1])
                        : ((kk == K - 1) ? cnext : cj[kk + 1]);
      if constexpr (kHopf) {
        if (kk == 0) pn[kk] = F::shrink_hopf1(P, v, tsd * cr, sigma, first, tau);  // node 1: with g*
        else pn[kk] = F::shrink(v, tsd * cr);
      } else {
        pn[kk] = F::shrink(v, tsd * cr);
      }
#pragma unroll
      for (int i = 0; i < D; i++) {
        if constexpr (kLazyRp) {
          pold[kk][i] = ps[kk][i];
        } else {
          const T dp = v[i] - ps[kk][i];
          rp += dp * dp;
        }
        ps[kk][i] = v[i];
      }
    }
    // ---- primal step: x_j in slot kk; p_j of the first slot from the previous
    //      lane (p_0 = 0 in the first lane) --------------------------------------
    T pprev[D];
#pragma unroll
    for (int i = 0; i < D; i++) pprev[i] = group_prev0<L>(ps[K - 1][i], l);
    const T pnprev = group_prev0<L>(pn[K - 1], l);
#pragma unroll
    for (int kk = 0; kk < K; kk++) {
      // tau delta |p_j| (interval (j-1, j)); the weighted rule takes
      // tau delta (wr |p_j| + wl |p_{j+1}|), x_j bounding both intervals
      const T pj = (kk == 0) ? pnprev : pn[kk - 1];
      const T coef = kMix ? delta * (wr * pj + wl * pn[kk]) : delta * pj;
      T dx[D];
#pragma unroll
      for (int i = 0; i < D; i++) dx[i] = ps[kk][i] - ((kk == 0) ? pprev[i] : ps[kk - 1][i]);
      dx[0] += coef * gc0[kk];
      dx[1] += coef * gc1[kk];
      if constexpr (!kHopf) {
        if (kk == 0) {
          // node 0 (first lane): the prox of g after the step
          if (aff0) {
#pragma unroll
            for (int i = 0; i < D; i++) dx[i] = m0 * dx[i] + (mm0 * x[0][i] + f0[i]);
          } else {
            T v[D];
#pragma unroll
            for (int i = 0; i < D; i++) v[i] = x[0][i] + dx[i];
            F::prox0(P, v, tau, first);
#pragma unroll
            for (int i = 0; i < D; i++) dx[i] = v[i] - x[0][i];
          }
        }
      }
      T sx = T(0);
#pragma unroll
      for (int i = 0; i < D; i++) {
        sx += dx[i] * dx[i];
        x[kk][i] += mv[kk] * dx[i];
        z[kk][i] = x[kk][i] + mz[kk] * dx[i];
      }
      rx += mv[kk] * sx;
    }
    // ---- stopping rule (section 6 set-up) ------------------------------------
    k++;
    // Lazy form: the p residual decides only where the x residual is already
    // below tol, so it is formed (from the stored iterates) only when some
    // group of the wave gets there, and is 0 otherwise.
    const T rxs = group_sum<L>(rx);
    T rps = T(0);
    if constexpr (kLazyRp) {
      if (__any(active && rxs < a.tol)) {
#pragma unroll
        for (int kk = 0; kk < K; kk++)
#pragma unroll
          for (int i = 0; i < D; i++) {
            const T dp = ps[kk][i] - pold[kk][i];
            rp += dp * dp;
          }
        rps = group_sum<L>(rp);
      }
    } else {
      rps = group_sum<L>(rp);
    }
    const bool fin = M<T>::finite(rxs + rps);
    const bool small = (rxs < a.tol) && (rps < tolp);
    const bool done = active && (!fin || (!a.fixed && small) || k >= a.max_iter);
    if (done) {
      // value: g(x_0) + sum_j <p_j, x_j - x_{j-1}> - delta sum_j c(x_j) |p_j|,
      // the sum taken over tau p and scaled back
#pragma unroll
      for (int kk = 0; kk < K; kk++) F::speed(P, x[kk], cj[kk], gc0[kk], gc1[kk]);
      const T cn2 = group_next0<L>(cj[0], l) + ce;
      T xnext[D];
#pragma unroll
      for (int i = 0; i < D; i++) xnext[i] = group_next0<L>(x[0][i], l) + xe[i];
      T acc = T(0);
      int bad = 0;
#pragma unroll
      for (int kk = 0; kk < K; kk++) {
        const int j = l * K + kk + 1;  // dual node of the slot
        if (j <= Np) {
          T s = T(0), ss = T(0);
#pragma unroll
          for (int i = 0; i < D; i++) {
            s += ps[kk][i] * ((kk == K - 1 ? xnext[i] : x[kk + 1][i]) - x[kk][i]);
            ss += ps[kk][i] * ps[kk][i];
          }
          const T cr = kMix ? wl * cj[kk] + wr * ((kk == K - 1) ? cn2 : cj[kk + 1])
                            : ((kk == K - 1) ? cn2 : cj[kk + 1]);
          acc += s - delta * cr * M<T>::sqrt(ss);
          bad |= !(all_finite<T, D>(x[kk]) && all_finite<T, D>(ps[kk]));
        }
      }
      acc *= itau;
      if (first) {
        if constexpr (kHopf) {  // -g*(p_1), x_0 = 0
          T p1[D];
#pragma unroll
          for (int i = 0; i < D; i++) p1[i] = ps[0][i] * itau;
          acc -= F::gstar(P, p1);
        } else {
          acc += F::g(P, x[0]);
        }
      }
      acc = group_sum<L>(acc);
      bad = group_or<L>(bad);
      int st = !fin ? kNonFinite : (small ? kConverged : kMaxIter);
      if (bad || !M<T>::finite(acc)) st = kNonFinite;
      if (first) {
        a.phi[pt] = acc;
        a.iters[pt] = k;
        a.status[pt] = st;
      }
      const int64_t base = pt * int64_t(a.N_max + 1) * a.d;
      if (a.xtraj) {
#pragma unroll
        for (int kk = 0; kk < K; kk++) {
          const int j = l * K + kk;
          if (j <= Np)
#pragma unroll
            for (int i = 0; i < D; i++) a.xtraj[base + j * D + i] = x[kk][i];
        }
        if (first && Np == L * K)  // node N lies past the tile: the query point
#pragma unroll
          for (int i = 0; i < D; i++) a.xtraj[base + Np * D + i] = a.x[pt * a.d + i];
      }
      if (a.ptraj) {
#pragma unroll
        for (int kk = 0; kk < K; kk++) {
          const int j = l * K + kk + 1;
          if (j <= Np)
#pragma unroll
            for (int i = 0; i < D; i++) a.ptraj[base + j * D + i] = ps[kk][i] * itau;
        }
        if (first)
#pragma unroll
          for (int i = 0; i < D; i++) a.ptraj[base + i] = T(0);
      }
      pop_and_init();
    }
    if (__any(done || (active && prio.step(k)))) set_wave_priority(active, k, prio);
  }
}


// ---------------------------------------------------------------------------
// Persistent lane-group kernel, game path (Algorithm 3) for games whose
// Hamiltonian separates as H = Hx(x, p) + Hy(y, q): block order p, q, x, y.
// kRec adds the two recipes of section 6 that the paper applies to a game
// (sigma raised at the iteration cap, continuing from the iterate; after the
// first cap a value-change stop), with per-point step sizes; kRec = false is
// the plain iteration with constant steps.
// ---------------------------------------------------------------------------
template <typename T, class F, int L, int K, bool kRec = false>
__global__ void __launch_bounds__(256, (kFamWaves<T, F, K>)) k_group_game(KArgs<T> a) {
  constexpr int DX = F::DX, DY = F::DY, D = F::D;
  const int lane = threadIdx.x & 63;
  const int l = lane & (L - 1);
  const int leader = lane - l;

  typename F::template Par<T> P;
  F::load(P, a.hp, a.gp, a.gkind, a.tau);
  const WavePrio prio(a.max_iter);
  const int beg = a.cls_range[2 * a.cls], end = a.cls_range[2 * a.cls + 1];
  int32_t* head = a.heads + a.cls;
  const T theta = a.theta;
  // step sizes: kernel constants, or per point when the recipes raise sigma
  T sigma = a.sigma, tau = a.tau;

  T x[K][DX], p[K][DX], z[K][DX], y[K][DY], q[K][DY], w[K][DY];
  T x0[DX], z0[DX], y0[DY], w0[DY];
  T tj[K], tdj[K];  // per node: tau and tau*delta where the node takes a primal step, else 0
  // per node: sigma*delta and the velocity-costate factors of the p- and q-steps
  // where the node has a dual (j <= N), else 0 and 1 (the step then maps the
  // zero costate of a node past N to itself, with no branch)
  T sdj[K], ipj[K], iqj[K];
  T delta = T(0), sd = T(0), td = T(0);
  int Np = 0, k = 0;
  int64_t pt = -1;
  bool active = false;
  // recipe state (dead code without kRec)
  int phase = 0, kp = 0;
  T prev_val = T(0);
  bool have_prev = false;

  // per-node step sizes of the current point
  auto set_steps = [&]() __attribute__((always_inline)) {
    sd = sigma * delta;
    td = tau * delta;
    T ip, iq;
    F::dual_scales(P, sd, ip, iq);
#pragma unroll
    for (int kk = 0; kk < K; kk++) {
      const int j = 1 + l * K + kk;
      tj[kk] = (j < Np) ? tau : T(0);
      tdj[kk] = (j < Np) ? td : T(0);
      sdj[kk] = (j <= Np) ? sd : T(0);
      ipj[kk] = (j <= Np) ? ip : T(1);
      iqj[kk] = (j <= Np) ? iq : T(1);
    }
  };

  auto pop_and_init = [&]() {
    int idx = 0;
    // without refill a group serves the one point it popped first
    if (l == 0) idx = (a.refill || pt < 0) ? atomicAdd(head, 1) : (end - beg);
    idx = __shfl(idx, leader, 64);
    const int qi = beg + idx;
    active = qi < end;
    if (!active) return;
    pt = a.queue[qi];
    if (a.pops && l == 0) atomicAdd(a.pops + pt, 1);
    Np = a.N[pt];
    delta = a.t[pt] / T(Np);
    k = 0;
    if constexpr (kRec) {
      phase = 0;
      kp = 0;
      have_prev = false;
      sigma = a.sigma;
      tau = a.tau;
    }
    T xt[D];
#pragma unroll
    for (int i = 0; i < D; i++) xt[i] = a.x[pt * a.d + i];
#pragma unroll
    for (int kk = 0; kk < K; kk++) {
      const int j = 1 + l * K + kk;
#pragma unroll
      for (int i = 0; i < DX; i++) {
        x[kk][i] = (j < Np) ? init_x(xt[i], a.seed, pt, kArrX, j, i) : xt[i];
        p[kk][i] = (j <= Np) ? T(start_noise(a.seed, uint64_t(pt), kArrP, j, i)) : T(0);
        z[kk][i] = x[kk][i];
      }
#pragma unroll
      for (int i = 0; i < DY; i++) {
        y[kk][i] = (j < Np) ? init_x(xt[DX + i], a.seed, pt, kArrY, j, i) : xt[DX + i];
        q[kk][i] = (j <= Np) ? T(start_noise(a.seed, uint64_t(pt), kArrQ, j, i)) : T(0);
        w[kk][i] = y[kk][i];
      }
    }
    // node 0 lives in the group's first lane; the other lanes keep x0 = z0 = y0 = w0 = 0
#pragma unroll
    for (int i = 0; i < DX; i++) {
      x0[i] = (l == 0) ? init_x(xt[i], a.seed, pt, kArrX, 0, i) : T(0);
      z0[i] = x0[i];
    }
#pragma unroll
    for (int i = 0; i < DY; i++) {
      y0[i] = (l == 0) ? init_x(xt[DX + i], a.seed, pt, kArrY, 0, i) : T(0);
      w0[i] = y0[i];
    }
    set_steps();
  };

  // The value: the Lagrangian at the current iterate, g(x_0, y_0) +
  // sum_j (<p_j, x_j - x_{j-1}> - <q_j, y_j - y_{j-1}>) - delta sum_j H,
  // summed over the group; `bad` flags a non-finite entry.
  auto lagrangian = [&](int& bad) __attribute__((always_inline)) {
    T xprev[DX], yprev[DY];
#pragma unroll
    for (int i = 0; i < DX; i++) xprev[i] = group_prev_fill<L>(x[K - 1][i], l, x0[i]);
#pragma unroll
    for (int i = 0; i < DY; i++) yprev[i] = group_prev_fill<L>(y[K - 1][i], l, y0[i]);
    T acc = T(0);
    bad = 0;
#pragma unroll
    for (int kk = 0; kk < K; kk++) {
      const int j = 1 + l * K + kk;
      if (j <= Np) {
        T s = T(0);
#pragma unroll
        for (int i = 0; i < DX; i++) s += p[kk][i] * (x[kk][i] - (kk == 0 ? xprev[i] : x[kk - 1][i]));
#pragma unroll
        for (int i = 0; i < DY; i++) s -= q[kk][i] * (y[kk][i] - (kk == 0 ? yprev[i] : y[kk - 1][i]));
        acc += s - delta * F::H(P, x[kk], y[kk], p[kk], q[kk]);
        bad |= !(all_finite<T, DX>(x[kk]) && all_finite<T, DX>(p[kk]) && all_finite<T, DY>(y[kk]) &&
                 all_finite<T, DY>(q[kk]));
      }
    }
    if (l == 0) {
      acc += F::g(P, x0, y0);
      bad |= !(all_finite<T, DX>(x0) && all_finite<T, DY>(y0));
    }
    bad = group_or<L>(bad);
    return group_sum<L>(acc);
  };

  pop_and_init();

  while (__any(active)) {
    T zprev[DX], wprev[DY];
#pragma unroll
    for (int i = 0; i < DX; i++) zprev[i] = group_prev_fill<L>(z[K - 1][i], l, z0[i]);
#pragma unroll
    for (int i = 0; i < DY; i++) wprev[i] = group_prev_fill<L>(w[K - 1][i], l, w0[i]);
    typename F::template CacheX<T> CX[K];
    typename F::template CacheY<T> CY[K];
    T rp = T(0), rq = T(0), rx = T(0), ry = T(0);
    // ---- p block, then q block ----------------------------------------------
#pragma unroll
    for (int kk = 0; kk < K; kk++) {
      T v[DX];
#pragma unroll
      for (int i = 0; i < DX; i++) v[i] = p[kk][i] + sigma * (z[kk][i] - (kk == 0 ? zprev[i] : z[kk - 1][i]));
      F::dual_p(P, x[kk], v, sdj[kk], ipj[kk], CX[kk]);
      T u[DY];
#pragma unroll
      for (int i = 0; i < DY; i++) u[i] = q[kk][i] + sigma * (w[kk][i] - (kk == 0 ? wprev[i] : w[kk - 1][i]));
      F::dual_q(P, y[kk], u, sdj[kk], iqj[kk], CY[kk]);
      // nodes past N: v = u = 0 and the step leaves them at 0 (p = q = 0 stays, no residual)
#pragma unroll
      for (int i = 0; i < DX; i++) {
        const T dp = v[i] - p[kk][i];
        rp += dp * dp;
        p[kk][i] = v[i];
      }
#pragma unroll
      for (int i = 0; i < DY; i++) {
        const T dq = u[i] - q[kk][i];
        rq += dq * dq;
        q[kk][i] = u[i];
      }
    }
    T pnext[DX], qnext[DY];
#pragma unroll
    for (int i = 0; i < DX; i++) pnext[i] = group_next0<L>(p[0][i], l);
#pragma unroll
    for (int i = 0; i < DY; i++) qnext[i] = group_next0<L>(q[0][i], l);
    // ---- node 0 (the group's first lane): x_0 by the prox of g(., y_0^k), then
    //      y_0 by the prox of -g(x_0^{k+1}, .), in one branch (neither depends
    //      on the other nodes' primal steps).  A branch, not masked arithmetic
    //      in every lane: measured, the branch costs the wave less.
    if (l == 0) {
      T v0[DX], xn0[DX], u0[DY], yn0[DY];
#pragma unroll
      for (int i = 0; i < DX; i++) v0[i] = x0[i] + tau * p[0][i];
      F::prox_x0(P, v0, y0, tau, xn0);
#pragma unroll
      for (int i = 0; i < DY; i++) u0[i] = y0[i] + tau * q[0][i];
      F::stretch_y0(P, u0, xn0, tau, yn0);
#pragma unroll
      for (int i = 0; i < DX; i++) {
        const T dx = xn0[i] - x0[i];
        rx += dx * dx;
        z0[i] = xn0[i] + theta * dx;
        x0[i] = xn0[i];
      }
#pragma unroll
      for (int i = 0; i < DY; i++) {
        const T dy = yn0[i] - y0[i];
        ry += dy * dy;
        w0[i] = yn0[i] + theta * dy;
        y0[i] = yn0[i];
      }
    }
    // ---- x block: descent steps ---------------------------------------------------
#pragma unroll
    for (int kk = 0; kk < K; kk++) {
      T g[DX];
      F::grad_x(P, x[kk], p[kk], CX[kk], g);
#pragma unroll
      for (int i = 0; i < DX; i++) {
        const T pp = (kk == K - 1) ? pnext[i] : p[kk + 1][i];
        const T dx = tdj[kk] * g[i] - tj[kk] * (p[kk][i] - pp);
        rx += dx * dx;
        z[kk][i] = x[kk][i] + (T(1) + theta) * dx;
        x[kk][i] += dx;
      }
    }
    // ---- y block: ascent steps -----------------------------------------------------
#pragma unroll
    for (int kk = 0; kk < K; kk++) {
      T g[DY];
      F::grad_y(P, y[kk], q[kk], CY[kk], g);
#pragma unroll
      for (int i = 0; i < DY; i++) {
        const T qq = (kk == K - 1) ? qnext[i] : q[kk + 1][i];
        const T dy = -tdj[kk] * g[i] - tj[kk] * (q[kk][i] - qq);
        ry += dy * dy;
        w[kk][i] = y[kk][i] + (T(1) + theta) * dy;
        y[kk][i] += dy;
      }
    }
    // ---- stopping rule ------------------------------------------------------------
    k++;
    const T rxs = group_sum<L>(rx), rps = group_sum<L>(rp), rys = group_sum<L>(ry), rqs = group_sum<L>(rq);
    const bool fin = M<T>::finite(rxs + rps + rys + rqs);
    const bool small = (rxs < a.tol) && (rps < a.tol) && (rys < a.tol) && (rqs < a.tol);
    bool done;
    int st = kMaxIter;
    if constexpr (!kRec) {
      done = active && (!fin || (!a.fixed && small) || k >= a.max_iter);
    } else {
      // recipes (tolerance mode): cap -> raise sigma and continue, up to
      // a.restarts times; after the first cap also stop on a stalled value
      kp++;
      done = false;
      if (active) {
        if (!fin) {
          done = true;
          st = kNonFinite;
        } else if (small) {
          done = true;
          st = kConverged;
        } else {
          if (phase >= 1 && a.value_tol > T(0)) {
            int bad_v = 0;
            const T val = lagrangian(bad_v);
            if (have_prev && M<T>::fabs_(val - prev_val) <= a.value_tol * M<T>::fmax(M<T>::fabs_(val), T(1))) {
              done = true;
              st = kValueStalled;
            }
            prev_val = val;
            have_prev = true;
          }
          if (!done && kp >= a.max_iter) {
            if (phase < a.restarts) {
              phase++;
              kp = 0;
              have_prev = false;
              sigma += a.sigma_inc;
              tau = a.sigma * a.tau / sigma;
              set_steps();
            } else {
              done = true;
              st = kMaxIter;
            }
          }
        }
      }
    }
    if (done) {
      // the value, as lagrangian() computes it, written out here: calling the
      // lambda in this place measured 6 % slower for the plain kernel (the
      // compiler schedules the iteration differently)
      T xprev[DX], yprev[DY];
#pragma unroll
      for (int i = 0; i < DX; i++) xprev[i] = group_prev_fill<L>(x[K - 1][i], l, x0[i]);
#pragma unroll
      for (int i = 0; i < DY; i++) yprev[i] = group_prev_fill<L>(y[K - 1][i], l, y0[i]);
      T acc = T(0);
      int bad = 0;
#pragma unroll
      for (int kk = 0; kk < K; kk++) {
        const int j = 1 + l * K + kk;
        if (j <= Np) {
          T s = T(0);
#pragma unroll
          for (int i = 0; i < DX; i++) s += p[kk][i] * (x[kk][i] - (kk == 0 ? xprev[i] : x[kk - 1][i]));
#pragma unroll
          for (int i = 0; i < DY; i++) s -= q[kk][i] * (y[kk][i] - (kk == 0 ? yprev[i] : y[kk - 1][i]));
          acc += s - delta * F::H(P, x[kk], y[kk], p[kk], q[kk]);
          bad |= !(all_finite<T, DX>(x[kk]) && all_finite<T, DX>(p[kk]) && all_finite<T, DY>(y[kk]) &&
                   all_finite<T, DY>(q[kk]));
        }
      }
      if (l == 0) {
        acc += F::g(P, x0, y0);
        bad |= !(all_finite<T, DX>(x0) && all_finite<T, DY>(y0));
      }
      acc = group_sum<L>(acc);
      bad = group_or<L>(bad);
      if constexpr (!kRec) st = !fin ? kNonFinite : (small ? kConverged : kMaxIter);
      if (bad || !M<T>::finite(acc)) st = kNonFinite;
      if (l == 0) {
        a.phi[pt] = acc;
        a.iters[pt] = k;
        a.status[pt] = st;
      }
      const int64_t base = pt * int64_t(a.N_max + 1) * a.d;
      if (a.xtraj) {
#pragma unroll
        for (int kk = 0; kk < K; kk++) {
          const int j = 1 + l * K + kk;
          if (j <= Np) {
#pragma unroll
            for (int i = 0; i < DX; i++) a.xtraj[base + j * D + i] = x[kk][i];
#pragma unroll
            for (int i = 0; i < DY; i++) a.xtraj[base + j * D + DX + i] = y[kk][i];
          }
        }
        if (l == 0) {
#pragma unroll
          for (int i = 0; i < DX; i++) a.xtraj[base + i] = x0[i];
#pragma unroll
          for (int i = 0; i < DY; i++) a.xtraj[base + DX + i] = y0[i];
        }
      }
      if (a.ptraj) {
#pragma unroll
        for (int kk = 0; kk < K; kk++) {
          const int j = 1 + l * K + kk;
          if (j <= Np) {
#pragma unroll
            for (int i = 0; i < DX; i++) a.ptraj[base + j * D + i] = p[kk][i];
#pragma unroll
            for (int i = 0; i < DY; i++) a.ptraj[base + j * D + DX + i] = q[kk][i];
          }
        }
        if (l == 0)
#pragma unroll
          for (int i = 0; i < D; i++) a.ptraj[base + i] = T(0);
      }
      pop_and_init();
    }
    if (__any(done || (active && prio.step(k)))) set_wave_priority(active, k, prio);
  }
}

// ---------------------------------------------------------------------------
// Persistent lane-group kernel, game Hopf formulation (Algorithm 4) for a
// separable convex-concave initial cost, families with scalar players
// (Isaacs).  Nodes 1..N, no node 0: z_0 = w_0 = 0 (the Hopf difference
// operator), and at node 1 the costate steps take -e*(p_1) and -h_*(-q_1)
// in.  Per iteration, node by node: p (uses x^k, y^k, q^k), then q (uses the
// new p); then x (descent, at y^k), then y (ascent, at the new x).  Value:
//   -e*(p_1) - h_*(-q_1) + sum_j (p_j (x_j - x_{j-1}) - q_j (y_j - y_{j-1}))
//   - delta sum_j H(x_j, y_j, p_j, -q_j),  x_0 = y_0 = 0,
// which is eq. discgenlaxhopfdghopf's objective after summation by parts.
// ---------------------------------------------------------------------------
template <typename T, class F, int L, int K, bool kLax = false>
__global__ void __launch_bounds__(256, (kFamWaves<T, F, K>)) k_group_game_hopf(KArgs<T> a) {
  static_assert(F::DX == 1 && F::DY == 1, "scalar players");
  constexpr int D = F::D;
  const int lane = threadIdx.x & 63;
  const int l = lane & (L - 1);
  const int leader = lane - l;

  typename F::template Par<T> P;
  F::load(P, a.hp, a.gp, a.gkind, a.tau);
  const WavePrio prio(a.max_iter);
  const int beg = a.cls_range[2 * a.cls], end = a.cls_range[2 * a.cls + 1];
  int32_t* head = a.heads + a.cls;
  const T sigma = a.sigma, tau = a.tau, theta = a.theta;

  T x[K], y[K], p[K], q[K], z[K], w[K];
  // node 0 (kLax: Algorithm 3) in the group's first lane; zero elsewhere and in the Hopf formulation
  T x0 = T(0), y0 = T(0), z0 = T(0), w0 = T(0);
  T tj[K], tdj[K];  // per node: tau and tau*delta where the node takes a primal step, else 0
  T delta = T(0), sd = T(0), td = T(0), xN = T(0), yN = T(0);
  int Np = 0, k = 0;
  int64_t pt = -1;
  bool active = false;

  auto pop_and_init = [&]() {
    int idx = 0;
    // without refill a group serves the one point it popped first
    if (l == 0) idx = (a.refill || pt < 0) ? atomicAdd(head, 1) : (end - beg);
    idx = __shfl(idx, leader, 64);
    const int qi = beg + idx;
    active = qi < end;
    if (!active) return;
    pt = a.queue[qi];
    if (a.pops && l == 0) atomicAdd(a.pops + pt, 1);
    Np = a.N[pt];
    delta = a.t[pt] / T(Np);
    sd = sigma * delta;
    td = tau * delta;
    k = 0;
    xN = a.x[pt * a.d];
    yN = a.x[pt * a.d + 1];
#pragma unroll
    for (int kk = 0; kk < K; kk++) {
      const int j = 1 + l * K + kk;
      x[kk] = (j < Np) ? init_x(xN, a.seed, pt, kArrX, j, 0) : xN;
      y[kk] = (j < Np) ? init_x(yN, a.seed, pt, kArrY, j, 0) : yN;
      p[kk] = (j <= Np) ? T(start_noise(a.seed, uint64_t(pt), kArrP, j, 0)) : T(0);
      q[kk] = (j <= Np) ? T(start_noise(a.seed, uint64_t(pt), kArrQ, j, 0)) : T(0);
      z[kk] = x[kk];
      w[kk] = y[kk];
      tj[kk] = (j < Np) ? tau : T(0);
      tdj[kk] = (j < Np) ? td : T(0);
    }
    if constexpr (kLax) {
      x0 = (l == 0) ? init_x(xN, a.seed, pt, kArrX, 0, 0) : T(0);
      y0 = (l == 0) ? init_x(yN, a.seed, pt, kArrY, 0, 0) : T(0);
      z0 = x0;
      w0 = y0;
    }
  };

  pop_and_init();

  while (__any(active)) {
    // z_{j-1}, w_{j-1} of the lane's first node; in the group's first lane
    // node 0's (zero in the Hopf formulation, which has no node 0)
    const T zprev = group_prev_fill<L>(z[K - 1], l, z0), wprev = group_prev_fill<L>(w[K - 1], l, w0);
    T gx[K];  // d c/dx at (x^k, y^k)
    T rp = T(0), rq = T(0), rx = T(0), ry = T(0);
    // ---- p, then q, node by node ------------------------------------------------
#pragma unroll
    for (int kk = 0; kk < K; kk++) {
      const int j = 1 + l * K + kk;
      const bool first = !kLax && (l == 0) && (kk == 0);  // Hopf node 1: with e* and h_*
      T dcy;
      const T c = F::speed(P, x[kk], y[kk], gx[kk], dcy);
      const T v = p[kk] + sigma * (z[kk] - (kk == 0 ? zprev : z[kk - 1]));
      const T pn = F::dual_p(P, p[kk], q[kk], v, sd, sigma, first);
      const T u = q[kk] + sigma * (w[kk] - (kk == 0 ? wprev : w[kk - 1]));
      const T qn = F::dual_q(P, c, pn, q[kk], u, sd, sigma, first);
      if (j <= Np) {
        rp += (pn - p[kk]) * (pn - p[kk]);
        rq += (qn - q[kk]) * (qn - q[kk]);
        p[kk] = pn;
        q[kk] = qn;
      }
    }
    const T pnext = group_next0<L>(p[0], l), qnext = group_next0<L>(q[0], l);
    // ---- x: node 0 by the prox of e (Algorithm 3), then descent, grad_x H(x, y, p, -q) = q dc/dx
    if constexpr (kLax) {
      if (l == 0) {
        const T dx0 = F::prox_e(P, x0 + tau * p[0], tau) - x0;
        rx += dx0 * dx0;
        z0 = x0 + (T(1) + theta) * dx0;
        x0 += dx0;
      }
    }
#pragma unroll
    for (int kk = 0; kk < K; kk++) {
      const T pp = (kk == K - 1) ? pnext : p[kk + 1];
      const T dx = tdj[kk] * q[kk] * gx[kk] - tj[kk] * (p[kk] - pp);
      rx += dx * dx;
      z[kk] = x[kk] + (T(1) + theta) * dx;
      x[kk] += dx;
    }
    // ---- y: node 0 by the prox of -h (Algorithm 3), then ascent at the new x ---------
    if constexpr (kLax) {
      if (l == 0) {
        const T dy0 = F::prox_mh(P, y0 + tau * q[0], tau) - y0;
        ry += dy0 * dy0;
        w0 = y0 + (T(1) + theta) * dy0;
        y0 += dy0;
      }
    }
#pragma unroll
    for (int kk = 0; kk < K; kk++) {
      T dcx, dcy;
      (void)F::speed(P, x[kk], y[kk], dcx, dcy);
      const T qq = (kk == K - 1) ? qnext : q[kk + 1];
      const T dy = -tdj[kk] * q[kk] * dcy - tj[kk] * (q[kk] - qq);
      ry += dy * dy;
      w[kk] = y[kk] + (T(1) + theta) * dy;
      y[kk] += dy;
    }
    // ---- stopping rule: all four blocks -------------------------------------------
    k++;
    const T rxs = group_sum<L>(rx), rps = group_sum<L>(rp), rys = group_sum<L>(ry), rqs = group_sum<L>(rq);
    const bool fin = M<T>::finite(rxs + rps + rys + rqs);
    const bool small = (rxs < a.tol) && (rps < a.tol) && (rys < a.tol) && (rqs < a.tol);
    const bool done = active && (!fin || (!a.fixed && small) || k >= a.max_iter);
    if (done) {
      const T xprev = group_prev_fill<L>(x[K - 1], l, x0), yprev = group_prev_fill<L>(y[K - 1], l, y0);
      T acc = T(0);
      int bad = 0;
#pragma unroll
      for (int kk = 0; kk < K; kk++) {
        const int j = 1 + l * K + kk;
        if (j <= Np) {
          T dcx, dcy;
          const T c = F::speed(P, x[kk], y[kk], dcx, dcy);
          acc += p[kk] * (x[kk] - (kk == 0 ? xprev : x[kk - 1])) - q[kk] * (y[kk] - (kk == 0 ? yprev : y[kk - 1]))
                 - delta * F::H(c, p[kk], q[kk]);
          bad |= !(M<T>::finite(x[kk]) && M<T>::finite(y[kk]) && M<T>::finite(p[kk]) && M<T>::finite(q[kk]));
        }
      }
      if (l == 0) {
        // Algorithm 3: g(x_0, y_0); Algorithm 4: -e*(p_1) - h_*(-q_1)
        if constexpr (kLax) acc += F::g(P, x0, y0);
        else acc += F::conj_terms(P, p[0], q[0]);
        bad |= !(M<T>::finite(x0) && M<T>::finite(y0));
      }
      acc = group_sum<L>(acc);
      bad = group_or<L>(bad);
      int st = !fin ? kNonFinite : (small ? kConverged : kMaxIter);
      if (bad || !M<T>::finite(acc)) st = kNonFinite;
      if (l == 0) {
        a.phi[pt] = acc;
        a.iters[pt] = k;
        a.status[pt] = st;
      }
      const int64_t base = pt * int64_t(a.N_max + 1) * a.d;
      if (a.xtraj) {
#pragma unroll
        for (int kk = 0; kk < K; kk++) {
          const int j = 1 + l * K + kk;
          if (j <= Np) {
            a.xtraj[base + j * D] = x[kk];
            a.xtraj[base + j * D + 1] = y[kk];
          }
        }
        if (l == 0) {
          a.xtraj[base] = x0;
          a.xtraj[base + 1] = y0;
        }
      }
      if (a.ptraj) {
#pragma unroll
        for (int kk = 0; kk < K; kk++) {
          const int j = 1 + l * K + kk;
          if (j <= Np) {
            a.ptraj[base + j * D] = p[kk];
            a.ptraj[base + j * D + 1] = q[kk];
          }
        }
        if (l == 0) {
          a.ptraj[base] = T(0);
          a.ptraj[base + 1] = T(0);
        }
      }
      pop_and_init();
    }
    if (__any(done || (active && prio.step(k)))) set_wave_priority(active, k, prio);
  }
}

// ---------------------------------------------------------------------------
// Plain kernel, optimal-control path: one point per lane.
// Workspace arrays X, P, Z, each [N_max+1][D][S] (S = lanes launched).
// One fused sweep per iteration: the dual step of node j+1 (reads the old
// z_j, z_{j+1}) precedes the primal step of node j (writes z_j).
// ---------------------------------------------------------------------------
template <typename T, class F>
__global__ void __launch_bounds__(256) k_plain_control(KArgs<T> a) {
  constexpr int D = F::D;
  const int64_t slot = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t S = a.work_stride;
  const int beg = a.cls_range[2 * a.cls], end = a.cls_range[2 * a.cls + 1];
  if (slot >= S || beg + slot >= end) return;
  const int64_t pt = a.queue[beg + slot];
  typename F::template Par<T> P;
  F::load(P, a.hp, a.gp, a.gkind, a.tau);
  const T sigma = a.sigma, tau = a.tau, theta = a.theta;
  const int Np = a.N[pt];
  const T delta = a.t[pt] / T(Np), sd = sigma * delta, td = tau * delta;
  const int64_t arr = int64_t(a.N_max + 1) * D * S;
  T* WX = a.work;
  T* WP = a.work + arr;
  T* WZ = a.work + 2 * arr;
  auto at = [&](int j, int i) { return (int64_t(j) * D + i) * S + slot; };

  T xt[D];
#pragma unroll
  for (int i = 0; i < D; i++) xt[i] = a.x[pt * a.d + i];
  for (int j = 0; j <= Np; j++) {
#pragma unroll
    for (int i = 0; i < D; i++) {
      // the Hopf formulation has no node 0 (kept at zero)
      const T xv = (j == 0 && a.hopf) ? T(0) : ((j < Np) ? init_x(xt[i], a.seed, pt, kArrX, j, i) : xt[i]);
      WX[at(j, i)] = xv;
      WZ[at(j, i)] = xv;
      WP[at(j, i)] = (j >= 1) ? T(start_noise(a.seed, uint64_t(pt), kArrP, j, i)) : T(0);
    }
  }

  int k = 0, st = kMaxIter;
  for (;;) {
    T rx = T(0), rp = T(0);
    typename F::template Cache<T> Cj, Cn;
    T xj[D], pj[D], xn1[D], pn1[D], zm[D];
    // node 1 dual (uses z_0, z_1 old)
#pragma unroll
    for (int i = 0; i < D; i++) {
      zm[i] = WZ[at(0, i)];
      xj[i] = WX[at(1, i)];
      const T z1 = WZ[at(1, i)];
      const T pold = WP[at(1, i)];
      pj[i] = pold + sigma * (z1 - zm[i]);
      zm[i] = z1;
    }
    {
      T pold[D];
#pragma unroll
      for (int i = 0; i < D; i++) pold[i] = WP[at(1, i)];
      if constexpr (F::kHopf) {
        if (a.hopf) F::dual_hopf1(P, xj, pj, sd, sigma, Cj);
        else F::dual(P, xj, pj, sd, Cj);
      } else {
        F::dual(P, xj, pj, sd, Cj);
      }
#pragma unroll
      for (int i = 0; i < D; i++) {
        const T dp = pj[i] - pold[i];
        rp += dp * dp;
      }
    }
    // node 0 (Lax formulation only)
    if (!a.hopf) {
      T x0[D], v0[D], xn0[D];
#pragma unroll
      for (int i = 0; i < D; i++) {
        x0[i] = WX[at(0, i)];
        v0[i] = x0[i] + tau * pj[i];
      }
      F::prox_g(P, v0, tau, xn0);
#pragma unroll
      for (int i = 0; i < D; i++) {
        const T dx = xn0[i] - x0[i];
        rx += dx * dx;
        WX[at(0, i)] = xn0[i];
        WZ[at(0, i)] = xn0[i] + theta * dx;
      }
    }
    for (int j = 1; j <= Np; j++) {
      // dual step of node j+1 (reads old z_j kept in zm, old z_{j+1})
      if (j < Np) {
        T pold[D];
#pragma unroll
        for (int i = 0; i < D; i++) {
          xn1[i] = WX[at(j + 1, i)];
          const T z1 = WZ[at(j + 1, i)];
          pold[i] = WP[at(j + 1, i)];
          pn1[i] = pold[i] + sigma * (z1 - zm[i]);
          zm[i] = z1;
        }
        F::dual(P, xn1, pn1, sd, Cn);
#pragma unroll
        for (int i = 0; i < D; i++) {
          const T dp = pn1[i] - pold[i];
          rp += dp * dp;
        }
        // primal step of node j
        T g[D];
        F::grad(P, xj, pj, Cj, g);
#pragma unroll
        for (int i = 0; i < D; i++) {
          const T xn = xj[i] - tau * (pj[i] - pn1[i]) + td * g[i];
          const T dx = xn - xj[i];
          rx += dx * dx;
          WX[at(j, i)] = xn;
          WZ[at(j, i)] = xn + theta * dx;
          WP[at(j, i)] = pj[i];
          xj[i] = xn1[i];
          pj[i] = pn1[i];
        }
        Cj = Cn;
      } else {
#pragma unroll
        for (int i = 0; i < D; i++) WP[at(j, i)] = pj[i];
      }
    }
    k++;
    const bool fin = M<T>::finite(rx + rp);
    const bool small = (rx < a.tol) && (rp < a.tol);
    if (!fin) { st = kNonFinite; break; }
    if (!a.fixed && small) { st = kConverged; break; }
    if (k >= a.max_iter) { st = small ? kConverged : kMaxIter; break; }
  }

  // value and outputs
  const int64_t base = pt * int64_t(a.N_max + 1) * a.d;
  T xprev[D], acc = T(0);
  bool ok = true;
#pragma unroll
  for (int i = 0; i < D; i++) {
    xprev[i] = WX[at(0, i)];
    ok = ok && M<T>::finite(xprev[i]);
    if (a.xtraj) a.xtraj[base + i] = xprev[i];
    if (a.ptraj) a.ptraj[base + i] = T(0);
  }
  // Lax: g(x_0); Hopf (node 0 is zero): -g*(p_1)
  if constexpr (F::kHopf) {
    T p1[D];
#pragma unroll
    for (int i = 0; i < D; i++) p1[i] = WP[at(1, i)];
    acc = a.hopf ? -F::gstar(P, p1) : F::g(P, xprev);
  } else {
    acc = F::g(P, xprev);
  }
  for (int j = 1; j <= Np; j++) {
    T xv[D], pv[D], s = T(0);
#pragma unroll
    for (int i = 0; i < D; i++) {
      xv[i] = WX[at(j, i)];
      pv[i] = WP[at(j, i)];
      s += pv[i] * (xv[i] - xprev[i]);
      xprev[i] = xv[i];
      ok = ok && M<T>::finite(xv[i]) && M<T>::finite(pv[i]);
      if (a.xtraj) a.xtraj[base + j * D + i] = xv[i];
      if (a.ptraj) a.ptraj[base + j * D + i] = pv[i];
    }
    acc += s - delta * F::H(P, xv, pv);
  }
  if (!ok || !M<T>::finite(acc)) st = kNonFinite;
  a.phi[pt] = acc;
  a.iters[pt] = k;
  a.status[pt] = st;
}

// ---------------------------------------------------------------------------
// Plain kernel, game path: one point per lane, workspace X, P, Z (DX) and
// Y, Q, W (DY), each [N_max+1][dim][S].
// ---------------------------------------------------------------------------
template <typename T, class F>
__global__ void __launch_bounds__(256) k_plain_game(KArgs<T> a) {
  constexpr int DX = F::DX, DY = F::DY, D = F::D;
  const int64_t slot = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t S = a.work_stride;
  const int beg = a.cls_range[2 * a.cls], end = a.cls_range[2 * a.cls + 1];
  if (slot >= S || beg + slot >= end) return;
  const int64_t pt = a.queue[beg + slot];
  typename F::template Par<T> P;
  F::load(P, a.hp, a.gp, a.gkind, a.tau);
  const T sigma = a.sigma, tau = a.tau, theta = a.theta;
  const int Np = a.N[pt];
  const T delta = a.t[pt] / T(Np), sd = sigma * delta, td = tau * delta;
  T ip, iq;
  F::dual_scales(P, sd, ip, iq);
  const int64_t ax = int64_t(a.N_max + 1) * DX * S, ay = int64_t(a.N_max + 1) * DY * S;
  T* WX = a.work;
  T* WP = WX + ax;
  T* WZ = WP + ax;
  T* WY = WZ + ax;
  T* WQ = WY + ay;
  T* WW = WQ + ay;
  auto ix = [&](int j, int i) { return (int64_t(j) * DX + i) * S + slot; };
  auto iy = [&](int j, int i) { return (int64_t(j) * DY + i) * S + slot; };

  T xt[D];
#pragma unroll
  for (int i = 0; i < D; i++) xt[i] = a.x[pt * a.d + i];
  for (int j = 0; j <= Np; j++) {
#pragma unroll
    for (int i = 0; i < DX; i++) {
      const T v = (j < Np) ? init_x(xt[i], a.seed, pt, kArrX, j, i) : xt[i];
      WX[ix(j, i)] = v;
      WZ[ix(j, i)] = v;
      WP[ix(j, i)] = (j >= 1) ? T(start_noise(a.seed, uint64_t(pt), kArrP, j, i)) : T(0);
    }
#pragma unroll
    for (int i = 0; i < DY; i++) {
      const T v = (j < Np) ? init_x(xt[DX + i], a.seed, pt, kArrY, j, i) : xt[DX + i];
      WY[iy(j, i)] = v;
      WW[iy(j, i)] = v;
      WQ[iy(j, i)] = (j >= 1) ? T(start_noise(a.seed, uint64_t(pt), kArrQ, j, i)) : T(0);
    }
  }

  int k = 0, st = kMaxIter;
  for (;;) {
    T rx = T(0), rp = T(0), ry = T(0), rq = T(0);
    typename F::template CacheX<T> CXj, CXn;
    typename F::template CacheY<T> CYj, CYn;
    T xj[DX], pj[DX], zm[DX], yj[DY], qj[DY], wm[DY];
    T xn1[DX], pn1[DX], yn1[DY], qn1[DY];
    auto dual_node = [&](int jn, T (&xv)[DX], T (&pv)[DX], T (&yv)[DY], T (&qv)[DY],
                         typename F::template CacheX<T>& cx, typename F::template CacheY<T>& cy) {
      T pold[DX], qold[DY];
#pragma unroll
      for (int i = 0; i < DX; i++) {
        xv[i] = WX[ix(jn, i)];
        const T zz = WZ[ix(jn, i)];
        pold[i] = WP[ix(jn, i)];
        pv[i] = pold[i] + sigma * (zz - zm[i]);
        zm[i] = zz;
      }
#pragma unroll
      for (int i = 0; i < DY; i++) {
        yv[i] = WY[iy(jn, i)];
        const T ww = WW[iy(jn, i)];
        qold[i] = WQ[iy(jn, i)];
        qv[i] = qold[i] + sigma * (ww - wm[i]);
        wm[i] = ww;
      }
      F::dual_p(P, xv, pv, sd, ip, cx);
      F::dual_q(P, yv, qv, sd, iq, cy);
#pragma unroll
      for (int i = 0; i < DX; i++) {
        const T d = pv[i] - pold[i];
        rp += d * d;
      }
#pragma unroll
      for (int i = 0; i < DY; i++) {
        const T d = qv[i] - qold[i];
        rq += d * d;
      }
    };
#pragma unroll
    for (int i = 0; i < DX; i++) zm[i] = WZ[ix(0, i)];
#pragma unroll
    for (int i = 0; i < DY; i++) wm[i] = WW[iy(0, i)];
    dual_node(1, xj, pj, yj, qj, CXj, CYj);
    // node 0: x_0 with the old y_0, then y_0 with the new x_0
    {
      T x0[DX], y0[DY], v0[DX], u0[DY], xn0[DX], yn0[DY];
#pragma unroll
      for (int i = 0; i < DX; i++) { x0[i] = WX[ix(0, i)]; v0[i] = x0[i] + tau * pj[i]; }
#pragma unroll
      for (int i = 0; i < DY; i++) { y0[i] = WY[iy(0, i)]; u0[i] = y0[i] + tau * qj[i]; }
      F::prox_x0(P, v0, y0, tau, xn0);
      F::stretch_y0(P, u0, xn0, tau, yn0);
#pragma unroll
      for (int i = 0; i < DX; i++) {
        const T d = xn0[i] - x0[i];
        rx += d * d;
        WX[ix(0, i)] = xn0[i];
        WZ[ix(0, i)] = xn0[i] + theta * d;
      }
#pragma unroll
      for (int i = 0; i < DY; i++) {
        const T d = yn0[i] - y0[i];
        ry += d * d;
        WY[iy(0, i)] = yn0[i];
        WW[iy(0, i)] = yn0[i] + theta * d;
      }
    }
    for (int j = 1; j <= Np; j++) {
      if (j < Np) {
        dual_node(j + 1, xn1, pn1, yn1, qn1, CXn, CYn);
        T gx[DX], gy[DY];
        F::grad_x(P, xj, pj, CXj, gx);
        F::grad_y(P, yj, qj, CYj, gy);
#pragma unroll
        for (int i = 0; i < DX; i++) {
          const T xn = xj[i] - tau * (pj[i] - pn1[i]) + td * gx[i];
          const T d = xn - xj[i];
          rx += d * d;
          WX[ix(j, i)] = xn;
          WZ[ix(j, i)] = xn + theta * d;
          WP[ix(j, i)] = pj[i];
          xj[i] = xn1[i];
          pj[i] = pn1[i];
        }
#pragma unroll
        for (int i = 0; i < DY; i++) {
          const T yn = yj[i] - tau * (qj[i] - qn1[i]) - td * gy[i];
          const T d = yn - yj[i];
          ry += d * d;
          WY[iy(j, i)] = yn;
          WW[iy(j, i)] = yn + theta * d;
          WQ[iy(j, i)] = qj[i];
          yj[i] = yn1[i];
          qj[i] = qn1[i];
        }
        CXj = CXn;
        CYj = CYn;
      } else {
#pragma unroll
        for (int i = 0; i < DX; i++) WP[ix(j, i)] = pj[i];
#pragma unroll
        for (int i = 0; i < DY; i++) WQ[iy(j, i)] = qj[i];
      }
    }
    k++;
    const bool fin = M<T>::finite(rx + rp + ry + rq);
    const bool small = rx < a.tol && rp < a.tol && ry < a.tol && rq < a.tol;
    if (!fin) { st = kNonFinite; break; }
    if (!a.fixed && small) { st = kConverged; break; }
    if (k >= a.max_iter) { st = small ? kConverged : kMaxIter; break; }
  }

  const int64_t base = pt * int64_t(a.N_max + 1) * a.d;
  T xprev[DX], yprev[DY];
  bool ok = true;
#pragma unroll
  for (int i = 0; i < DX; i++) {
    xprev[i] = WX[ix(0, i)];
    ok = ok && M<T>::finite(xprev[i]);
    if (a.xtraj) a.xtraj[base + i] = xprev[i];
  }
#pragma unroll
  for (int i = 0; i < DY; i++) {
    yprev[i] = WY[iy(0, i)];
    ok = ok && M<T>::finite(yprev[i]);
    if (a.xtraj) a.xtraj[base + DX + i] = yprev[i];
  }
  if (a.ptraj)
#pragma unroll
    for (int i = 0; i < D; i++) a.ptraj[base + i] = T(0);
  T acc = F::g(P, xprev, yprev);
  for (int j = 1; j <= Np; j++) {
    T xv[DX], pv[DX], yv[DY], qv[DY], s = T(0);
#pragma unroll
    for (int i = 0; i < DX; i++) {
      xv[i] = WX[ix(j, i)];
      pv[i] = WP[ix(j, i)];
      s += pv[i] * (xv[i] - xprev[i]);
      xprev[i] = xv[i];
      ok = ok && M<T>::finite(xv[i]) && M<T>::finite(pv[i]);
      if (a.xtraj) a.xtraj[base + j * D + i] = xv[i];
      if (a.ptraj) a.ptraj[base + j * D + i] = pv[i];
    }
#pragma unroll
    for (int i = 0; i < DY; i++) {
      yv[i] = WY[iy(j, i)];
      qv[i] = WQ[iy(j, i)];
      s -= qv[i] * (yv[i] - yprev[i]);
      yprev[i] = yv[i];
      ok = ok && M<T>::finite(yv[i]) && M<T>::finite(qv[i]);
      if (a.xtraj) a.xtraj[base + j * D + DX + i] = yv[i];
      if (a.ptraj) a.ptraj[base + j * D + DX + i] = qv[i];
    }
    acc += s - delta * F::H(P, xv, yv, pv, qv);
  }
  if (!ok || !M<T>::finite(acc)) st = kNonFinite;
  a.phi[pt] = acc;
  a.iters[pt] = k;
  a.status[pt] = st;
}

}  // namespace hjpd
