// Linear-tanh family with quadratic initial cost, dense d (differentiation
// workload).  H = -<p, A x + eps tanh x> + |p|^2/2 (paper convention, section
// 2.1), g = x^T Q_s x / 2, Algorithm 1 with:
//   dual   p_j <- (p_j + sigma (z_j - z_{j-1}) + lam (A x_j + eps tanh x_j)) / (1 + lam),
//          lam = sigma delta                                   (closed-form prox)
//   node 0 x_0 <- M (x_0 + tau p_1),  M = (I + tau Q_s)^{-1}
//   primal x_j <- x_j - tau (p_j - p_{j+1}) - tau delta (A^T p_j + eps (1 - tanh^2 x_j) p_j)
//   extrapolation z = x_new + theta (x_new - x_old).
//
// Forward kernel: one point per workgroup of eight wave64s, the stacked state
// X, P, Z [(N+1) x d] in LDS (row stride d+1).  The dense products A X and
// A^T P over all nodes of the point are matrix-core GEMMs
// (v_mfma_f32_16x16x4_f32): wave w owns output row tile w (rows 16w .. 16w+15)
// and keeps those rows of A and A^T as MFMA A-operand fragments in registers
// for the whole kernel; B operands are read from LDS.  Elementwise steps run on
// the VALU in the accumulator layout; the node-0 product with M runs on the
// VALU.  Workgroups are persistent and pop points from a counter.
//
// Reverse mode (hjpd_value_grad): the forward pass stores the state every E
// iterations; the backward kernel, per point, recomputes each segment of E
// iterations from its checkpoint into a per-workgroup buffer (x^k and the new
// multipliers p^{k+1}), then applies the transposed Jacobian of each iteration
// (vector-Jacobian product) from the last iteration down to the first.  The
// VJP's dense products A xbar and A^T vbar reuse the forward fragments; the
// parameter gradient dA = sum of outer products over nodes is an MFMA product
// accumulated in registers; dM and the direct dQ term are rank-1 VALU updates.
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "hjpd_device.hpp"
#include "hjpd_lintanh.hpp"

namespace hjpd {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// tanh from the exponential, tanh|x| = 1 - 2 / (exp(2|x|) + 1), sign restored:
// one hardware exp and one reciprocal; absolute error at FP32 rounding level.
__device__ __forceinline__ float tanh_fast(float x) {
  const float e = __expf(2.f * fabsf(x));
  const float t = 1.f - 2.f * __builtin_amdgcn_rcpf(e + 1.f);
  return copysignf(t, x);
}

constexpr int kLtThreads = 512;
constexpr int kLtWaves = kLtThreads / 64;
constexpr int kLtNT = 4;                                                    // 16-node column tiles: up to 64 nodes

// LDS rows per array: nodes 0 .. 16*NT + 1 (NT column tiles of 16 nodes), so
// every GEMM column read and every j+1 read stays inside the array.
__host__ __device__ constexpr int lt_rows(int N_max) { return 16 * ((N_max + 15) / 16) + 2; }
inline size_t lt_lds_forward(int d, int N_max) { return size_t(3) * lt_rows(N_max) * (d + 1) * sizeof(float); }
inline size_t lt_lds_backward(int d, int N_max) { return size_t(5) * lt_rows(N_max) * (d + 1) * sizeof(float); }
// Per-workgroup reverse-mode buffer (floats): E recomputed steps of (x^k, p^{k+1}) in the LDS layout,
// the saved adjoint (3 arrays), and E staged (XB_0, w) pairs for dM.
__host__ __device__ inline int64_t lt_seg_floats(int d, int N_max, int E) {
  const int64_t CK = int64_t(N_max + 1) * d, RL = int64_t(lt_rows(N_max)) * (d + 1);
  return int64_t(E) * 2 * RL + 3 * CK + int64_t(E) * 2 * d;
}

struct LtArgs {
  const float* x;
  const float* t;
  const int32_t* N;
  const float* hp;  // [eps, A (d*d)]
  const float* Q;   // [d*d]
  const float* M;   // (I + tau Q_s)^{-1}
  float* phi;
  float* xtraj;
  float* ptraj;
  int32_t* iters;
  int32_t* status;
  int32_t* head;
  int64_t n;
  float sigma, tau, theta, tol;
  int max_iter, fixed, N_max;
  uint64_t seed;
  // checkpoints: per point n_ckpt + 1 snapshots of (X, P, Z), each 3 (N_max+1) d;
  // snapshot c holds the state before iteration c E, the last one the final state
  float* ckpt;
  int ckpt_every;
  int n_ckpt;
};

struct LtBwdArgs {
  LtArgs f;
  const float* grad_phi;  // [n]
  float* dphi_dx;         // [n][d]
  float* seg;             // per workgroup: E snapshots of (x^k, p^{k+1}) + adjoint save area
  float* part;            // per workgroup: dA (d*d), dM (d*d), dQ direct (d*d), deps (1)
  int K;
};

// Per-thread constants of the accumulator layout.
template <int D>
struct LtLane {
  static constexpr int KS = D / 4, RT = (D + 15) / 16, LD = D + 1;
  int tid, wave, lr, lk;
  bool has;
  int ic[4];
  bool iok[4];
  __device__ LtLane() {
    tid = threadIdx.x;
    wave = tid >> 6;
    const int lane = tid & 63;
    lr = lane & 15;
    lk = lane >> 4;
    has = wave < RT;
#pragma unroll
    for (int r = 0; r < 4; r++) {
      const int i = 16 * wave + 4 * lk + r;
      iok[r] = has && i < D;
      ic[r] = iok[r] ? i : D;  // rows past d land on the padding column
    }
  }
};

// Reduce a float over the workgroup (all threads get the total).
__device__ __forceinline__ float wg_sum(float v, float* s_red) {
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) v += __shfl_xor(v, m, 64);
  const int wave = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) s_red[wave] = v;
  __syncthreads();
  float t = 0.f;
#pragma unroll
  for (int w = 0; w < kLtWaves; w++) t += s_red[w];
  return t;
}

// acc[c] = rows of this wave x nodes 16c+1 .. 16c+16:  sum_k frag[row][k] B[node][k],
// for all kLtNT column tiles (a fixed count keeps the MFMA chain free of
// branches).  Node rows at or past R (the array's row count) read row R-1,
// which is zero (every array is zero past N); those columns are not used.
template <int D>
__device__ __forceinline__ void gemm_nodes(const float (&frag)[D / 4], const float* sB, const LtLane<D>& L, int R,
                                           f4 (&acc)[kLtNT]) {
  constexpr int LD = D + 1;
  int base[kLtNT];
#pragma unroll
  for (int c = 0; c < kLtNT; c++) {
    const int row = 16 * c + L.lr + 1;
    base[c] = (row < R ? row : R - 1) * LD + L.lk;
    asm volatile("" : "+v"(base[c]));
    acc[c] = f4{0.f, 0.f, 0.f, 0.f};
  }
  // Scheduling fence after every k-step: the scheduler cannot hoist B reads
  // ahead of earlier k-steps' MFMAs (each hoisted read holds a VGPR).  A fence
  // every second or fourth step measured slower in both kernels.
#pragma unroll
  for (int s = 0; s < D / 4; s++) {
#pragma unroll
    for (int c = 0; c < kLtNT; c++) acc[c] = mfma4(frag[s], sB[base[c] + 4 * s], acc[c]);
    __builtin_amdgcn_sched_barrier(0);
  }
}

// out[ct] += sum_{j in [jlo, jhi]} scale U[j][row] V[j][col] for this wave's 16
// rows and column tiles ct (16 columns each): outer products summed over nodes.
template <int D>
__device__ __forceinline__ void gemm_outer(const LtLane<D>& L, const float* sU, const float* sV, float scale, int jlo,
                                           int jhi, f4 (&out)[(D + 15) / 16]) {
  constexpr int LD = D + 1, CT = (D + 15) / 16;
  const int row = 16 * L.wave + L.lr;
  const int rc = (L.has && row < D) ? row : D;
  // two k-steps per trip, all of their LDS reads issued before the products;
  // the second step of the last trip runs only if it has nodes
  for (int j0 = jlo; j0 <= jhi; j0 += 8) {
    float a[2], b[2][CT];
#pragma unroll
    for (int h = 0; h < 2; h++) {
      const int j = j0 + 4 * h + L.lk;
      const bool ok = j <= jhi;
      const int jr = ok ? j : jlo;
      a[h] = ok ? scale * sU[jr * LD + rc] : 0.f;
#pragma unroll
      for (int ct = 0; ct < CT; ct++) {
        const int col = 16 * ct + L.lr;
        b[h][ct] = sV[jr * LD + (col < D ? col : D)];
      }
    }
#pragma unroll
    for (int ct = 0; ct < CT; ct++) out[ct] = mfma4(a[0], b[0][ct], out[ct]);
    if (j0 + 4 <= jhi) {
#pragma unroll
      for (int ct = 0; ct < CT; ct++) out[ct] = mfma4(a[1], b[1][ct], out[ct]);
    }
  }
}

// One iteration of the splitting (dual, node 0, primal, extrapolation) on the
// LDS state.  If sx_out / sp_out are given, x^k (before the iteration) and
// p^{k+1} (after the dual step) are stored there ([N+1][d], row stride d).
// Adds this thread's partial residual sums to rx, rp.
template <int D, bool kReuseTanh = false>
__device__ void lt_iterate(const LtLane<D>& L, const LtArgs& a, const float (&af)[D / 4], const float (&atf)[D / 4],
                           float* sX, float* sP, float* sZ, int Np, int NT, float delta, float eps, float* sx_out,
                           float* sp_out, float& rx, float& rp) {
  constexpr int LD = D + 1;
  const int R = lt_rows(a.N_max);
  const float sigma = a.sigma, tau = a.tau, theta = a.theta;
  const float lam = sigma * delta, c1 = 1.f / (1.f + lam), td = tau * delta;
  int lo = (L.lr + 1) * LD;
  asm volatile("" : "+v"(lo));
  if (sx_out)
    for (int e = L.tid; e < (Np + 1) * LD; e += kLtThreads) sx_out[e] = sX[e];
  // ---- dual step: p_j <- (p_j + sigma (z_j - z_{j-1}) + lam f_j) c1 ----------
  f4 acc[kLtNT];
  // With kReuseTanh the dual step keeps tanh(x_j) for the primal step (x is
  // unchanged until then): faster in the reverse sweep's recompute, slower in
  // the forward kernel, whose 128 registers then spill more.
  f4 thc[kLtNT];
  gemm_nodes<D>(af, sX, L, R, acc);
#pragma unroll
  for (int c = 0; c < kLtNT; c++) {
    thc[c] = f4{0.f, 0.f, 0.f, 0.f};
    if (c >= NT) continue;
    const int j = 16 * c + L.lr + 1;
#pragma unroll
    for (int r = 0; r < 4; r++) {
      const bool ok = L.iok[r] && j <= Np;
      const int e = lo + 16 * c * LD + L.ic[r];
      const float xv = sX[e], pv = sP[e];
      const float v = pv + sigma * (sZ[e] - sZ[e - LD]);
      const float thd = tanh_fast(xv);
      if constexpr (kReuseTanh) thc[c][r] = thd;
      const float f = acc[c][r] + eps * thd;
      const float pn = (v + lam * f) * c1;
      const float dp = pn - pv;
      rp += ok ? dp * dp : 0.f;
      sP[e] = ok ? pn : pv;
    }
  }
  __syncthreads();
  if (sp_out)
    for (int e = L.tid; e < (Np + 1) * LD; e += kLtThreads) sp_out[e] = sP[e];
  // ---- node 0 (VALU): x_0 <- M (x_0 + tau p_1), M symmetric, read by columns.
  // The four lanes of a quad share output i = tid / 4, each summing a quarter
  // of its terms, and add the quarters with two quad exchanges (the forward
  // kernel and the reverse kernel's recompute use this same summation order,
  // so the recompute reproduces the forward bit for bit).
  float x0n = 0.f, z0n = 0.f;
  const int i0 = L.tid >> 2, q0 = L.tid & 3;
  // With d up to 112, half of M's terms are loaded before the primal product
  // and the rest after it, and all are summed after it, so part of their
  // latency overlaps the product (loading all of them first spills registers);
  // at d = 128 that measured slower, and the sum runs before the product.
  constexpr int KQ = (D + 3) / 4;
  if constexpr (D <= 112) {
    // Quads past row d load row d - 1 and discard the sum.  The opaque column
    // keeps the loads in the iteration.
    int col = i0 < D ? i0 : D - 1;
    asm volatile("" : "+v"(col));
    constexpr int KP = KQ / 2;  // terms loaded ahead of the product
    float mv[KQ];
#pragma unroll
    for (int s = 0; s < KP; s++) {
      const int kq = q0 * KQ + s;
      mv[s] = (4 * KQ == D || kq < D) ? a.M[kq * D + col] : 0.f;
    }
    // ---- primal step, j = 1..N-1, with G = A^T P: the product ---------------------
    gemm_nodes<D>(atf, sP, L, R, acc);
#pragma unroll
    for (int s = KP; s < KQ; s++) {
      const int kq = q0 * KQ + s;
      mv[s] = (4 * KQ == D || kq < D) ? a.M[kq * D + col] : 0.f;
    }
    float part = 0.f;
#pragma unroll
    for (int s = 0; s < KQ; s++) {
      const int kq = q0 * KQ + s;
      if (4 * KQ == D || kq < D) part += mv[s] * (sX[kq] + tau * sP[LD + kq]);
    }
    part += dpp_f<kDppQuad1032>(part);
    part += dpp_f<kDppQuad2301>(part);
    if (i0 < D && q0 == 0) {
      const float old = sX[i0];
      const float dx = part - old;
      rx += dx * dx;
      x0n = part;
      z0n = part + theta * dx;
    }
  } else {
    // opaque column index: the loop-invariant loads of M stay in the iteration
    int col = i0;
    asm volatile("" : "+v"(col));
    float part = 0.f;
    if (i0 < D) {
#pragma unroll
      for (int s = 0; s < KQ; s++) {
        const int kq = q0 * KQ + s;
        if (kq < D) part += a.M[kq * D + col] * (sX[kq] + tau * sP[LD + kq]);
      }
    }
    part += dpp_f<kDppQuad1032>(part);
    part += dpp_f<kDppQuad2301>(part);
    if (i0 < D && q0 == 0) {
      const float old = sX[i0];
      const float dx = part - old;
      rx += dx * dx;
      x0n = part;
      z0n = part + theta * dx;
    }
    // ---- primal step, j = 1..N-1, with G = A^T P: the product ---------------------
    gemm_nodes<D>(atf, sP, L, R, acc);
  }
  // ---- primal step: the update ----------------------------------------------------
#pragma unroll
  for (int c = 0; c < kLtNT; c++) {
    if (c >= NT) continue;
    const int j = 16 * c + L.lr + 1;
#pragma unroll
    for (int r = 0; r < 4; r++) {
      const bool ok = L.iok[r] && j <= Np - 1;
      const int e = lo + 16 * c * LD + L.ic[r];
      const float xv = sX[e], pv = sP[e], pp = sP[e + LD], zv = sZ[e];
      const float th = kReuseTanh ? thc[c][r] : tanh_fast(xv);
      const float gx = acc[c][r] + eps * (1.f - th * th) * pv;  // -grad_x H
      const float xn = xv - tau * (pv - pp) - td * gx;
      const float dx = xn - xv;
      rx += ok ? dx * dx : 0.f;
      sZ[e] = ok ? xn + theta * dx : zv;
      sX[e] = ok ? xn : xv;
    }
  }
  __syncthreads();
  if (i0 < D && q0 == 0) {
    sX[i0] = x0n;
    sZ[i0] = z0n;
  }
  __syncthreads();
}

// Random start (section 6 set-up) into LDS; rows past N and the padding column zero.
template <int D>
__device__ void lt_init(const LtArgs& a, int64_t pt, int Np, int R, float* sX, float* sP, float* sZ) {
  constexpr int LD = D + 1;
  for (int e = threadIdx.x; e < R * LD; e += kLtThreads) {
    const int j = e / LD, i = e - j * LD;
    float xv = 0.f, pv = 0.f;
    if (j <= Np && i < D) {
      const float xt = a.x[pt * D + i];
      xv = (j < Np) ? float(double(xt) + start_noise(a.seed, uint64_t(pt), kArrX, j, i)) : xt;
      pv = (j >= 1) ? float(start_noise(a.seed, uint64_t(pt), kArrP, j, i)) : 0.f;
    }
    sX[e] = xv;
    sZ[e] = xv;
    sP[e] = pv;
  }
  __syncthreads();
}

// Copy LDS arrays (row stride d+1) to a compact global snapshot (row stride d).
template <int D>
__device__ void lt_save(const float* sX, const float* sP, const float* sZ, int Np, int N_max, float* dst) {
  constexpr int LD = D + 1;
  const int64_t CK = int64_t(N_max + 1) * D;
  for (int e = threadIdx.x; e < (Np + 1) * D; e += kLtThreads) {
    const int j = e / D, i = e - j * D;
    dst[e] = sX[j * LD + i];
    dst[CK + e] = sP[j * LD + i];
    dst[2 * CK + e] = sZ[j * LD + i];
  }
  __syncthreads();
}

// Load up to three consecutive snapshot arrays into LDS (zero past N and in the
// padding column); null targets are skipped.  The loads of one array are
// issued together before their LDS stores (one memory latency per array and
// call, not one per element).
template <int D>
__device__ void lt_load(float* s0, float* s1, float* s2, int Np, int N_max, int R, const float* src) {
  constexpr int LD = D + 1;
  constexpr int NL = (lt_rows(kLtMaxN) * LD + kLtThreads - 1) / kLtThreads;
  const int64_t CK = int64_t(N_max + 1) * D;
  float* dst[3] = {s0, s1, s2};
  // opaque thread index: the per-element row/column divisions below are
  // recomputed per call instead of being hoisted and held for the kernel
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
#pragma unroll
  for (int q = 0; q < 3; q++) {
    if (!dst[q]) continue;
    const float* sq = src + q * CK;
    float v[NL];
#pragma unroll
    for (int u = 0; u < NL; u++) {
      const int e = tid + u * kLtThreads;
      const int j = e / LD, i = e - j * LD;
      const bool ok = e < R * LD && j <= Np && i < D;
      v[u] = ok ? sq[j * D + i] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < NL; u++) {
      const int e = tid + u * kLtThreads;
      if (e < R * LD) dst[q][e] = v[u];
    }
  }
  __syncthreads();
}

// Rows 0..N of two arrays stored in the LDS layout (src, src + RL), read into
// registers by lt_rows_load and written to LDS by lt_rows_store; rows past N
// already hold zero there.  Every thread issues its loads together and no
// branch guards them: indices past row N are clamped to the last entry of row
// N, which those threads then write with its own value.
template <int D>
constexpr int lt_rows_per_thread() { return (lt_rows(kLtMaxN) * (D + 1) + kLtThreads - 1) / kLtThreads; }

template <int D>
__device__ __forceinline__ void lt_rows_load(const float* src, int64_t RL, int Np, float (&v)[2][lt_rows_per_thread<D>()]) {
  constexpr int NL = lt_rows_per_thread<D>();
  const int last = (Np + 1) * (D + 1) - 1;
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
#pragma unroll
  for (int q = 0; q < 2; q++)
#pragma unroll
    for (int u = 0; u < NL; u++) v[q][u] = src[q * RL + min(tid + u * kLtThreads, last)];
}

template <int D>
__device__ __forceinline__ void lt_rows_store(float* s0, float* s1, int Np, const float (&v)[2][lt_rows_per_thread<D>()]) {
  constexpr int NL = lt_rows_per_thread<D>();
  const int last = (Np + 1) * (D + 1) - 1;
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
#pragma unroll
  for (int u = 0; u < NL; u++) {
    const int e = min(tid + u * kLtThreads, last);
    s0[e] = v[0][u];
    s1[e] = v[1][u];
  }
}

template <int D>
__device__ bool lt_bad_input(const LtArgs& a, int64_t pt) {
  const int Np = a.N[pt];
  const float tt = a.t[pt];
  bool bad = !(tt > 0.f) || !__builtin_isfinite(tt) || Np < 1 || Np > a.N_max;
  for (int i = 0; i < D && !bad; i++) bad = !__builtin_isfinite(a.x[pt * D + i]);
  return bad;
}

template <int D>
__device__ void lt_load_fragments(const float* A, int wave, int lr, int lk, float (&af)[D / 4], float (&atf)[D / 4]) {
  const int row = 16 * wave + lr;
#pragma unroll
  for (int s = 0; s < D / 4; s++) {
    const int k = 4 * s + lk;
    af[s] = row < D ? A[row * D + k] : 0.f;
    atf[s] = row < D ? A[k * D + row] : 0.f;
  }
}

template <int D>
__global__ void __launch_bounds__(kLtThreads, 4) k_lt_forward(LtArgs a) {
  static_assert(D % 4 == 0, "d must be a multiple of 4");
  constexpr int LD = D + 1;
  extern __shared__ float smem[];
  __shared__ float s_red[2 * kLtWaves];
  __shared__ int s_pt;
  const LtLane<D> L;
  const int R = lt_rows(a.N_max);
  const int NT = (a.N_max + 15) / 16;
  float* sX = smem;
  float* sP = sX + R * LD;
  float* sZ = sP + R * LD;
  const float eps = a.hp[0];
  float af[D / 4], atf[D / 4];
  lt_load_fragments<D>(a.hp + 1, L.wave, L.lr, L.lk, af, atf);

  for (;;) {
    if (L.tid == 0) s_pt = atomicAdd(a.head, 1);
    __syncthreads();
    const int64_t pt = s_pt;
    __syncthreads();
    if (pt >= a.n) break;
    if (lt_bad_input<D>(a, pt)) {
      if (L.tid == 0) {
        if (a.phi) a.phi[pt] = NAN;
        a.iters[pt] = 0;
        a.status[pt] = kBadInput;
      }
      continue;
    }
    const int Np = a.N[pt];
    const float delta = a.t[pt] / float(Np);
    lt_init<D>(a, pt, Np, R, sX, sP, sZ);
    const int64_t slot = 3 * int64_t(a.N_max + 1) * D;
    int k = 0, st = kMaxIter;
    for (;;) {
      if (a.ckpt && k % a.ckpt_every == 0 && k / a.ckpt_every < a.n_ckpt)
        lt_save<D>(sX, sP, sZ, Np, a.N_max, a.ckpt + (pt * (a.n_ckpt + 1) + k / a.ckpt_every) * slot);
      const bool need_res = !a.fixed || k + 1 >= a.max_iter;
      float rx = 0.f, rp = 0.f;
      lt_iterate<D>(L, a, af, atf, sX, sP, sZ, Np, NT, delta, eps, nullptr, nullptr, rx, rp);
      k++;
      bool done = k >= a.max_iter;
      if (need_res) {
        const float rxs = wg_sum(rx, s_red);
        const float rps = wg_sum(rp, s_red + kLtWaves);
        const bool fin = __builtin_isfinite(rxs + rps);
        const bool small = rxs < a.tol && rps < a.tol;
        if (!fin) {
          st = kNonFinite;
          done = true;
        } else if (small && (!a.fixed || done)) {
          st = kConverged;
          done = true;
        }
      }
      if (done) break;
    }
    if (a.ckpt) lt_save<D>(sX, sP, sZ, Np, a.N_max, a.ckpt + (pt * (a.n_ckpt + 1) + a.n_ckpt) * slot);

    // ---- value: g(x_0) + sum <p_j, x_j - x_{j-1}> - delta sum H(x_j, p_j) ----------
    int lo = (L.lr + 1) * LD;
    asm volatile("" : "+v"(lo));
    f4 acc[kLtNT];
    gemm_nodes<D>(af, sX, L, R, acc);
    float val = 0.f, badf = 0.f;
#pragma unroll
    for (int c = 0; c < kLtNT; c++) {
      if (c >= NT) continue;
      const int j = 16 * c + L.lr + 1;
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const bool ok = L.iok[r] && j <= Np;
        const int e = lo + 16 * c * LD + L.ic[r];
        const float xv = sX[e], pv = sP[e], xm = sX[e - LD];
        const float f = acc[c][r] + eps * tanh_fast(xv);
        const float term = pv * (xv - xm) - delta * (0.5f * pv * pv - pv * f);
        val += ok ? term : 0.f;
        badf += (ok && !(__builtin_isfinite(xv) && __builtin_isfinite(pv))) ? 1.f : 0.f;
      }
    }
    if (L.tid < D) {
      float qx = 0.f;
      for (int kq = 0; kq < D; kq++) qx += 0.5f * (a.Q[L.tid * D + kq] + a.Q[kq * D + L.tid]) * sX[kq];
      val += 0.5f * sX[L.tid] * qx;
      if (!__builtin_isfinite(sX[L.tid])) badf = 1.f;
    }
    val = wg_sum(val, s_red);
    badf = wg_sum(badf, s_red + kLtWaves);
    if (badf > 0.f || !__builtin_isfinite(val)) st = kNonFinite;
    if (L.tid == 0) {
      if (a.phi) a.phi[pt] = val;
      a.iters[pt] = k;
      a.status[pt] = st;
    }
    if (a.xtraj || a.ptraj) {
      const int64_t base = pt * int64_t(a.N_max + 1) * D;
      for (int e = L.tid; e < (Np + 1) * D; e += kLtThreads) {
        const int j = e / D, i = e - j * D;
        if (a.xtraj) a.xtraj[base + e] = sX[j * LD + i];
        if (a.ptraj) a.ptraj[base + e] = sP[j * LD + i];
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Reverse sweep.  Adjoint arrays XB, PB, ZB (of x, p, z after an iteration)
// live in LDS; per iteration k (from K-1 down to 0), with x^k in S0 and
// p^{k+1} in S1, the transposed Jacobian of the iteration is applied:
//   z' = x' + theta (x' - x)        XB += (1+theta) ZB;  Xpre = -theta ZB   (z'_N = x_N: Xpre_N = ZB_N + XB_N)
//   x'_0 = M w, w = x_0 + tau p'_1  wbar = M XB_0;  Xpre_0 += wbar;  PB_1 += tau wbar;  dM += XB_0 w^T
//   x'_j = x_j - tau (p'_j - p'_{j+1}) - tau delta (A^T p'_j + eps (1 - th_j^2) p'_j),  j < N:
//        Xpre_j += XB_j + 2 tau delta eps (1 - th_j^2) th_j p'_j XB_j
//        PB_j += -tau XB_j - tau delta (A XB)_j - tau delta eps (1 - th_j^2) XB_j + tau XB_{j-1}
//        dA += -tau delta p'_j XB_j^T;  deps += -tau delta sum (1 - th^2) p' XB
//   p'_j = c1 (p_j + sigma (z_j - z_{j-1}) + lam (A x_j + eps th_j)):
//        vbar = c1 PB;  Ppre = vbar;  Zpre_j = sigma (vbar_j - vbar_{j+1})
//        Xpre_j += lam (A^T vbar)_j + lam eps (1 - th_j^2) vbar_j;  dA += lam vbar_j x_j^T;  deps += lam th vbar
// ---------------------------------------------------------------------------
template <int D>
__global__ void __launch_bounds__(kLtThreads, 2) k_lt_backward(LtBwdArgs b) {
  constexpr int LD = D + 1, CT = (D + 15) / 16;
  const LtArgs& a = b.f;
  extern __shared__ float smem[];
  __shared__ float s_red[2 * kLtWaves];
  __shared__ float s_wb[4 * 128];  // wbar = M XB_0 (B1): whole sums, or quarters when no wave is idle
  constexpr int kIdleWaves = kLtWaves - (D + 15) / 16;  // waves with no row tile of their own
  auto wbar = [&](int i) {
    if constexpr (kIdleWaves > 0) return s_wb[i];
    else return (s_wb[i] + s_wb[128 + i]) + (s_wb[256 + i] + s_wb[384 + i]);
  };
  const LtLane<D> L;
  const int R = lt_rows(a.N_max);
  const int NT = (a.N_max + 15) / 16;
  float* S0 = smem;
  float* S1 = S0 + R * LD;
  float* S2 = S1 + R * LD;
  float* S3 = S2 + R * LD;
  float* S4 = S3 + R * LD;
  const float eps = a.hp[0];
  const float sigma = a.sigma, tau = a.tau, theta = a.theta;
  float af[D / 4], atf[D / 4];
  lt_load_fragments<D>(a.hp + 1, L.wave, L.lr, L.lk, af, atf);
  f4 dA[CT];
#pragma unroll
  for (int ct = 0; ct < CT; ct++) dA[ct] = f4{0.f, 0.f, 0.f, 0.f};
  float deps = 0.f;
  // dM and the direct dQ term accumulate in this workgroup's partial block in
  // global memory, in the accumulator layout (wave rows x column tiles), so no
  // per-thread d*d/threads arrays or index divisions stay live in registers.
  const int64_t DD = int64_t(D) * D;
  float* part = b.part + int64_t(blockIdx.x) * (3 * DD + 1);
#pragma unroll
  for (int ct = 0; ct < CT; ct++)
#pragma unroll
    for (int r = 0; r < 4; r++) {
      const int row = 16 * L.wave + 4 * L.lk + r, col = 16 * ct + L.lr;
      if (L.has && row < D && col < D) {
        part[DD + row * D + col] = 0.f;
        part[2 * DD + row * D + col] = 0.f;
      }
    }

  const int E = a.ckpt_every;
  const int64_t CK = int64_t(a.N_max + 1) * D;
  const int64_t slot = 3 * CK;
  const int64_t RL = int64_t(R) * LD;  // a recomputed x^k or p^{k+1}, in the LDS layout
  float* segx = b.seg + int64_t(blockIdx.x) * lt_seg_floats(D, a.N_max, E);
  float* adjsave = segx + int64_t(E) * 2 * RL;
  float* stage = adjsave + 3 * CK;  // per step of a segment: XB_0 (node-0 adjoint) and w = x_0 + tau p'_1

  // Points are dealt to the workgroups in a fixed order (every point costs
  // the same K iterations), so each workgroup's partial sums of dA, dM, dQ and
  // deps, and with them the gradients, are the same from call to call.
  for (int64_t pt = blockIdx.x; pt < a.n; pt += gridDim.x) {
    const float w = b.grad_phi[pt];
    if (lt_bad_input<D>(a, pt) || w == 0.f) {
      for (int i = L.tid; i < D; i += kLtThreads) b.dphi_dx[pt * D + i] = 0.f;
      continue;
    }
    const int Np = a.N[pt];
    const float delta = a.t[pt] / float(Np), lam = sigma * delta, c1 = 1.f / (1.f + lam), td = tau * delta;
    const float* ck_pt = a.ckpt + pt * (a.n_ckpt + 1) * slot;

    // ---- adjoint of the value at the final iterate ---------------------------------
    float* XB = S2;
    float* PB = S3;
    float* ZB = S4;
    lt_load<D>(S0, S1, nullptr, Np, a.N_max, R, ck_pt + a.n_ckpt * slot);
    {
      int lo = (L.lr + 1) * LD;
      asm volatile("" : "+v"(lo));
      f4 ax[kLtNT], atp[kLtNT];
      gemm_nodes<D>(af, S0, L, R, ax);
      gemm_nodes<D>(atf, S1, L, R, atp);
      for (int e = L.tid; e < R * LD; e += kLtThreads) {
        XB[e] = 0.f;
        PB[e] = 0.f;
        ZB[e] = 0.f;
      }
      __syncthreads();
#pragma unroll
      for (int c = 0; c < kLtNT; c++) {
        if (c >= NT) continue;
        const int j = 16 * c + L.lr + 1;
#pragma unroll
        for (int r = 0; r < 4; r++) {
          const bool ok = L.iok[r] && j <= Np;
          const int e = lo + 16 * c * LD + L.ic[r];
          const float xv = S0[e], pv = S1[e], xm = S0[e - LD];
          const float pn = (j < Np) ? S1[e + LD] : 0.f;
          const float th = tanh_fast(xv);
          const float gx = pv - pn + delta * (atp[c][r] + eps * (1.f - th * th) * pv);
          const float gp = xv - xm + delta * (ax[c][r] + eps * th - pv);
          if (ok) {
            XB[e] = w * gx;
            PB[e] = w * gp;
          }
          deps += ok ? w * delta * pv * th : 0.f;
        }
      }
      if (L.tid < D) {
        float qx = 0.f;
        for (int kq = 0; kq < D; kq++) qx += 0.5f * (a.Q[L.tid * D + kq] + a.Q[kq * D + L.tid]) * S0[kq];
        XB[L.tid] = w * (qx - S1[LD + L.tid]);
      }
      // dQ (direct) += w x_0 x_0^T / 2 ; dA += w delta sum_j p_j x_j^T
      {
        // opaque per-lane base: keeps the 28 addresses from being hoisted
        // out of the point loop (and held in registers for the whole kernel)
        int rb = 16 * L.wave + 4 * L.lk;
        asm volatile("" : "+v"(rb));
        float* pq = part + 2 * DD + int64_t(rb) * D + L.lr;
#pragma unroll
        for (int ct = 0; ct < CT; ct++)
#pragma unroll
          for (int r = 0; r < 4; r++) {
            const int row = rb + r, col = 16 * ct + L.lr;
            if (L.has && row < D && col < D) pq[r * D + 16 * ct] += 0.5f * w * S0[row] * S0[col];
          }
      }
      gemm_outer<D>(L, S1, S0, w * delta, 1, Np, dA);
      __syncthreads();
    }

    // ---- segments, last to first ------------------------------------------------------
    const int nseg = (b.K + E - 1) / E;
    for (int sg = nseg - 1; sg >= 0; sg--) {
      const int k0 = sg * E, k1 = min(b.K, k0 + E);
      // save the adjoint, recompute the segment forward from its checkpoint
      lt_save<D>(XB, PB, ZB, Np, a.N_max, adjsave);
      lt_load<D>(S0, S1, S2, Np, a.N_max, R, ck_pt + sg * slot);
      for (int k = k0; k < k1; k++) {
        float rx = 0.f, rp = 0.f;
        float* so = segx + int64_t(k - k0) * 2 * RL;
        lt_iterate<D, true>(L, a, af, atf, S0, S1, S2, Np, NT, delta, eps, so, so + RL, rx, rp);
      }
      XB = S2;
      PB = S3;
      ZB = S4;
      lt_load<D>(XB, PB, ZB, Np, a.N_max, R, adjsave);
      // reverse sweep through the segment
      // x^k and p^{k+1} of each step are loaded into registers during the
      // previous step's last outer product and written to LDS at the step's
      // start (read after the barrier that ends (A))
      float rows[2][lt_rows_per_thread<D>()];
      lt_rows_load<D>(segx + int64_t(k1 - 1 - k0) * 2 * RL, RL, Np, rows);
      for (int k = k1 - 1; k >= k0; k--) {
        lt_rows_store<D>(S0, S1, Np, rows);
        int lo = (L.lr + 1) * LD;
        asm volatile("" : "+v"(lo));
        // (A) extrapolation
        // branch-free: the padding column holds zero in both arrays and stays
        // zero (0 - theta * 0 = +0), row N's x-adjoint is written back unchanged
        for (int e = L.tid; e < (Np + 1) * LD; e += kLtThreads) {
          const int j = e / LD;
          const float zb = ZB[e], xb = XB[e];
          const bool mid = j < Np;
          XB[e] = mid ? xb + (1.f + theta) * zb : xb;
          ZB[e] = mid ? 0.f - theta * zb : zb + xb;
        }
        __syncthreads();
        f4 thk[kLtNT];  // tanh(x_j^k): formed in (B2), used again in (C2)
#pragma unroll
        for (int c = 0; c < kLtNT; c++) thk[c] = f4{0.f, 0.f, 0.f, 0.f};
        // (B1) node 0: w = x_0 + tau p'_1, wbar = M XB_0; dM += XB_0 w^T is
        // applied once per segment from the staged (XB_0, w) pairs.  With fewer
        // row tiles than waves, the waves past the last tile (whose product
        // tiles are padding) form wbar, one thread per output summing its terms
        // in order, and stage the pair while the others run (B2)'s product
        // A XB; otherwise the eight waves first sum quarters of each row's terms.
        float* st = stage + int64_t(k - k0) * 2 * D;
        f4 acc[kLtNT];
        if constexpr (kIdleWaves > 0) {
          if (L.has) {
            gemm_nodes<D>(af, XB, L, R, acc);  // (A XB)_j
          } else {
#pragma unroll
            for (int c = 0; c < kLtNT; c++) acc[c] = f4{0.f, 0.f, 0.f, 0.f};
            // the terms' loads are issued W at a time ahead of their products;
            // the opaque column keeps M's loads inside the step
            constexpr int W = D % 25 == 0 ? 25 : (D % 16 == 0 ? 16 : (D % 8 == 0 ? 8 : 4));
            for (int i = L.tid - 64 * L.RT; i < D; i += 64 * kIdleWaves) {
              int col = i;
              asm volatile("" : "+v"(col));
              float part = 0.f;
              for (int s0 = 0; s0 < D; s0 += W) {
                float mv[W], xv[W];
#pragma unroll
                for (int h = 0; h < W; h++) {
                  mv[h] = a.M[(s0 + h) * D + col];
                  xv[h] = XB[s0 + h];
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int h = 0; h < W; h++) part += mv[h] * xv[h];
              }
              s_wb[i] = part;
              st[i] = XB[i];
              st[D + i] = S0[i] + tau * S1[LD + i];
            }
          }
          __syncthreads();
        } else {
          const int i = L.tid & 127, g = L.tid >> 7;
          if (i < D) {
            constexpr int KQ = (D + 3) / 4;
            // W terms per trip, their loads issued together ahead of the
            // products (g < 4, so with d a multiple of 4 every term exists and
            // no branch guards a load); the opaque column keeps M's loads
            // inside the step
            constexpr int W = KQ % 5 == 0 ? 5 : (KQ % 4 == 0 ? 4 : 1);
            int col = i;
            asm volatile("" : "+v"(col));
            float part = 0.f;
            for (int s0 = 0; s0 < KQ; s0 += W) {
              float mv[W], xv[W];
#pragma unroll
              for (int h = 0; h < W; h++) {
                const int kq = g * KQ + s0 + h;
                const bool ok = 4 * KQ == D || kq < D;
                mv[h] = ok ? a.M[kq * D + col] : 0.f;
                xv[h] = ok ? XB[kq] : 0.f;
              }
              __builtin_amdgcn_sched_barrier(0);
#pragma unroll
              for (int h = 0; h < W; h++) part += mv[h] * xv[h];
            }
            s_wb[g * 128 + i] = part;
          }
          if (L.tid < D) {
            st[L.tid] = XB[L.tid];
            st[D + L.tid] = S0[L.tid] + tau * S1[LD + L.tid];
          }
          __syncthreads();
          gemm_nodes<D>(af, XB, L, R, acc);  // (A XB)_j
        }
        if (L.tid < D) ZB[L.tid] += wbar(L.tid);
        // (B2) primal step transposed
        {
#pragma unroll
          for (int c = 0; c < kLtNT; c++) {
            if (c >= NT) continue;
            const int j = 16 * c + L.lr + 1;
#pragma unroll
            for (int r = 0; r < 4; r++) {
              const bool ok = L.iok[r] && j <= Np;
              const bool prim = j <= Np - 1;
              const int e = lo + 16 * c * LD + L.ic[r];
              const float xb = prim ? XB[e] : 0.f;
              const float xbm = (j >= 2) ? XB[e - LD] : 0.f;
              const float pp = S1[e], xk = S0[e];
              const float th = tanh_fast(xk), om = 1.f - th * th;
              thk[c][r] = th;
              // x_N is fixed: no primal step and no (A XB)_N term at j = N
              float pbd = -tau * xb - (prim ? td * acc[c][r] : 0.f) - td * eps * om * xb + tau * xbm;
              if (j == 1) pbd += tau * wbar(L.ic[r] < D ? L.ic[r] : 0);
              // entries that do not move are written back unchanged (no branch)
              const float pbo = PB[e], zbo = ZB[e];
              PB[e] = ok ? (pbo + pbd) * c1 : pbo;  // with (C1) vbar = c1 PB folded in
              ZB[e] = ok ? zbo + (xb + 2.f * td * eps * om * th * pp * xb) : zbo;
              deps += (ok && prim) ? -td * om * pp * xb : 0.f;
            }
          }
          gemm_outer<D>(L, S1, XB, -td, 1, Np - 1, dA);
        }
        __syncthreads();
        // (C1) vbar = c1 PB: applied above where (B2) writes PB (every entry
        // of nodes 1..N is written there once; node 0's row and the padding
        // column stay 0)
        // (C2) dual step transposed; Zpre into the XB array
        {
          f4 acc[kLtNT];
          gemm_nodes<D>(atf, PB, L, R, acc);  // (A^T vbar)_j
#pragma unroll
          for (int c = 0; c < kLtNT; c++) {
            if (c >= NT) continue;
            const int j = 16 * c + L.lr + 1;
#pragma unroll
            for (int r = 0; r < 4; r++) {
              const bool ok = L.iok[r] && j <= Np;
              const int e = lo + 16 * c * LD + L.ic[r];
              const float vb = PB[e], vbn = (j < Np) ? PB[e + LD] : 0.f;
              const float th = thk[c][r];
              // entries past N and in the padding column hold zero in every array
              const float zbo = ZB[e];
              ZB[e] = ok ? zbo + (lam * acc[c][r] + lam * eps * (1.f - th * th) * vb) : zbo;
              XB[e] = ok ? sigma * (vb - vbn) : 0.f;
              deps += ok ? lam * th * vb : 0.f;
            }
          }
          if (L.tid < D) XB[L.tid] = -sigma * PB[LD + L.tid];
          if (k > k0) lt_rows_load<D>(segx + int64_t(k - 1 - k0) * 2 * RL, RL, Np, rows);
          gemm_outer<D>(L, PB, S0, lam, 1, Np, dA);
        }
        __syncthreads();
        // (D) roles: x-adjoint <- Xpre (ZB array), z-adjoint <- Zpre (XB array)
        float* tmp = XB;
        XB = ZB;
        ZB = tmp;
      }
      // dM += sum over the segment's steps of XB_0 w^T: one matrix-core outer
      // product over the staged rows (S0, S1 are free until the next segment)
      __syncthreads();
      for (int r0 = 0; r0 < k1 - k0; r0 += R) {
        const int nr = min(R, k1 - k0 - r0);
        for (int e = L.tid; e < R * LD; e += kLtThreads) {
          const int j = e / LD, i = e - j * LD;
          const bool ok = j < nr && i < D;
          const float* st = stage + int64_t(r0 + j) * 2 * D;
          S0[e] = ok ? st[i] : 0.f;
          S1[e] = ok ? st[D + i] : 0.f;
        }
        __syncthreads();
        int rb = 16 * L.wave + 4 * L.lk;
        asm volatile("" : "+v"(rb));
        float* pm = part + DD + int64_t(rb) * D + L.lr;
        f4 dMf[CT];
#pragma unroll
        for (int ct = 0; ct < CT; ct++)
#pragma unroll
          for (int r = 0; r < 4; r++) {
            const int row = rb + r, col = 16 * ct + L.lr;
            dMf[ct][r] = (L.has && row < D && col < D) ? pm[r * D + 16 * ct] : 0.f;
          }
        gemm_outer<D>(L, S0, S1, 1.f, 0, nr - 1, dMf);
#pragma unroll
        for (int ct = 0; ct < CT; ct++)
#pragma unroll
          for (int r = 0; r < 4; r++) {
            const int row = rb + r, col = 16 * ct + L.lr;
            if (L.has && row < D && col < D) pm[r * D + 16 * ct] = dMf[ct][r];
          }
        __syncthreads();
      }
    }
    // d phi / d x: every x_j^0 = x + noise (j < N), x_N = x, z^0 = x^0
    if (L.tid < D) {
      float g = 0.f;
      for (int j = 0; j <= Np; j++) g += XB[j * LD + L.tid] + ZB[j * LD + L.tid];
      b.dphi_dx[pt * D + L.tid] = g;
    }
    __syncthreads();
  }
  // ---- per-workgroup partial parameter gradients (dM, dQ are already there) ----------------
#pragma unroll
  for (int ct = 0; ct < CT; ct++)
#pragma unroll
    for (int r = 0; r < 4; r++) {
      const int row = 16 * L.wave + 4 * L.lk + r, col = 16 * ct + L.lr;
      if (L.has && row < D && col < D) part[row * D + col] = dA[ct][r];
    }
  deps = wg_sum(deps, s_red);
  if (L.tid == 0) part[3 * DD] = deps;
}

// Sum the per-workgroup partials (fixed order: deterministic).
__global__ void k_lt_reduce_parts(const float* part, int nwg, int d, float* out /* [3 d^2 + 1] */) {
  const int64_t DD = int64_t(d) * d, W = 3 * DD + 1;
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= W) return;
  float s = 0.f;
  for (int g = 0; g < nwg; g++) s += part[g * W + e];
  out[e] = s;
}

// C = scale A B (row-major d x d)
__global__ void k_lt_matmul(const float* Aa, const float* Bb, int d, float* C, float scale) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= d * d) return;
  const int r = e / d, c = e - r * d;
  float s = 0.f;
  for (int k = 0; k < d; k++) s += Aa[r * d + k] * Bb[k * d + c];
  C[e] = scale * s;
}

// dh = [deps, dA]; dg = dQ_direct + sym(S) with S = -tau M dM M.
__global__ void k_lt_grad_out(const float* sums, const float* S, int d, float* dh, float* dg) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t DD = int64_t(d) * d;
  if (e == 0) dh[0] = sums[3 * DD];
  if (e >= d * d) return;
  const int r = e / d, c = e - r * d;
  dh[1 + e] = sums[e];
  dg[e] = sums[2 * DD + e] + 0.5f * (S[r * d + c] + S[c * d + r]);
}

// (I + tau Q_s)^{-1} by Gauss-Jordan elimination with partial pivoting in
// double precision, one workgroup; W is a d x 2d double scratch.
__global__ void k_lt_inverse(const float* Q, int d, double tau, double* W, float* Mout, int* fail) {
  __shared__ int s_piv;
  __shared__ double s_f[kLtMaxD];
  const int tid = threadIdx.x, nt = blockDim.x, w2 = 2 * d;
  for (int e = tid; e < d * w2; e += nt) {
    const int r = e / w2, c = e - r * w2;
    double v;
    if (c < d)
      v = (r == c ? 1.0 : 0.0) + tau * 0.5 * (double(Q[r * d + c]) + double(Q[c * d + r]));
    else
      v = (c - d == r) ? 1.0 : 0.0;
    W[e] = v;
  }
  if (tid == 0) *fail = 0;
  __syncthreads();
  for (int c = 0; c < d; c++) {
    if (tid == 0) {
      int best = c;
      double bv = fabs(W[c * w2 + c]);
      for (int r = c + 1; r < d; r++) {
        const double v = fabs(W[r * w2 + c]);
        if (v > bv) {
          bv = v;
          best = r;
        }
      }
      s_piv = best;
      if (!(bv > 0.0)) *fail = 1;
    }
    __syncthreads();
    const int pr = s_piv;
    if (pr != c)
      for (int e = tid; e < w2; e += nt) {
        const double tmp = W[c * w2 + e];
        W[c * w2 + e] = W[pr * w2 + e];
        W[pr * w2 + e] = tmp;
      }
    __syncthreads();
    const double inv = 1.0 / W[c * w2 + c];
    __syncthreads();
    for (int e = tid; e < w2; e += nt) W[c * w2 + e] *= inv;
    __syncthreads();
    for (int r = tid; r < d; r += nt) s_f[r] = W[r * w2 + c];
    __syncthreads();
    for (int e = tid; e < d * w2; e += nt) {
      const int r = e / w2, col = e - r * w2;
      if (r != c) W[e] -= s_f[r] * W[c * w2 + col];
    }
    __syncthreads();
  }
  for (int e = tid; e < d * d; e += nt) {
    const int r = e / d, c = e - r * d;
    Mout[e] = float(W[r * w2 + d + c]);
  }
}

__global__ void k_lt_zero(int32_t* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

struct LtState {
  int d = 0;
  int n_cu = 0;
  float* M = nullptr;           // d*d
  double* W = nullptr;          // d*2d
  int32_t* counters = nullptr;  // [0] forward head, [1] inverse failure, [2] backward head
  int32_t* scratch_i = nullptr; // iterations and statuses of the forward pass in value_grad
  size_t scratch_bytes = 0;
  float* ckpt = nullptr;
  size_t ckpt_bytes = 0;
  float* seg = nullptr;
  size_t seg_bytes = 0;
  float* part = nullptr;
  size_t part_bytes = 0;
  float* sums = nullptr;  // 3 d^2 + 1
  float* tmp = nullptr;   // 2 d^2
};

typedef const void* KernelPtr;

static KernelPtr forward_kernel(int d) {
  switch (d) {
    case 16: return reinterpret_cast<KernelPtr>(&k_lt_forward<16>);
    case 32: return reinterpret_cast<KernelPtr>(&k_lt_forward<32>);
    case 100: return reinterpret_cast<KernelPtr>(&k_lt_forward<100>);
    case 128: return reinterpret_cast<KernelPtr>(&k_lt_forward<128>);
  }
  return nullptr;
}

static KernelPtr backward_kernel(int d) {
  switch (d) {
    case 16: return reinterpret_cast<KernelPtr>(&k_lt_backward<16>);
    case 32: return reinterpret_cast<KernelPtr>(&k_lt_backward<32>);
    case 100: return reinterpret_cast<KernelPtr>(&k_lt_backward<100>);
    case 128: return reinterpret_cast<KernelPtr>(&k_lt_backward<128>);
  }
  return nullptr;
}

#define LT_HIP(expr, what)                                                                                    \
  do {                                                                                                        \
    hipError_t e_ = (expr);                                                                                   \
    if (e_ != hipSuccess) return hjpd_fail(HJPD_EDEVICE, (std::string(what) + ": " + hipGetErrorString(e_)).c_str()); \
  } while (0)

int lt_create(LtState** out, const hjpd_desc& desc) {
  *out = nullptr;
  if (!forward_kernel(desc.d)) return hjpd_fail(HJPD_EUNSUPPORTED, "LINEAR_TANH is built for d in {16,32,100,128}");
  if (desc.N_max > kLtMaxN) return hjpd_fail(HJPD_EUNSUPPORTED, "LINEAR_TANH is built for N_max <= 64");
  LtState* s = new LtState();
  s->d = desc.d;
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    delete s;
    return hjpd_fail(HJPD_EDEVICE, "device query failed");
  }
  s->n_cu = prop.multiProcessorCount;
  if (hipFuncSetAttribute(forward_kernel(desc.d), hipFuncAttributeMaxDynamicSharedMemorySize,
                          int(lt_lds_forward(desc.d, desc.N_max))) != hipSuccess ||
      hipFuncSetAttribute(backward_kernel(desc.d), hipFuncAttributeMaxDynamicSharedMemorySize,
                          int(lt_lds_backward(desc.d, desc.N_max))) != hipSuccess) {
    delete s;
    return hjpd_fail(HJPD_EDEVICE, "cannot reserve LDS for the linear-tanh kernels");
  }
  const size_t dd = size_t(desc.d) * desc.d;
  if (hipMalloc(&s->M, sizeof(float) * dd) != hipSuccess || hipMalloc(&s->W, sizeof(double) * 2 * dd) != hipSuccess ||
      hipMalloc(&s->counters, sizeof(int32_t) * 8) != hipSuccess ||
      hipMalloc(&s->sums, sizeof(float) * (3 * dd + 1)) != hipSuccess ||
      hipMalloc(&s->tmp, sizeof(float) * 2 * dd) != hipSuccess) {
    lt_destroy(s);
    return hjpd_fail(HJPD_ENOMEM, "linear-tanh workspace");
  }
  *out = s;
  return HJPD_OK;
}

void lt_destroy(LtState* s) {
  if (!s) return;
  if (s->M) (void)hipFree(s->M);
  if (s->W) (void)hipFree(s->W);
  if (s->counters) (void)hipFree(s->counters);
  if (s->scratch_i) (void)hipFree(s->scratch_i);
  if (s->ckpt) (void)hipFree(s->ckpt);
  if (s->seg) (void)hipFree(s->seg);
  if (s->part) (void)hipFree(s->part);
  if (s->sums) (void)hipFree(s->sums);
  if (s->tmp) (void)hipFree(s->tmp);
  delete s;
}

static int lt_grid(LtState* st, KernelPtr k, size_t lds) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, kLtThreads, lds) != hipSuccess || nb < 1) nb = 1;
  return nb * st->n_cu;
}

static void fill_args(LtArgs& a, LtState* st, const hjpd_desc& d, int64_t n, const void* x, const void* t,
                      const int32_t* N, const void* hp, const void* gp, void* phi, void* xtraj, void* ptraj,
                      int32_t* iters, int32_t* status, int max_iter, bool fixed) {
  std::memset(&a, 0, sizeof(a));
  a.x = (const float*)x;
  a.t = (const float*)t;
  a.N = N;
  a.hp = (const float*)hp;
  a.Q = (const float*)gp;
  a.M = st->M;
  a.phi = (float*)phi;
  a.xtraj = (float*)xtraj;
  a.ptraj = (float*)ptraj;
  a.iters = iters;
  a.status = status;
  a.head = st->counters;
  a.n = n;
  a.sigma = float(d.sigma);
  a.tau = float(d.tau);
  a.theta = float(d.theta);
  a.tol = float(d.tol);
  a.max_iter = max_iter;
  a.fixed = fixed ? 1 : 0;
  a.N_max = d.N_max;
  a.seed = d.seed;
  a.ckpt_every = 1;
}

static int lt_setup(LtState* st, const hjpd_desc& d, const void* gp, hipStream_t s) {
  hipLaunchKernelGGL(k_lt_zero, dim3(1), dim3(64), 0, s, st->counters, 8);
  hipLaunchKernelGGL(k_lt_inverse, dim3(1), dim3(256), 0, s, (const float*)gp, d.d, d.tau, st->W, st->M,
                     st->counters + 1);
  LT_HIP(hipGetLastError(), "linear-tanh set-up kernels");
  return HJPD_OK;
}

int lt_solve(LtState* st, const hjpd_desc& d, int64_t n, const void* x, const void* t, const int32_t* N,
             const void* hp, const void* gp, void* phi, void* xtraj, void* ptraj, int32_t* iters, int32_t* status,
             hipStream_t s, hipEvent_t ev0, hipEvent_t ev1, int* launches, bool* timing_valid) {
  int rc = lt_setup(st, d, gp, s);
  if (rc) return rc;
  LtArgs a;
  fill_args(a, st, d, n, x, t, N, hp, gp, phi, xtraj, ptraj, iters, status, d.max_iter,
            (d.flags & HJPD_FIXED_ITERS) != 0);
  const size_t lds = lt_lds_forward(d.d, d.N_max);
  KernelPtr k = forward_kernel(d.d);
  void* args[] = {&a};
  if (ev0) LT_HIP(hipEventRecord(ev0, s), "hipEventRecord");
  LT_HIP(hipLaunchKernel(k, dim3(lt_grid(st, k, lds)), dim3(kLtThreads), args, lds, s), "linear-tanh forward");
  if (ev1) LT_HIP(hipEventRecord(ev1, s), "hipEventRecord");
  if (launches) *launches = 1;
  if (timing_valid) *timing_valid = ev0 != nullptr;
  return HJPD_OK;
}

static int grow(void** p, size_t* cap, size_t need) {
  if (need <= *cap) return HJPD_OK;
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  *cap = 0;
  if (hipMalloc(p, need) != hipSuccess) return hjpd_fail(HJPD_ENOMEM, "linear-tanh reverse-mode buffers");
  *cap = need;
  return HJPD_OK;
}

int lt_value_grad(LtState* st, const hjpd_desc& d, int64_t n, const void* x, const void* t, const int32_t* N,
                  const void* hp, const void* gp, const void* grad_phi, int K, int E, void* phi, void* dphi_dx,
                  void* dh, void* dg, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1, int* launches,
                  bool* timing_valid) {
  if (timing_valid) *timing_valid = false;
  if (E > K) E = K;
  const int n_ckpt = (K + E - 1) / E;
  const size_t CK = size_t(d.N_max + 1) * d.d;
  const size_t dd = size_t(d.d) * d.d;
  // buffers may be reallocated: finish earlier work on this context first
  LT_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
  int rc = grow((void**)&st->ckpt, &st->ckpt_bytes, sizeof(float) * size_t(n) * (n_ckpt + 1) * 3 * CK);
  if (rc) return rc;
  KernelPtr kb = backward_kernel(d.d);
  const size_t lds_b = lt_lds_backward(d.d, d.N_max);
  const int grid_b = lt_grid(st, kb, lds_b);
  rc = grow((void**)&st->seg, &st->seg_bytes, sizeof(float) * size_t(grid_b) * lt_seg_floats(d.d, d.N_max, E));
  if (rc) return rc;
  rc = grow((void**)&st->part, &st->part_bytes, sizeof(float) * size_t(grid_b) * (3 * dd + 1));
  if (rc) return rc;
  rc = grow((void**)&st->scratch_i, &st->scratch_bytes, sizeof(int32_t) * 2 * size_t(n));
  if (rc) return rc;
  rc = lt_setup(st, d, gp, s);
  if (rc) return rc;
  LtArgs a;
  fill_args(a, st, d, n, x, t, N, hp, gp, phi, nullptr, nullptr, st->scratch_i, st->scratch_i + n, K, true);
  a.ckpt = st->ckpt;
  a.ckpt_every = E;
  a.n_ckpt = n_ckpt;
  KernelPtr kf = forward_kernel(d.d);
  const size_t lds_f = lt_lds_forward(d.d, d.N_max);
  void* fargs[] = {&a};
  LT_HIP(hipLaunchKernel(kf, dim3(lt_grid(st, kf, lds_f)), dim3(kLtThreads), fargs, lds_f, s), "linear-tanh forward");
  LtBwdArgs b;
  b.f = a;
  b.f.phi = nullptr;
  b.grad_phi = (const float*)grad_phi;
  b.dphi_dx = (float*)dphi_dx;
  b.seg = st->seg;
  b.part = st->part;
  b.K = K;
  void* bargs[] = {&b};
  if (ev0) LT_HIP(hipEventRecord(ev0, s), "hipEventRecord");
  LT_HIP(hipLaunchKernel(kb, dim3(grid_b), dim3(kLtThreads), bargs, lds_b, s), "linear-tanh backward");
  if (ev1) LT_HIP(hipEventRecord(ev1, s), "hipEventRecord");
  const int W = int(3 * dd + 1);
  hipLaunchKernelGGL(k_lt_reduce_parts, dim3((W + 255) / 256), dim3(256), 0, s, st->part, grid_b, d.d, st->sums);
  // S = -tau M (dM M)
  const int nb = int((dd + 255) / 256);
  hipLaunchKernelGGL(k_lt_matmul, dim3(nb), dim3(256), 0, s, st->sums + dd, st->M, d.d, st->tmp, 1.f);
  hipLaunchKernelGGL(k_lt_matmul, dim3(nb), dim3(256), 0, s, st->M, st->tmp, d.d, st->tmp + dd, -float(d.tau));
  hipLaunchKernelGGL(k_lt_grad_out, dim3(nb), dim3(256), 0, s, st->sums, st->tmp + dd, d.d, (float*)dh, (float*)dg);
  LT_HIP(hipGetLastError(), "linear-tanh gradient kernels");
  if (ev0 && ev1) {
    if (launches) *launches = 1;
    if (timing_valid) *timing_valid = true;
  }
  return HJPD_OK;
}

}  // namespace hjpd
