// Problem families for the lane-group kernels.
//
// Each family supplies, for one time node, the pieces of one iteration of the
// splitting of section 5 (Algorithm 1; games Algorithm 3) in the form of
// section 5.3: the closed-form proximal map of sigma*delta*H(x_j, .) for the
// dual step, the gradient of H in x for the single explicit primal step, H
// itself for the value, and the initial cost g with its proximal map for
// node 0.  Hamiltonians are in the initial-value convention
// H = max_u {<f,p> - L} with time-reversed dynamics (section 2.1): for a
// physically specified problem with H_c = min_u {<f_phys,p> + L}, H = -H_c.
//
// A `Cache` carries the state-dependent quantities evaluated at x_j^k in the
// dual step (trigonometric values, norms) to the primal step, which uses the
// same x_j^k.
#pragma once

#include "hjpd_device.hpp"

namespace hjpd {

enum : int { kGNorm = 0, kGQuadShift = 1, kGPairDist = 2, kGQuadForm = 3 };

// ===========================================================================
// Eikonal with state-dependent speed (section 6.1):
//   H(x,p) = c(x) ||p||,  c(x) = 1 + alpha sin(x_1) cos(x_2).
// prox of lam*H(x,.) is shrink_2(v, lam c(x)) (section 6.1.2), and
// grad_x H = ||p|| grad c(x) with grad c = alpha (cos x1 cos x2, -sin x1 sin x2, 0...).
// Initial cost: ||x|| - r (prox: shrink_2(v, tau)) or ||x - a||^2/2 - c0
// (prox: (v + tau a)/(1 + tau)).
// ===========================================================================
template <int D_>
struct CNorm {
  static constexpr int D = D_;
  static constexpr int kWavesK[5] = {0, 4, 3, 2, 2};  // FP32 waves per SIMD by nodes per lane
  static constexpr bool kGame = false;
  // dual step maps v = 0 to p = 0 exactly (nodes past N stay at p = 0 without a mask)
  static constexpr bool kZeroSafe = true;
  // Hopf formulation (Algorithm 2) available: closed-form conjugates of both g
  static constexpr bool kHopf = true;
  // Weighted Euler discretisations (forward Euler, trapezoid) available: a
  // weighted sum of c(x_{j-1})|p| and c(x_j)|p| is again a multiple of |p|,
  // so its prox stays a shrink
  static constexpr bool kMix = true;

  template <typename T> struct Par {
    T alpha;
    int gkind;
    T r;            // NORM radius
    T c0;           // QUAD_SHIFT constant
    T ta[D];        // tau * a   (QUAD_SHIFT)
    T a[D];
    T inv1pt;       // 1 / (1 + tau)
    T s1pt;         // tau / (1 + tau)
    T sa[D];        // tau / (1 + tau) * a
  };
  template <typename T> struct Cache {
    T pn;           // ||p_new||
    T gc0, gc1;     // grad c at x_j^k (first two coordinates)
  };

  template <typename T>
  __device__ static void load(Par<T>& P, const T* hp, const T* gp, int gkind, T tau) {
    P.alpha = hp[0];
    P.gkind = gkind;
    P.r = gp[0];
    P.c0 = gp[0];
#pragma unroll
    for (int i = 0; i < D; i++) P.a[i] = (gkind == kGQuadShift) ? gp[1 + i] : T(0);
    set_tau(P, tau, gkind);
  }

  // Parameters that depend on the primal step tau (recomputed when a recipe
  // raises sigma and lowers tau).
  template <typename T>
  __device__ static void set_tau(Par<T>& P, T tau, int) {
#pragma unroll
    for (int i = 0; i < D; i++) P.ta[i] = tau * P.a[i];
    P.inv1pt = T(1) / (T(1) + tau);
    P.s1pt = tau / (T(1) + tau);
#pragma unroll
    for (int i = 0; i < D; i++) P.sa[i] = P.s1pt * P.a[i];
  }

  template <typename T>
  __device__ static void dual(const Par<T>& P, const T (&x)[D], T (&v)[D], T lam, Cache<T>& C) {
    T s1, c1, s2, c2;
    M<T>::sincos(x[0], &s1, &c1);
    M<T>::sincos(x[1], &s2, &c2);
    const T c = T(1) + P.alpha * s1 * c2;
    T ss = T(0);
#pragma unroll
    for (int i = 0; i < D; i++) ss += v[i] * v[i];
    const T rs = M<T>::rsqrt(ss);                 // +inf at v = 0
    const bool nz = ss > T(0);
    const T scale = nz ? M<T>::fmax(T(1) - lam * c * rs, T(0)) : T(0);
    C.pn = nz ? scale * (ss * rs) : T(0);         // = max(||v|| - lam c, 0)
#pragma unroll
    for (int i = 0; i < D; i++) v[i] *= scale;
    C.gc0 = P.alpha * c1 * c2;
    C.gc1 = -P.alpha * s1 * s2;
  }

  // Speed c(x) = 1 + alpha sin(x_1) cos(x_2) and the two non-zero
  // components of its gradient.
  template <typename T>
  __device__ static void speed(const Par<T>& P, const T (&x)[D], T& c, T& gc0, T& gc1) {
    T s1, c1, s2, c2;
    M<T>::sincos(x[0], &s1, &c1);
    M<T>::sincos(x[1], &s2, &c2);
    c = T(1) + P.alpha * s1 * c2;
    gc0 = P.alpha * c1 * c2;
    gc1 = -P.alpha * s1 * s2;
  }

  // Node-0 prox in the shifted layout: v <- prox_{tau g}(v) in the group's
  // first lane, v unchanged elsewhere (first = false).
  template <typename T>
  __device__ static void prox0(const Par<T>& P, T (&v)[D], T tau, bool first) {
    if (P.gkind == kGNorm) {
      T ss = T(0);
#pragma unroll
      for (int i = 0; i < D; i++) ss += v[i] * v[i];
      const T sc = M<T>::fmax(T(1) - tau * M<T>::rsqrt(ss), T(0));
      const T m = first ? sc : T(1);
#pragma unroll
      for (int i = 0; i < D; i++) v[i] *= m;
    } else {
      // (v + tau a)/(1 + tau) = v/(1 + tau) + sa
      const T m = first ? P.inv1pt : T(1);
      const T f = first ? T(1) : T(0);
#pragma unroll
      for (int i = 0; i < D; i++) v[i] = m * v[i] + f * P.sa[i];
    }
  }

  // The node-0 prox of the shifted layout when it is affine, prox(v) = m v + f:
  // true for the shifted quadratic g, with (m, f) = (1/(1 + tau), tau a/(1 + tau))
  // in the group's first lane and (1, 0) elsewhere; false for the norm g, whose
  // prox (prox0) is not affine.
  template <typename T>
  __device__ static bool prox0_affine(const Par<T>& P, bool first, T& m, T (&f)[D]) {
    m = first ? P.inv1pt : T(1);
#pragma unroll
    for (int i = 0; i < D; i++) f[i] = first ? P.sa[i] : T(0);
    return P.gkind != kGNorm;
  }

  // v <- shrink_2(v, mu) = v max(1 - mu/|v|, 0) (shrink_2(0) = 0); returns |v| after.
  template <typename T>
  __device__ static T shrink(T (&v)[D], T mu) {
    T ss = T(0);
#pragma unroll
    for (int i = 0; i < D; i++) ss += v[i] * v[i];
    const T rs = M<T>::rsqrt(ss);
    const bool nz = ss > T(0);
    const T scale = nz ? M<T>::fmax(T(1) - mu * rs, T(0)) : T(0);
#pragma unroll
    for (int i = 0; i < D; i++) v[i] *= scale;
    return nz ? scale * (ss * rs) : T(0);
  }

  // Dual step of the shifted layout's slot 0 in the Hopf formulation, given
  // the threshold mu = sigma delta c(x_1): in the group's first lane (node 1)
  // the joint prox with g* (see dual_hopf1), elsewhere the plain shrink.
  // v and mu are in units of `unit` (the kernel keeps the dual scaled by tau):
  // the prox commutes with that scaling once a and the unit ball of g* are
  // scaled too.  Returns |p| after, in the same units.
  template <typename T>
  __device__ static T shrink_hopf1(const Par<T>& P, T (&v)[D], T mu, T sigma, bool first, T unit) {
    if (P.gkind != kGNorm) {
      const T r1 = first ? M<T>::div(T(1), T(1) + sigma) : T(1);
      const T sg = first ? sigma * unit : T(0);
#pragma unroll
      for (int i = 0; i < D; i++) v[i] = (v[i] - sg * P.a[i]) * r1;
      mu *= r1;
    }
    T ss = T(0);
#pragma unroll
    for (int i = 0; i < D; i++) ss += v[i] * v[i];
    const bool nz = ss > T(0);
    const T rs = M<T>::rsqrt(ss);
    T len = nz ? M<T>::fmax(ss * rs - mu, T(0)) : T(0);
    if (P.gkind == kGNorm && first) len = len < unit ? len : unit;
    const T scale = nz ? len * rs : T(0);
#pragma unroll
    for (int i = 0; i < D; i++) v[i] *= scale;
    return len;
  }

  // Hopf formulation, dual step at j = 1 (Algorithm 2): the joint prox
  //   argmin_p g*(p) + lam/sigma c(x)|p| + |p - v|^2/(2 sigma),  lam = sigma delta.
  // Shifted quadratic g: g*(p) = |p|^2/2 + <a,p> + c0, so completing the square
  // gives p = shrink_2((v - sigma a)/(1 + sigma), lam c/(1 + sigma)).
  // Norm g: g* = r on the unit ball, so p = v/|v| min(max(|v| - lam c, 0), 1).
  template <typename T>
  __device__ static void dual_hopf1(const Par<T>& P, const T (&x)[D], T (&v)[D], T lam, T sigma, Cache<T>& C) {
    T s1, c1, s2, c2;
    M<T>::sincos(x[0], &s1, &c1);
    M<T>::sincos(x[1], &s2, &c2);
    const T c = T(1) + P.alpha * s1 * c2;
    T mu = lam * c;
    if (P.gkind != kGNorm) {
      const T r1 = M<T>::div(T(1), T(1) + sigma);
#pragma unroll
      for (int i = 0; i < D; i++) v[i] = (v[i] - sigma * P.a[i]) * r1;
      mu *= r1;
    }
    T ss = T(0);
#pragma unroll
    for (int i = 0; i < D; i++) ss += v[i] * v[i];
    const bool nz = ss > T(0);
    const T rs = M<T>::rsqrt(ss);
    T len = nz ? M<T>::fmax(ss * rs - mu, T(0)) : T(0);  // shrunk length
    if (P.gkind == kGNorm) len = len < T(1) ? len : T(1);
    const T scale = nz ? len * rs : T(0);
    C.pn = len;
#pragma unroll
    for (int i = 0; i < D; i++) v[i] *= scale;
    C.gc0 = P.alpha * c1 * c2;
    C.gc1 = -P.alpha * s1 * s2;
  }

  // Convex conjugate of g at p (finite branch: the Hopf iterates keep |p| <= 1 for the norm g).
  template <typename T>
  __device__ static T gstar(const Par<T>& P, const T (&p)[D]) {
    if (P.gkind == kGNorm) return P.r;
    T s = T(0);
#pragma unroll
    for (int i = 0; i < D; i++) s += p[i] * (T(0.5) * p[i] + P.a[i]);
    return s + P.c0;
  }

  // Only the first two coordinates of grad_x H are non-zero.
  template <typename T>
  __device__ static void grad(const Par<T>&, const T (&)[D], const T (&)[D], const Cache<T>& C, T (&g)[D]) {
#pragma unroll
    for (int i = 0; i < D; i++) g[i] = T(0);
    g[0] = C.pn * C.gc0;
    g[1] = C.pn * C.gc1;
  }

  template <typename T>
  __device__ static T H(const Par<T>& P, const T (&x)[D], const T (&p)[D]) {
    T s1, c1, s2, c2;
    M<T>::sincos(x[0], &s1, &c1);
    M<T>::sincos(x[1], &s2, &c2);
    T ss = T(0);
#pragma unroll
    for (int i = 0; i < D; i++) ss += p[i] * p[i];
    return (T(1) + P.alpha * s1 * c2) * M<T>::sqrt(ss);
  }

  template <typename T>
  __device__ static void prox_g(const Par<T>& P, const T (&v)[D], T tau, T (&o)[D]) {
    if (P.gkind == kGNorm) {
      T ss = T(0);
#pragma unroll
      for (int i = 0; i < D; i++) ss += v[i] * v[i];
      const T scale = M<T>::fmax(T(1) - tau * M<T>::rsqrt(ss), T(0));
#pragma unroll
      for (int i = 0; i < D; i++) o[i] = scale * v[i];
    } else {
#pragma unroll
      for (int i = 0; i < D; i++) o[i] = (v[i] + P.ta[i]) * P.inv1pt;
    }
  }

  // Node-0 increment prox_{tau g}(x0 + tau p1) - x0.  For the shifted
  // quadratic this is tau/(1+tau) (p1 + a - x0).
  template <typename T>
  __device__ static void step0(const Par<T>& P, const T (&x0)[D], const T (&p1)[D], T tau, T (&dx)[D]) {
    if (P.gkind == kGNorm) {
      T v[D], o[D];
#pragma unroll
      for (int i = 0; i < D; i++) v[i] = x0[i] + tau * p1[i];
      prox_g(P, v, tau, o);
#pragma unroll
      for (int i = 0; i < D; i++) dx[i] = o[i] - x0[i];
    } else {
#pragma unroll
      for (int i = 0; i < D; i++) dx[i] = P.s1pt * (p1[i] - x0[i]) + P.sa[i];
    }
  }

  template <typename T>
  __device__ static T g(const Par<T>& P, const T (&x)[D]) {
    T ss = T(0);
    if (P.gkind == kGNorm) {
#pragma unroll
      for (int i = 0; i < D; i++) ss += x[i] * x[i];
      return M<T>::sqrt(ss) - P.r;
    }
#pragma unroll
    for (int i = 0; i < D; i++) ss += (x[i] - P.a[i]) * (x[i] - P.a[i]);
    return T(0.5) * ss - P.c0;
  }
};

// ===========================================================================
// Quadrotor-like control, d = 12: x = (r, v, eta, omega), eta = (roll phi,
// pitch th, yaw psi).  Physical dynamics f = f0 + B u:
//   f0 = (v, -g_z e3, W(eta) omega, 0),  B u = (0, (u_1/m) R e3, 0, J^{-1} u_{2:4}),
//   R = Rz(psi) Ry(th) Rx(phi), W = ZYX Euler-rate matrix with the pitch
//   clamped to [-c, c] (zero slope outside), cost |u|^2/2.
// H = -<p, f0> + ((b.p_v)^2 + sum_i (p_w,i/J_i)^2)/2 with b = R e3 / m.
// Dual prox of lam*H(x,.): p_r = v_r + lam vel; p_eta = v_eta + lam W omega;
// p_v = w - lam (b.w)/(1 + lam |b|^2) b with w = v_v - lam g_z e3
// (Sherman-Morrison); p_w,i = v_w,i / (1 + lam / J_i^2).
// Initial cost ||x - a||^2/2 - c0.
// ===========================================================================
struct Quad {
  static constexpr int D = 12;
  // FP32 waves per SIMD by nodes per lane: x, p, z and the 29-value geometry
  // cache of a node take about 65 registers
  static constexpr int kWavesK[5] = {0, 3, 2, 2, 2};
  static constexpr bool kGame = false;
  static constexpr bool kZeroSafe = false;
  static constexpr bool kHopf = false;      // no Hopf step in the plain kernel
  static constexpr bool kHopfGroup = true;  // Hopf formulation in k_group_control
  static constexpr bool kMix = false;
  static constexpr bool kWeighted = true;  // forward Euler / trapezoid in k_group_control (kW)

  template <typename T> struct Par {
    T m_inv, gz, clamp;
    T iJ2[3];                 // 1 / J_i^2
    T c0, a[12], ta[12], inv1pt, s1pt, sa[12];
  };
  template <typename T> struct Cache {
    T b[3];                   // R e3 / m
    T db[3][3];               // d b / d(phi, th, psi)
    T W01, W02, W11, W12, W21, W22;       // W (row 0 col 0 is 1, col 0 below is 0)
    T dWf01, dWf02, dWf11, dWf12, dWf21, dWf22;  // d W / d phi
    T dWt01, dWt02, dWt21, dWt22;                // d W / d th (rows 0 and 2)
    T bp;                     // b . p_v (new p)
  };

  template <typename T>
  __device__ static void load(Par<T>& P, const T* hp, const T* gp, int, T tau) {
    P.m_inv = T(1) / hp[0];
#pragma unroll
    for (int i = 0; i < 3; i++) P.iJ2[i] = T(1) / (hp[1 + i] * hp[1 + i]);
    P.gz = hp[4];
    P.clamp = hp[5];
    P.c0 = gp[0];
#pragma unroll
    for (int i = 0; i < 12; i++) P.a[i] = gp[1 + i];
    set_tau(P, tau, 0);
  }

  // Parameters that depend on the primal step tau.
  template <typename T>
  __device__ static void set_tau(Par<T>& P, T tau, int) {
#pragma unroll
    for (int i = 0; i < 12; i++) P.ta[i] = tau * P.a[i];
    P.inv1pt = T(1) / (T(1) + tau);
    P.s1pt = tau / (T(1) + tau);
#pragma unroll
    for (int i = 0; i < 12; i++) P.sa[i] = P.s1pt * P.a[i];
  }

  template <typename T>
  __device__ static void geometry(const Par<T>& P, const T (&x)[12], Cache<T>& C) {
    T sf, cf, st, ct, ss, cs;
    M<T>::sincos(x[6], &sf, &cf);
    M<T>::sincos(x[7], &st, &ct);
    M<T>::sincos(x[8], &ss, &cs);
    const T mi = P.m_inv;
    C.b[0] = (cs * st * cf + ss * sf) * mi;
    C.b[1] = (ss * st * cf - cs * sf) * mi;
    C.b[2] = (ct * cf) * mi;
    C.db[0][0] = (ss * cf - cs * st * sf) * mi;
    C.db[0][1] = (-ss * st * sf - cs * cf) * mi;
    C.db[0][2] = (-ct * sf) * mi;
    C.db[1][0] = (cs * ct * cf) * mi;
    C.db[1][1] = (ss * ct * cf) * mi;
    C.db[1][2] = (-st * cf) * mi;
    C.db[2][0] = (cs * sf - ss * st * cf) * mi;
    C.db[2][1] = (cs * st * cf + ss * sf) * mi;
    C.db[2][2] = T(0);
    // Euler-rate matrix at the clamped pitch
    const T th = x[7];
    const bool inside = (th > -P.clamp) && (th < P.clamp);
    T stc = st, ctc = ct;
    if (!inside) M<T>::sincos(th > T(0) ? P.clamp : -P.clamp, &stc, &ctc);
    const T sec = M<T>::rcp(ctc);
    const T tt = stc * sec;
    C.W01 = sf * tt;  C.W02 = cf * tt;
    C.W11 = cf;       C.W12 = -sf;
    C.W21 = sf * sec; C.W22 = cf * sec;
    C.dWf01 = cf * tt;  C.dWf02 = -sf * tt;
    C.dWf11 = -sf;      C.dWf12 = -cf;
    C.dWf21 = cf * sec; C.dWf22 = -sf * sec;
    const T k = inside ? T(1) : T(0);
    const T sec2 = k * sec * sec, sect = k * sec * tt;
    C.dWt01 = sf * sec2; C.dWt02 = cf * sec2;
    C.dWt21 = sf * sect; C.dWt22 = cf * sect;
  }

  template <typename T>
  __device__ static void dual(const Par<T>& P, const T (&x)[12], T (&v)[12], T lam, Cache<T>& C) {
    geometry(P, x, C);
    const T w0 = x[9], w1 = x[10], w2 = x[11];
    // position costate
    v[0] += lam * x[3];
    v[1] += lam * x[4];
    v[2] += lam * x[5];
    // angle costate: + lam W omega
    v[6] += lam * (w0 + C.W01 * w1 + C.W02 * w2);
    v[7] += lam * (C.W11 * w1 + C.W12 * w2);
    v[8] += lam * (C.W21 * w1 + C.W22 * w2);
    // velocity costate
    v[5] -= lam * P.gz;
    const T bw = C.b[0] * v[3] + C.b[1] * v[4] + C.b[2] * v[5];
    const T bb = C.b[0] * C.b[0] + C.b[1] * C.b[1] + C.b[2] * C.b[2];
    const T coef = M<T>::div(lam * bw, T(1) + lam * bb);
    v[3] -= coef * C.b[0];
    v[4] -= coef * C.b[1];
    v[5] -= coef * C.b[2];
    // body-rate costate
#pragma unroll
    for (int i = 0; i < 3; i++) v[9 + i] = M<T>::div(v[9 + i], T(1) + lam * P.iJ2[i]);
    C.bp = C.b[0] * v[3] + C.b[1] * v[4] + C.b[2] * v[5];
  }

  template <typename T>
  __device__ static void grad(const Par<T>&, const T (&x)[12], const T (&p)[12], const Cache<T>& C, T (&g)[12]) {
    const T w0 = x[9], w1 = x[10], w2 = x[11];
    (void)w0;
    g[0] = g[1] = g[2] = T(0);
    g[3] = -p[0];
    g[4] = -p[1];
    g[5] = -p[2];
    const T pe0 = p[6], pe1 = p[7], pe2 = p[8];
    const T dwf = pe0 * (C.dWf01 * w1 + C.dWf02 * w2) + pe1 * (C.dWf11 * w1 + C.dWf12 * w2) +
                  pe2 * (C.dWf21 * w1 + C.dWf22 * w2);
    const T dwt = pe0 * (C.dWt01 * w1 + C.dWt02 * w2) + pe2 * (C.dWt21 * w1 + C.dWt22 * w2);
    const T bp = C.bp;
    g[6] = -dwf + bp * (C.db[0][0] * p[3] + C.db[0][1] * p[4] + C.db[0][2] * p[5]);
    g[7] = -dwt + bp * (C.db[1][0] * p[3] + C.db[1][1] * p[4] + C.db[1][2] * p[5]);
    g[8] = bp * (C.db[2][0] * p[3] + C.db[2][1] * p[4]);
    // -W^T p_eta
    g[9] = -pe0;
    g[10] = -(C.W01 * pe0 + C.W11 * pe1 + C.W21 * pe2);
    g[11] = -(C.W02 * pe0 + C.W12 * pe1 + C.W22 * pe2);
  }

  // Weighted discretisations (forward Euler, trapezoid): an interval's dual
  // step takes the Hamiltonians of both its end nodes, weighted (wl, wr).  What
  // it needs of a node: its velocity, W(eta) omega and the thrust direction b.
  template <typename T> struct Side {
    T v[3], Ww[3], b[3];
  };
  template <typename T>
  __device__ static void side(const T (&x)[12], const Cache<T>& C, Side<T>& S) {
    const T w0 = x[9], w1 = x[10], w2 = x[11];
#pragma unroll
    for (int i = 0; i < 3; i++) {
      S.v[i] = x[3 + i];
      S.b[i] = C.b[i];
    }
    S.Ww[0] = w0 + C.W01 * w1 + C.W02 * w2;
    S.Ww[1] = C.W11 * w1 + C.W12 * w2;
    S.Ww[2] = C.W21 * w1 + C.W22 * w2;
  }

  // v -> argmin_p lam (wl H(x_a, p) + wr H(x_b, p)) + |p - v|^2/2, with the
  // end nodes' side data Sa, Sb.  The drift terms are linear, the velocity
  // block is (I + lam (wl a a^T + wr b b^T)) p_v = w: writing p_v = w -
  // lam wl (a.p_v) a - lam wr (b.p_v) b gives two equations for a.p_v and
  // b.p_v, solved by Cramer's rule; the body-rate scale is Algorithm 1's.
  template <typename T>
  __device__ static void dual_w(const Par<T>& P, const Side<T>& Sa, const Side<T>& Sb, T (&v)[12], T lam, T wl,
                                T wr) {
    const T la = lam * wl, lb = lam * wr;
#pragma unroll
    for (int i = 0; i < 3; i++) {
      v[i] += la * Sa.v[i] + lb * Sb.v[i];
      v[6 + i] += la * Sa.Ww[i] + lb * Sb.Ww[i];
    }
    v[5] -= lam * P.gz;
    const T aa = Sa.b[0] * Sa.b[0] + Sa.b[1] * Sa.b[1] + Sa.b[2] * Sa.b[2];
    const T bb = Sb.b[0] * Sb.b[0] + Sb.b[1] * Sb.b[1] + Sb.b[2] * Sb.b[2];
    const T ab = Sa.b[0] * Sb.b[0] + Sa.b[1] * Sb.b[1] + Sa.b[2] * Sb.b[2];
    const T aw = Sa.b[0] * v[3] + Sa.b[1] * v[4] + Sa.b[2] * v[5];
    const T bw = Sb.b[0] * v[3] + Sb.b[1] * v[4] + Sb.b[2] * v[5];
    const T m11 = T(1) + la * aa, m22 = T(1) + lb * bb;
    const T idet = M<T>::div(T(1), m11 * m22 - la * lb * ab * ab);
    const T u = (m22 * aw - lb * ab * bw) * idet;  // a . p_v
    const T t = (m11 * bw - la * ab * aw) * idet;  // b . p_v
#pragma unroll
    for (int i = 0; i < 3; i++) v[3 + i] -= la * u * Sa.b[i] + lb * t * Sb.b[i];
#pragma unroll
    for (int i = 0; i < 3; i++) v[9 + i] = M<T>::div(v[9 + i], T(1) + lam * P.iJ2[i]);
  }

  // wr grad_x H(x, p) + wl grad_x H(x, pn), x's geometry in C: the terms
  // linear in the costate take wr p + wl pn, the thrust term (quadratic in
  // p_v) is weighted per costate.
  template <typename T>
  __device__ static void grad_w(const Par<T>&, const T (&x)[12], const T (&p)[12], const T (&pn)[12], T wl, T wr,
                                const Cache<T>& C, T (&g)[12]) {
    const T w1 = x[10], w2 = x[11];
    T q[12];
#pragma unroll
    for (int i = 0; i < 12; i++) q[i] = wr * p[i] + wl * pn[i];
    const T bp = C.b[0] * p[3] + C.b[1] * p[4] + C.b[2] * p[5];
    const T bq = C.b[0] * pn[3] + C.b[1] * pn[4] + C.b[2] * pn[5];
    const T cp = wr * bp, cq = wl * bq;
    g[0] = g[1] = g[2] = T(0);
    g[3] = -q[0];
    g[4] = -q[1];
    g[5] = -q[2];
    const T pe0 = q[6], pe1 = q[7], pe2 = q[8];
    const T dwf = pe0 * (C.dWf01 * w1 + C.dWf02 * w2) + pe1 * (C.dWf11 * w1 + C.dWf12 * w2) +
                  pe2 * (C.dWf21 * w1 + C.dWf22 * w2);
    const T dwt = pe0 * (C.dWt01 * w1 + C.dWt02 * w2) + pe2 * (C.dWt21 * w1 + C.dWt22 * w2);
    g[6] = -dwf + cp * (C.db[0][0] * p[3] + C.db[0][1] * p[4] + C.db[0][2] * p[5]) +
           cq * (C.db[0][0] * pn[3] + C.db[0][1] * pn[4] + C.db[0][2] * pn[5]);
    g[7] = -dwt + cp * (C.db[1][0] * p[3] + C.db[1][1] * p[4] + C.db[1][2] * p[5]) +
           cq * (C.db[1][0] * pn[3] + C.db[1][1] * pn[4] + C.db[1][2] * pn[5]);
    g[8] = cp * (C.db[2][0] * p[3] + C.db[2][1] * p[4]) + cq * (C.db[2][0] * pn[3] + C.db[2][1] * pn[4]);
    g[9] = -pe0;
    g[10] = -(C.W01 * pe0 + C.W11 * pe1 + C.W21 * pe2);
    g[11] = -(C.W02 * pe0 + C.W12 * pe1 + C.W22 * pe2);
  }

  template <typename T>
  __device__ static T H(const Par<T>& P, const T (&x)[12], const T (&p)[12]) {
    Cache<T> C;
    geometry(P, x, C);
    const T w0 = x[9], w1 = x[10], w2 = x[11];
    T drift = p[0] * x[3] + p[1] * x[4] + p[2] * x[5] - P.gz * p[5];
    drift += p[6] * (w0 + C.W01 * w1 + C.W02 * w2) + p[7] * (C.W11 * w1 + C.W12 * w2) +
             p[8] * (C.W21 * w1 + C.W22 * w2);
    const T bp = C.b[0] * p[3] + C.b[1] * p[4] + C.b[2] * p[5];
    T ctrl = bp * bp;
#pragma unroll
    for (int i = 0; i < 3; i++) ctrl += p[9 + i] * p[9 + i] * P.iJ2[i];
    return -drift + T(0.5) * ctrl;
  }

  template <typename T>
  __device__ static void prox_g(const Par<T>& P, const T (&v)[12], T, T (&o)[12]) {
#pragma unroll
    for (int i = 0; i < 12; i++) o[i] = (v[i] + P.ta[i]) * P.inv1pt;
  }
  // Node-0 increment prox_{tau g}(x0 + tau p1) - x0 = tau/(1+tau) (p1 + a - x0).
  template <typename T>
  __device__ static void step0(const Par<T>& P, const T (&x0)[12], const T (&p1)[12], T, T (&dx)[12]) {
#pragma unroll
    for (int i = 0; i < 12; i++) dx[i] = P.s1pt * (p1[i] - x0[i]) + P.sa[i];
  }


  // Hopf formulation, dual step at j = 1 (Algorithm 2): the joint prox of
  // g* + delta H(x_1,.) for the shifted quadratic g, g*(p) = |p|^2/2 + <a,p> +
  // c0.  Completing the square, sigma g*(p) + |p - v|^2/2 = (1 + sigma)/2
  // |p - w|^2 + const with w = (v - sigma a)/(1 + sigma), so it is the p-prox
  // of w with lam/(1 + sigma).  Applied to (v, lam) before dual() in the
  // group's first lane; identity elsewhere (first = false).
  template <typename T>
  __device__ static void hopf1_in(const Par<T>& P, T (&v)[12], T& lam, T sigma, bool first) {
    const T r1 = first ? M<T>::div(T(1), T(1) + sigma) : T(1);
    const T sg = first ? sigma : T(0);
#pragma unroll
    for (int i = 0; i < 12; i++) v[i] = (v[i] - sg * P.a[i]) * r1;
    lam *= r1;
  }

  // g*(p) = |p|^2/2 + <a,p> + c0 (the value's -g*(p_1) term, Hopf formulation)
  template <typename T>
  __device__ static T gstar(const Par<T>& P, const T (&p)[12]) {
    T s = P.c0;
#pragma unroll
    for (int i = 0; i < 12; i++) s += p[i] * (T(0.5) * p[i] + P.a[i]);
    return s;
  }

  template <typename T>
  __device__ static T g(const Par<T>& P, const T (&x)[12]) {
    T ss = T(0);
#pragma unroll
    for (int i = 0; i < 12; i++) ss += (x[i] - P.a[i]) * (x[i] - P.a[i]);
    return T(0.5) * ss - P.c0;
  }
};

// ===========================================================================
// Pursuit-evasion game, d = 12, d_y = 6 (section 4.2 / Algorithm 3).
// Pursuer x = (r_P, v_P) minimises, evader y = (r_E, v_E) maximises; each is
// a point mass with drag, F(r,v) = (v, -kappa |v| v), control on velocity.
// In the game variables (costate (p, -q)):
//   H(x,y,p,q) = -<p, F(x)> + <q, F(y)> + wP |p_v|^2/2 - wE |q_v|^2/2.
// p-step (argmin_p lam H + |p - v|^2/2): p_r = v_r + lam v_P,
//   p_v = (v_v - lam kappa |v_P| v_P) / (1 + lam wP);
// q-step (argmin_q -lam H + |q - v|^2/2): q_r = v_r + lam v_E,
//   q_v = (v_v - lam kappa |v_E| v_E) / (1 + lam wE);
// grad_x H = -J_F(x)^T p, grad_y H = J_F(y)^T q with
//   J_F(s)^T pi = (0, pi_r - kappa (|v| pi_v + (v.pi_v) v / |v|)).
// Initial cost g = |r_P - r_E| - r: node-0 pursuer prox moves r_P toward
// r_E by shrink_2; the evader's prox of -g moves r_E away from r_P by tau
// ("stretch"; direction e_1 when they coincide).
// ===========================================================================
struct Pursuit {
  static constexpr int D = 12;
  static constexpr int kWavesK[5] = {0, 4, 2, 2, 2};  // FP32 waves per SIMD by nodes per lane
  static constexpr int DX = 6, DY = 6;
  static constexpr bool kGame = true;
  static constexpr bool kZeroSafe = false;
  static constexpr bool kHopf = false;
  static constexpr bool kMix = false;
  static constexpr bool kGameHopf = false;  // Algorithm 3 (k_group_game, k_plain_game)

  template <typename T> struct Par {
    T kappa, wP, wE, r;
  };
  template <typename T> struct CacheX {
    T knv, kinv;  // kappa |v_P| at x_j^k and kappa / |v_P| (0 at v_P = 0)
  };
  template <typename T> struct CacheY {
    T knv, kinv;  // kappa |v_E| at y_j^k and kappa / |v_E| (0 at v_E = 0)
  };

  template <typename T>
  __device__ static void load(Par<T>& P, const T* hp, const T* gp, int, T) {
    P.kappa = hp[0];
    P.wP = hp[1];
    P.wE = hp[2];
    P.r = gp[0];
  }

  template <typename T>
  __device__ static T speed(const T (&s)[6]) {
    return M<T>::sqrt_fast(s[3] * s[3] + s[4] * s[4] + s[5] * s[5]);
  }

  // kappa |v| and kappa / |v| of a state from one reciprocal square root, of
  // max(|v|^2, e) with e = 1e-30 (FP32) or 1e-300 (FP64): at v = 0 the two
  // terms they scale (kappa |v| and kappa (v.pi) v/|v|) come out exactly 0
  // (|v|^2 and v.pi are 0, the reciprocal finite), and for |v|^2 < e each
  // differs from its exact value by less than kappa |pi| sqrt(e).
  template <typename T>
  __device__ static void speed_inv(const Par<T>& P, const T (&s)[6], T& knv, T& kinv) {
    const T ss = s[3] * s[3] + s[4] * s[4] + s[5] * s[5];
    const T e = sizeof(T) == 4 ? T(1e-30) : T(1e-300);
    kinv = P.kappa * M<T>::rsqrt(M<T>::fmax(ss, e));
    knv = ss * kinv;
  }

  // Velocity-costate factors of the p- and q-steps for the step lam = sigma
  // delta: 1/(1 + lam wP) and 1/(1 + lam wE) (constants of a point).
  template <typename T>
  __device__ static void dual_scales(const Par<T>& P, T lam, T& ip, T& iq) {
    ip = M<T>::div(T(1), T(1) + lam * P.wP);
    iq = M<T>::div(T(1), T(1) + lam * P.wE);
  }

  // p-step for node j: v -> p^{k+1}, with ip = 1/(1 + lam wP).  lam = 0 (and
  // ip = 1) leaves v unchanged: a node past N keeps p = 0.
  template <typename T>
  __device__ static void dual_p(const Par<T>& P, const T (&x)[6], T (&v)[6], T lam, T ip, CacheX<T>& C) {
    speed_inv(P, x, C.knv, C.kinv);
    const T lkn = lam * C.knv;
#pragma unroll
    for (int i = 0; i < 3; i++) {
      v[i] += lam * x[3 + i];
      v[3 + i] = (v[3 + i] - lkn * x[3 + i]) * ip;
    }
  }

  // q-step for node j, with iq = 1/(1 + lam wE).
  template <typename T>
  __device__ static void dual_q(const Par<T>& P, const T (&y)[6], T (&v)[6], T lam, T iq, CacheY<T>& C) {
    speed_inv(P, y, C.knv, C.kinv);
    const T lkn = lam * C.knv;
#pragma unroll
    for (int i = 0; i < 3; i++) {
      v[i] += lam * y[3 + i];
      v[3 + i] = (v[3 + i] - lkn * y[3 + i]) * iq;
    }
  }

  // J_F(s)^T pi with kappa |v| and kappa / |v| precomputed (the term
  // (v.pi) v/|v| is 0 at v = 0): velocity rows pi_i - kappa |v| pi_{3+i} -
  // kappa (v.pi)/|v| v_i, position rows 0.
  template <typename T>
  __device__ static void jft(const T (&s)[6], T knv, T kinv, const T (&pi)[6], T (&o)[6]) {
    const T vp = s[3] * pi[3] + s[4] * pi[4] + s[5] * pi[5];
    const T kw = vp * kinv;
#pragma unroll
    for (int i = 0; i < 3; i++) {
      o[i] = T(0);
      o[3 + i] = pi[i] - knv * pi[3 + i] - kw * s[3 + i];
    }
  }

  template <typename T>
  __device__ static void grad_x(const Par<T>&, const T (&x)[6], const T (&p)[6], const CacheX<T>& C, T (&g)[6]) {
    jft(x, C.knv, C.kinv, p, g);
#pragma unroll
    for (int i = 0; i < 6; i++) g[i] = -g[i];
  }

  template <typename T>
  __device__ static void grad_y(const Par<T>&, const T (&y)[6], const T (&q)[6], const CacheY<T>& C, T (&g)[6]) {
    jft(y, C.knv, C.kinv, q, g);
  }

  template <typename T>
  __device__ static T H(const Par<T>& P, const T (&x)[6], const T (&y)[6], const T (&p)[6], const T (&q)[6]) {
    const T kx = P.kappa * speed(x), ky = P.kappa * speed(y);
    T h = T(0);
#pragma unroll
    for (int i = 0; i < 3; i++) {
      h += -(p[i] * x[3 + i]) + p[3 + i] * kx * x[3 + i];
      h += q[i] * y[3 + i] - q[3 + i] * ky * y[3 + i];
      h += T(0.5) * P.wP * p[3 + i] * p[3 + i] - T(0.5) * P.wE * q[3 + i] * q[3 + i];
    }
    return h;
  }

  template <typename T>
  __device__ static void prox_x0(const Par<T>&, const T (&v)[6], const T (&y0)[6], T tau, T (&o)[6]) {
    const T w0 = v[0] - y0[0], w1 = v[1] - y0[1], w2 = v[2] - y0[2];
    const T ss = w0 * w0 + w1 * w1 + w2 * w2;
    const T scale = M<T>::fmax(T(1) - tau * M<T>::rsqrt(ss), T(0));
    o[0] = y0[0] + scale * w0;
    o[1] = y0[1] + scale * w1;
    o[2] = y0[2] + scale * w2;
    o[3] = v[3]; o[4] = v[4]; o[5] = v[5];
  }

  // Prox of -tau g(x0, .) at v: the position moves away from x0's by tau along
  // v - x0; where v's position equals x0's the direction is taken as the first
  // axis.  Branch-free.
  template <typename T>
  __device__ static void stretch_y0(const Par<T>&, const T (&v)[6], const T (&x0)[6], T tau, T (&o)[6]) {
    const T w0 = v[0] - x0[0], w1 = v[1] - x0[1], w2 = v[2] - x0[2];
    const T ss = w0 * w0 + w1 * w1 + w2 * w2;
    const bool nz = ss > T(0);
    const T scale = T(1) + (nz ? tau * M<T>::rsqrt(ss) : T(0));
    o[0] = x0[0] + scale * w0 + (nz ? T(0) : tau);
    o[1] = x0[1] + scale * w1;
    o[2] = x0[2] + scale * w2;
    o[3] = v[3]; o[4] = v[4]; o[5] = v[5];
  }

  template <typename T>
  __device__ static T g(const Par<T>& P, const T (&x0)[6], const T (&y0)[6]) {
    const T a = x0[0] - y0[0], b = x0[1] - y0[1], c = x0[2] - y0[2];
    return M<T>::sqrt(a * a + b * b + c * c) - P.r;
  }
};

// ===========================================================================
// Isaacs' game (section 6.3), d = 2: scalar x (minimiser) and y (maximiser),
// dynamics x' = 2 beta + sin(alpha), y' = -c(x,y) + cos(alpha), running cost
// 1, so H(x,y,p,q) = -c(x,y) q + 2|p| - sqrt(p^2 + q^2) - 1, taken by the
// game algorithms at the costate pair (p, -q):
//   c q + 2|p| - sqrt(p^2 + q^2) - 1.
// Bump speed c = b0 (1 + b1 exp(-b2 |(x,y) - (cx,cy)|^2)); hp = [b0,b1,b2,cx,cy].
// Convex-concave initial cost g = e(x) + h(y), e = (a x)^2/2 - c0,
// h = -(b y)^2/2; gp = [c0, a, b]; e*(p) = p^2/(2a^2) + c0, h_*(q) = -q^2/(2b^2).
// Built for the game Hopf formulation (Algorithm 4) only.  Costate steps
// (section 6.3): the root term is linearised at the current costates, the
// rest is solved exactly (a shrink for p, a linear step for q).
// ===========================================================================
struct Isaacs {
  static constexpr int D = 2;
  static constexpr int kWavesK[5] = {0, 4, 3, 2, 2};  // FP32 waves per SIMD by nodes per lane
  static constexpr int DX = 1, DY = 1;
  static constexpr bool kGame = true;
  static constexpr bool kZeroSafe = false;
  static constexpr bool kHopf = false;
  static constexpr bool kMix = false;
  static constexpr bool kGameHopf = true;  // Algorithm 4 (k_group_game_hopf)

  template <typename T> struct Par {
    T b0, b1, b2, cx, cy;
    T c0, ia2, ib2;  // c0, 1/a^2, 1/b^2
    T ea2, hb2;      // a^2, b^2 of the initial cost
  };

  template <typename T>
  __device__ static void load(Par<T>& P, const T* hp, const T* gp, int, T) {
    P.b0 = hp[0]; P.b1 = hp[1]; P.b2 = hp[2]; P.cx = hp[3]; P.cy = hp[4];
    P.c0 = gp[0];
    P.ea2 = gp[1] * gp[1];
    P.hb2 = gp[2] * gp[2];
    P.ia2 = T(1) / P.ea2;
    P.ib2 = T(1) / P.hb2;
  }

  // Algorithm 3's node 0: prox of tau e(x) = tau ((a x)^2/2 - c0) at v, and the
  // concave counterpart for y, prox of -tau h(y) = tau (b y)^2/2 at v.
  template <typename T>
  __device__ static T prox_e(const Par<T>& P, T v, T tau) { return M<T>::div(v, T(1) + tau * P.ea2); }
  template <typename T>
  __device__ static T prox_mh(const Par<T>& P, T v, T tau) { return M<T>::div(v, T(1) + tau * P.hb2); }

  // g(x_0, y_0) = e(x_0) + h(y_0) (Algorithm 3's value)
  template <typename T>
  __device__ static T g(const Par<T>& P, T x0, T y0) {
    return T(0.5) * P.ea2 * x0 * x0 - P.c0 - T(0.5) * P.hb2 * y0 * y0;
  }

  // c(x,y) and its partial derivatives.
  template <typename T>
  __device__ static T speed(const Par<T>& P, T x, T y, T& dcx, T& dcy) {
    const T rx = x - P.cx, ry = y - P.cy;
    const T be = P.b0 * P.b1 * M<T>::exp(-P.b2 * (rx * rx + ry * ry));
    dcx = T(-2) * P.b2 * rx * be;
    dcy = T(-2) * P.b2 * ry * be;
    return P.b0 + be;
  }

  // p-step: shrink_{2 sigma delta}(v + sigma delta p/|(p,q)|) at the current
  // (p, q); at the Hopf node 1 the e* quadratic scales both by 1/(1 + sigma/a^2).
  template <typename T>
  __device__ static T dual_p(const Par<T>& P, T p, T q, T v, T sd, T sigma, bool first) {
    const T ss = p * p + q * q;
    const T g = ss > T(0) ? p * M<T>::rsqrt(ss) : T(0);
    T vv = v + sd * g, lam = T(2) * sd;
    if (first) {
      const T r = M<T>::div(T(1), T(1) + sigma * P.ia2);
      vv *= r;
      lam *= r;
    }
    const T m = M<T>::fabs_(vv) - lam;
    return m > T(0) ? (vv > T(0) ? m : -m) : T(0);
  }

  // q-step with the new p: u + sigma delta c - sigma delta q/|(p,q)|; at the
  // Hopf node 1 the h_* quadratic divides by 1 + sigma/b^2.
  template <typename T>
  __device__ static T dual_q(const Par<T>& P, T c, T p, T q, T u, T sd, T sigma, bool first) {
    const T ss = p * p + q * q;
    const T g = ss > T(0) ? q * M<T>::rsqrt(ss) : T(0);
    const T uu = u + sd * c - sd * g;
    return first ? M<T>::div(uu, T(1) + sigma * P.ib2) : uu;
  }

  // H at the costate pair (p, -q).
  template <typename T>
  __device__ static T H(T c, T p, T q) {
    return c * q + T(2) * M<T>::fabs_(p) - M<T>::sqrt(p * p + q * q) - T(1);
  }

  // -e*(p_1) - h_*(-q_1).
  template <typename T>
  __device__ static T conj_terms(const Par<T>& P, T p1, T q1) {
    return -(T(0.5) * p1 * p1 * P.ia2 + P.c0) + T(0.5) * q1 * q1 * P.ib2;
  }
};

}  // namespace hjpd
