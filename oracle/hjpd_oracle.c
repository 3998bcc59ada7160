/*
 * hjpd oracle — TEST INFRASTRUCTURE ONLY.
 *
 * A plain, sequential, double-precision CPU implementation of the per-point
 * primal-dual splitting method of Lin, Chow and Osher (arXiv 1803.01215) for
 * Hamilton-Jacobi equations with state-dependent Hamiltonians.  It exists to
 * check the GPU library; nothing in the product path may link, load or call
 * it.  It shares no code with the GPU library: the two were written
 * separately from the paper.  Only tests/, the smoke check and the CPU
 * baseline leg of the benchmark use it.
 *
 * What is computed (section 4.1, eq. disclaxBE; section 5.1, Algorithm 1 and
 * its step-by-step version in Appendix A.1.1):
 *
 *   phi(x,t) ~ max_{p_1..p_N} min_{x_0..x_{N-1}}  g(x_0)
 *              + sum_{j=1..N} <p_j, x_j - x_{j-1}> - delta sum_{j=1..N} H(x_j,p_j,s_j)
 *
 * with x_N = x, delta = t/N, s_j = j delta, solved by the PDHG-type iteration
 *
 *   p_j   <- prox_{sigma delta H(x_j,.,s_j)}( p_j + sigma (z_j - z_{j-1}) ),  j = 1..N
 *   x_0   <- prox_{tau g}( x_0 + tau p_1 )
 *   x_j   <- x_j - tau (p_j - p_{j+1}) + tau delta grad_x H(x_j, p_j, s_j),  j = 1..N-1
 *   z     <- x_new + theta (x_new - x_old)
 *
 * (section 5.3 for "prox on the nonsmooth part, one gradient step on the
 * smooth part").
 *
 * Hopf formulation (section 4.1, eq. dischopf; section 5.1, Algorithm 2 and
 * Appendix A.1.2), control path, convex g:
 *
 *   phi(x,t) ~ max_{p_1..p_N} min_{x_1..x_{N-1}}  -g*(p_1) + <p_N, x>
 *              + sum_{j=1..N-1} <p_j - p_{j+1}, x_j> - delta sum_{j=1..N} H(x_j,p_j,s_j)
 *
 * with x_N = x and no node 0; the dual step at j = 1 is the joint prox of
 * g* + delta H(x_1,.), at j >= 2 the prox of delta H(x_j,.), both around
 * p_j + sigma (z_j - z_{j-1}) with z_0 = 0 (the Hopf difference matrix);
 * the x-steps are those of the Lax path.
 *
 * Forward Euler and trapezoidal discretisations (section 4.1, eq.
 * disclaxFE; the remark after Algorithm 1 that averaging the forward and
 * backward Euler approximations gives a trapezoidal rule), eikonal and
 * quadrotor families.
 * Writing p_j for the costate of the interval (j-1, j), j = 1..N, all three
 * discretisations are one saddle problem
 *
 *   g(x_0) + sum_{j=1..N} <p_j, x_j - x_{j-1}>
 *          - delta sum_{j=1..N} [ wl H(x_{j-1},p_j,s_{j-1}) + wr H(x_j,p_j,s_j) ]
 *
 * with weights (wl, wr) = (0, 1) backward Euler (eq. disclaxBE), (1, 0)
 * forward Euler (eq. disclaxFE, whose p_j is p_{j+1} here) and (1/2, 1/2)
 * trapezoid (the average of the two Hamiltonian sums).  The iteration keeps
 * Algorithm 1's pattern; x_0, which now meets both g and H, takes a
 * proximal-gradient step (section 5.3: gradient step on the smooth part,
 * prox on the nonsmooth part):
 *
 *   p_j <- argmin_p sigma delta (wl H(x_{j-1},p) + wr H(x_j,p)) + |p - (p_j + sigma (z_j - z_{j-1}))|^2/2
 *   x_0 <- prox_{tau g}( x_0 + tau p_1 + tau delta wl grad_x H(x_0, p_1) )
 *   x_j <- x_j - tau (p_j - p_{j+1}) + tau delta (wr grad_x H(x_j,p_j) + wl grad_x H(x_j,p_{j+1}))
 *
 * For H = c(x)|p| the p-step is a shrink by sigma delta (wl c(x_{j-1}) + wr c(x_j)).
 * For the quadrotor H is quadratic in p, and so is the weighted sum: the
 * p-step is one linear solve, (I + lam (wl b_{j-1} b_{j-1}^T + wr b_j b_j^T))
 * in the velocity costate, the drift terms weighted, the body-rate costate
 * scaled as in Algorithm 1 (its quadratic does not depend on x).
 *
 * Game Hopf formulation (section 4.2, eq. discgenlaxhopfdghopf; Algorithm 4)
 * for a separable convex-concave g(x,y) = e(x) + h(y), with e* the convex
 * and h_* the concave conjugate:
 *
 *   phi ~ min_q max_p min_{x_1..x_{N-1}} max_{y_1..y_{N-1}}  -e*(p_1) - h_*(-q_1)
 *         + <p_N, x> - <q_N, y> + sum_{j<N} (<p_j - p_{j+1}, x_j> - <q_j - q_{j+1}, y_j>)
 *         - delta sum_j H(x_j, y_j, p_j, -q_j)
 *
 * built for Isaacs' game of section 6.3 (see the family's block below),
 * together with Algorithm 3 for the same game so that the two formulations
 * can be compared.  The costate updates follow section 6.3: a shrink for p
 * after a gradient step on the smooth part, a gradient step for q (the
 * linear and quadratic parts are kept exact); x and y take one descent /
 * ascent step each, y after x.
 *
 * Robustness recipes (section 6, remarks on slow points), control path and
 * the pursuit-evasion game (Algorithm 3; section 6.2 applies the first two
 * to a game):
 *  - on reaching the iteration cap, continue from the current iterate with
 *    sigma raised by sigma_inc and tau = sigma0 tau0 / sigma, at most
 *    `restarts` times (sigma_inc = 0 is the plain rerun);
 *  - after the first cap, also stop when the value changes by at most
 *    value_tol max(|value|, 1) between consecutive iterations;
 *  - control path only: `starts` random starts (seed, seed+1, ...); the
 *    reported point is the lowest value among the starts that stopped by a
 *    tolerance rule, else the lowest finite value, ties to the earlier start.
 *
 * The two-player game path follows section 4.2, eq.
 * discgenlaxhopfdg, and Algorithm 3 / Appendix A.2.1: blocks p, q, x, y in
 * that order, with the evader's costate entering H as -q.
 *
 * Readings taken where the paper is silent or inconsistent:
 *  - N counts intervals: nodes 0..N, delta = t/N (Appendix A.1.1).
 *  - The p-prox is evaluated at the current x_j (Algorithm 1, Appendix A).
 *  - The x-step uses the new p (standard Chambolle-Pock, section 3.2).
 *  - x_j (j>=1) takes one explicit gradient step; x_0 takes the exact prox
 *    of g, which is closed form for every initial cost here.
 *  - Stopping: ||x^{k+1}-x^k||_2^2 < tol and ||p^{k+1}-p^k||_2^2 < tol over
 *    the stacked vectors (section 6 set-up; games add the y and q blocks).
 *  - The returned value is the Lagrangian at the last iterate (Algorithm 1).
 *  - Hamiltonians of the quadrotor, pursuit-evasion and linear-tanh families
 *    are given by the caller in the physical, terminal-value convention
 *    H_c = min_u {<f,p> + L} (section 2.1).  The algorithms use the
 *    initial-value (time-reversed) convention H = max_u {<f,p> - L} of
 *    the same section; reversing time turns f into -f, so H = -H_c.  The
 *    eikonal family is already in the paper's convention.
 *  - Initialisation (section 6 set-up): every free coordinate of x_j (j<N)
 *    is x + U[-0.1,0.1], every coordinate of p_j (j>=1) is U[-0.1,0.1],
 *    p_0 = 0, z = x.  The uniform numbers come from a counter-based
 *    SplitMix64 stream (Steele, Lea, Flood 2014) indexed by
 *    (point, array, node, coordinate).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/*
 * Rounding variants.  The default build evaluates everything in binary64 with
 * no fused multiply-add.  The same source is also compiled
 *  - with FMA contraction (-mfma -ffp-contract=fast): the same arithmetic with
 *    another rounding sequence;
 *  - with OR_BINARY32 (and -fsingle-precision-constant): every floating-point
 *    variable, argument and constant below becomes binary32, so every
 *    operation rounds to binary32 (libm transcendentals are evaluated in
 *    binary64 and rounded on assignment), with and without FMA contraction.
 * These variants compute nothing new.  They measure how far a second rounding
 * sequence of the same iteration, or any binary32 evaluation of it, lands
 * from this binary64 one after the same number of iterations: the rounding
 * floor below which no implementation's agreement with the oracle can be
 * expected at a given point.  (The macro is defined after the standard
 * headers, so their declarations keep binary64.)
 */
#ifdef OR_BINARY32
#define double float
#endif

/* Family ids: identical numbering to the public header, restated here. */
enum { OR_H_CNORM = 0, OR_H_QUADROTOR = 1, OR_H_PURSUIT_EVASION = 2, OR_H_LINEAR_TANH = 3, OR_H_ISAACS = 4 };
enum { OR_G_NORM = 0, OR_G_QUAD_SHIFT = 1, OR_G_PAIR_DIST = 2, OR_G_QUAD_FORM = 3, OR_G_SADDLE_QUAD = 4 };
enum { OR_PT_CONVERGED = 0, OR_PT_MAXITER = 1, OR_PT_NONFINITE = 2, OR_PT_BADINPUT = 3, OR_PT_VALUE_STALLED = 4 };
enum { OR_ARR_X = 0, OR_ARR_P = 1, OR_ARR_Y = 2, OR_ARR_Q = 3 };

typedef struct {
    int H, g;          /* family ids */
    int d;             /* full state dimension */
    int d_y;           /* > 0: game; x has d - d_y coordinates, y has d_y */
    const double *hp;  /* Hamiltonian parameters */
    const double *gp;  /* initial-cost parameters */
} or_problem;

/* ------------------------------------------------------------------ */
/* Counter-based uniform numbers for the random start (section 6).    */
/* ------------------------------------------------------------------ */

/* SplitMix64 output function (Steele, Lea, Flood 2014). */
uint64_t or_splitmix64_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* k-th output (k >= 1) of the SplitMix64 stream whose state starts at seed. */
uint64_t or_splitmix64_at(uint64_t seed, uint64_t k)
{
    return or_splitmix64_mix(seed + k * 0x9E3779B97F4A7C15ULL);
}

/* U[-0.1, 0.1] start perturbation of coordinate i of node j of one array. */
double or_init_noise(uint64_t seed, uint64_t point, int arr, int j, int i)
{
    uint64_t c = (point << 22) | ((uint64_t)arr << 20) | ((uint64_t)j << 10) | (uint64_t)i;
    uint64_t r = or_splitmix64_at(seed, c + 1);
    double u = (double)(r >> 11) * (1.0 / 9007199254740992.0); /* 2^-53 */
    return 0.2 * u - 0.1;
}

/* ------------------------------------------------------------------ */
/* Small vector helpers.                                              */
/* ------------------------------------------------------------------ */

static double dot(const double *a, const double *b, int n)
{
    double s = 0.0;
    for (int i = 0; i < n; i++) s += a[i] * b[i];
    return s;
}

static double norm2(const double *a, int n) { return sqrt(dot(a, a, n)); }

/* shrink_2(v, lam) = v max(||v|| - lam, 0)/||v||, 0 at v = 0: the prox of
 * lam ||.||_2 (section 6.1.2). */
void or_shrink2(const double *v, double lam, int n, double *out)
{
    double nv = norm2(v, n);
    double s = (nv > 0.0) ? fmax(nv - lam, 0.0) / nv : 0.0;
    for (int i = 0; i < n; i++) out[i] = s * v[i];
}

/* ------------------------------------------------------------------ */
/* Eikonal family: H(x,p) = c(x) ||p||, c(x) = 1 + alpha sin(x_1) cos(x_2) */
/* (section 6.1: H^+ = c(x)||p||, arising from f = c(x)u, ||u|| <= 1).  */
/* ------------------------------------------------------------------ */

static double cnorm_c(const double *hp, const double *x)
{
    return 1.0 + hp[0] * sin(x[0]) * cos(x[1]);
}

static void cnorm_grad_c(const double *hp, const double *x, int d, double *gc)
{
    for (int i = 0; i < d; i++) gc[i] = 0.0;
    gc[0] = hp[0] * cos(x[0]) * cos(x[1]);
    gc[1] = -hp[0] * sin(x[0]) * sin(x[1]);
}

/* ------------------------------------------------------------------ */
/* Quadrotor-like family, d = 12.  State (r, v, eta, omega):           */
/* position, velocity, Euler angles (roll phi, pitch th, yaw psi), body */
/* rates.  Physical dynamics f = f0(x) + B(x) u with                   */
/*   f0 = (v, -g_z e3, W(eta) omega, 0),                              */
/*   B u = (0, (u_1/m) R(eta) e3, 0, J^{-1} u_{2:4}),                 */
/* R = Rz(psi) Ry(th) Rx(phi) (so R e3 is the thrust direction of the   */
/* paper's quadcopter, section 6.4), running cost |u|^2/2.             */
/* Terminal-value H_c = <p,f0> - |B^T p|^2 / 2; the algorithm uses     */
/* H = -H_c = -<p,f0> + ((b.p_v)^2 + sum_i (p_w,i / J_i)^2) / 2,        */
/* b = R e3 / m.  The pitch inside the Euler-rate matrix W is clamped   */
/* to [-c, c] (part of the problem definition; zero slope outside).    */
/* hp = [m, J1, J2, J3, g_z, c].                                       */
/* ------------------------------------------------------------------ */

static double clampd(double a, double lo, double hi) { return a < lo ? lo : (a > hi ? hi : a); }

/* Thrust direction b = R(eta) e3 / m and its partials d b / d(phi,th,psi). */
static void quad_b(const double *hp, const double *x, double b[3], double db[3][3])
{
    double m = hp[0];
    double ph = x[6], th = x[7], ps = x[8];
    double sf = sin(ph), cf = cos(ph), st = sin(th), ct = cos(th), ss = sin(ps), cs = cos(ps);
    b[0] = (cs * st * cf + ss * sf) / m;
    b[1] = (ss * st * cf - cs * sf) / m;
    b[2] = (ct * cf) / m;
    if (db) {
        /* d/dphi */
        db[0][0] = (-cs * st * sf + ss * cf) / m;
        db[0][1] = (-ss * st * sf - cs * cf) / m;
        db[0][2] = (-ct * sf) / m;
        /* d/dth */
        db[1][0] = (cs * ct * cf) / m;
        db[1][1] = (ss * ct * cf) / m;
        db[1][2] = (-st * cf) / m;
        /* d/dpsi */
        db[2][0] = (-ss * st * cf + cs * sf) / m;
        db[2][1] = (cs * st * cf + ss * sf) / m;
        db[2][2] = 0.0;
    }
}

/* Euler-rate matrix W(phi, th) (ZYX convention) with th clamped, and
 * d W / d phi, d W / d th (the latter zero outside the clamp). */
static void quad_W(const double *hp, const double *x, double W[3][3], double dWf[3][3], double dWt[3][3])
{
    double c = hp[5];
    double ph = x[6], th_raw = x[7];
    double th = clampd(th_raw, -c, c);
    int inside = (th_raw > -c) && (th_raw < c);
    double sf = sin(ph), cf = cos(ph), tt = tan(th), ct = cos(th), sec = 1.0 / ct;
    W[0][0] = 1.0; W[0][1] = sf * tt;  W[0][2] = cf * tt;
    W[1][0] = 0.0; W[1][1] = cf;       W[1][2] = -sf;
    W[2][0] = 0.0; W[2][1] = sf * sec; W[2][2] = cf * sec;
    if (dWf) {
        dWf[0][0] = 0.0; dWf[0][1] = cf * tt;  dWf[0][2] = -sf * tt;
        dWf[1][0] = 0.0; dWf[1][1] = -sf;      dWf[1][2] = -cf;
        dWf[2][0] = 0.0; dWf[2][1] = cf * sec; dWf[2][2] = -sf * sec;
    }
    if (dWt) {
        double k = inside ? 1.0 : 0.0;
        /* d tan = sec^2, d sec = sec tan */
        dWt[0][0] = 0.0; dWt[0][1] = k * sf * sec * sec; dWt[0][2] = k * cf * sec * sec;
        dWt[1][0] = 0.0; dWt[1][1] = 0.0;                dWt[1][2] = 0.0;
        dWt[2][0] = 0.0; dWt[2][1] = k * sf * sec * tt;  dWt[2][2] = k * cf * sec * tt;
    }
}

static double quad_H(const double *hp, const double *x, const double *p)
{
    const double *v = x + 3, *w = x + 9;
    const double *pr = p, *pv = p + 3, *pe = p + 6, *pw = p + 9;
    double W[3][3], b[3];
    quad_W(hp, x, W, NULL, NULL);
    quad_b(hp, x, b, NULL);
    double drift = dot(pr, v, 3) - hp[4] * pv[2];
    for (int a = 0; a < 3; a++)
        for (int c = 0; c < 3; c++) drift += pe[a] * W[a][c] * w[c];
    double bp = dot(b, pv, 3);
    double ctrl = bp * bp;
    for (int i = 0; i < 3; i++) ctrl += (pw[i] / hp[1 + i]) * (pw[i] / hp[1 + i]);
    return -drift + 0.5 * ctrl;
}

/* argmin_p lam H(x,p) + |p - v|^2 / 2 */
static void quad_prox_p(const double *hp, const double *x, const double *v, double lam, double *p)
{
    const double *vel = x + 3, *w = x + 9;
    double W[3][3], b[3];
    quad_W(hp, x, W, NULL, NULL);
    quad_b(hp, x, b, NULL);
    /* position costate: linear term -lam <p_r, vel> */
    for (int i = 0; i < 3; i++) p[i] = v[i] + lam * vel[i];
    /* angle costate: linear term -lam <p_eta, W omega> */
    for (int a = 0; a < 3; a++) {
        double Ww = 0.0;
        for (int c = 0; c < 3; c++) Ww += W[a][c] * w[c];
        p[6 + a] = v[6 + a] + lam * Ww;
    }
    /* velocity costate: (I + lam b b^T) p_v = v_v - lam g_z e3 (Sherman-Morrison) */
    double wv[3] = { v[3], v[4], v[5] - lam * hp[4] };
    double bw = dot(b, wv, 3), bb = dot(b, b, 3);
    double coef = lam * bw / (1.0 + lam * bb);
    for (int i = 0; i < 3; i++) p[3 + i] = wv[i] - coef * b[i];
    /* body-rate costate: (1 + lam / J_i^2) p = v */
    for (int i = 0; i < 3; i++) p[9 + i] = v[9 + i] / (1.0 + lam / (hp[1 + i] * hp[1 + i]));
}

/* argmin_p lam (wl H(xa,p) + wr H(xb,p)) + |p - v|^2 / 2: the weighted
 * Hamiltonians are quadratic in p, so the minimiser solves one linear
 * system, written out here block by block (the 3 x 3 velocity block by
 * Gaussian elimination; it is symmetric positive definite). */
static void quad_prox_p_mix(const double *hp, const double *xa, const double *xb, double wl, double wr,
                            const double *v, double lam, double *p)
{
    double Wa[3][3], Wb[3][3], ba[3], bb[3];
    quad_W(hp, xa, Wa, NULL, NULL);
    quad_W(hp, xb, Wb, NULL, NULL);
    quad_b(hp, xa, ba, NULL);
    quad_b(hp, xb, bb, NULL);
    /* position costate: linear terms -lam (wl <p_r, v_a> + wr <p_r, v_b>) */
    for (int i = 0; i < 3; i++) p[i] = v[i] + lam * (wl * xa[3 + i] + wr * xb[3 + i]);
    /* angle costate: linear terms -lam (wl <p_eta, W_a omega_a> + wr <p_eta, W_b omega_b>) */
    for (int r = 0; r < 3; r++) {
        double wa = 0.0, wb = 0.0;
        for (int c = 0; c < 3; c++) {
            wa += Wa[r][c] * xa[9 + c];
            wb += Wb[r][c] * xb[9 + c];
        }
        p[6 + r] = v[6 + r] + lam * (wl * wa + wr * wb);
    }
    /* velocity costate: (I + lam (wl ba ba^T + wr bb bb^T)) p_v = v_v - lam (wl + wr) g_z e3 */
    double A[3][4];
    for (int r = 0; r < 3; r++) {
        for (int c = 0; c < 3; c++) A[r][c] = (r == c ? 1.0 : 0.0) + lam * (wl * ba[r] * ba[c] + wr * bb[r] * bb[c]);
        A[r][3] = v[3 + r] - (r == 2 ? lam * (wl + wr) * hp[4] : 0.0);
    }
    for (int c = 0; c < 3; c++)
        for (int r = c + 1; r < 3; r++) {
            double f = A[r][c] / A[c][c];
            for (int k = c; k < 4; k++) A[r][k] -= f * A[c][k];
        }
    for (int r = 2; r >= 0; r--) {
        double s2 = A[r][3];
        for (int c = r + 1; c < 3; c++) s2 -= A[r][c] * p[3 + c];
        p[3 + r] = s2 / A[r][r];
    }
    /* body-rate costate: (1 + lam (wl + wr) / J_i^2) p = v */
    for (int i = 0; i < 3; i++) p[9 + i] = v[9 + i] / (1.0 + lam * (wl + wr) / (hp[1 + i] * hp[1 + i]));
}

static void quad_grad_x(const double *hp, const double *x, const double *p, double *gx)
{
    const double *w = x + 9;
    const double *pr = p, *pv = p + 3, *pe = p + 6;
    double W[3][3], dWf[3][3], dWt[3][3], b[3], db[3][3];
    quad_W(hp, x, W, dWf, dWt);
    quad_b(hp, x, b, db);
    double bp = dot(b, pv, 3);
    for (int i = 0; i < 12; i++) gx[i] = 0.0;
    /* d/dr = 0; d/dv of -<p_r, v> */
    for (int i = 0; i < 3; i++) gx[3 + i] = -pr[i];
    /* d/deta: -p_eta . (dW omega) + (b.p_v) (db . p_v) */
    double dwf = 0.0, dwt = 0.0;
    for (int a = 0; a < 3; a++)
        for (int c = 0; c < 3; c++) {
            dwf += pe[a] * dWf[a][c] * w[c];
            dwt += pe[a] * dWt[a][c] * w[c];
        }
    gx[6] = -dwf + bp * dot(db[0], pv, 3);
    gx[7] = -dwt + bp * dot(db[1], pv, 3);
    gx[8] = bp * dot(db[2], pv, 3);
    /* d/domega: -W^T p_eta */
    for (int c = 0; c < 3; c++) {
        double s = 0.0;
        for (int a = 0; a < 3; a++) s += W[a][c] * pe[a];
        gx[9 + c] = -s;
    }
}

/* ------------------------------------------------------------------ */
/* Pursuit-evasion game, d = 12: pursuer x = (r_P, v_P) (minimiser),    */
/* evader y = (r_E, v_E) (maximiser), each a 3-D point mass with drag  */
/* F(r, v) = (v, -kappa |v| v) plus its control on the velocity.       */
/* Terminal-value H_c(X,P) = <P,F0(X)> - wP |P_vP|^2/2 + wE |P_vE|^2/2 */
/* (pursuer cost |u_P|^2/2, evader reward |u_E|^2/(2 wE)).             */
/* Paper convention H = -H_c, evaluated at the full costate P = (p,-q)  */
/* (section 4.2):                                                       */
/*   H(x,y,p,q) = -<p,F(x)> + <q,F(y)> + wP |p_v|^2/2 - wE |q_v|^2/2.   */
/* hp = [kappa, wP, wE].                                               */
/* ------------------------------------------------------------------ */

static void pe_F(double kappa, const double *s, double *F)
{
    const double *v = s + 3;
    double nv = norm2(v, 3);
    for (int i = 0; i < 3; i++) { F[i] = v[i]; F[3 + i] = -kappa * nv * v[i]; }
}

/* J_F(s)^T pi for F(r,v) = (v, -kappa |v| v):
 * (0, pi_r - kappa (|v| pi_v + (v.pi_v) v / |v|)); the last term is 0 at v = 0. */
static void pe_JFt(double kappa, const double *s, const double *pi, double *out)
{
    const double *v = s + 3;
    double nv = norm2(v, 3), vp = dot(v, pi + 3, 3);
    for (int i = 0; i < 3; i++) {
        out[i] = 0.0;
        out[3 + i] = pi[i] - kappa * (nv * pi[3 + i] + (nv > 0.0 ? vp * v[i] / nv : 0.0));
    }
}

/* H in the game variables (x, y, p, q), i.e. H_paper((x,y),(p,-q)). */
static double pe_H(const double *hp, const double *x, const double *y, const double *p, const double *q)
{
    double Fx[6], Fy[6];
    pe_F(hp[0], x, Fx);
    pe_F(hp[0], y, Fy);
    return -dot(p, Fx, 6) + dot(q, Fy, 6) + 0.5 * hp[1] * dot(p + 3, p + 3, 3) - 0.5 * hp[2] * dot(q + 3, q + 3, 3);
}

/* argmin_p lam H(x,y,p,q) + |p - v|^2/2 (H convex in p) */
static void pe_prox_p(const double *hp, const double *x, const double *v, double lam, double *p)
{
    double Fx[6];
    pe_F(hp[0], x, Fx);
    for (int i = 0; i < 3; i++) p[i] = v[i] + lam * Fx[i];
    for (int i = 0; i < 3; i++) p[3 + i] = (v[3 + i] + lam * Fx[3 + i]) / (1.0 + lam * hp[1]);
}

/* argmin_q -lam H(x,y,p,q) + |q - v|^2/2 (-H convex in q) */
static void pe_prox_q(const double *hp, const double *y, const double *v, double lam, double *q)
{
    double Fy[6];
    pe_F(hp[0], y, Fy);
    for (int i = 0; i < 3; i++) q[i] = v[i] + lam * Fy[i];
    for (int i = 0; i < 3; i++) q[3 + i] = (v[3 + i] + lam * Fy[3 + i]) / (1.0 + lam * hp[2]);
}

/* grad_x H = -J_F(x)^T p ; grad_y H = +J_F(y)^T q */
static void pe_grad_x(const double *hp, const double *x, const double *p, double *g)
{
    pe_JFt(hp[0], x, p, g);
    for (int i = 0; i < 6; i++) g[i] = -g[i];
}

static void pe_grad_y(const double *hp, const double *y, const double *q, double *g)
{
    pe_JFt(hp[0], y, q, g);
}

/* ------------------------------------------------------------------ */
/* Linear-tanh family: physical f = A x + eps tanh(x) + u, cost |u|^2/2, */
/* H_c = <p, A x + eps tanh x> - |p|^2/2; paper convention             */
/* H = -<p, A x + eps tanh x> + |p|^2/2.  hp = [eps, A (d x d, row-major)]. */
/* ------------------------------------------------------------------ */

static void lt_f(const double *hp, int d, const double *x, double *f)
{
    const double *A = hp + 1;
    for (int a = 0; a < d; a++) {
        double s = 0.0;
        for (int c = 0; c < d; c++) s += A[a * d + c] * x[c];
        f[a] = s + hp[0] * tanh(x[a]);
    }
}

static double lt_H(const double *hp, int d, const double *x, const double *p)
{
    double *f = malloc(sizeof(double) * d);
    lt_f(hp, d, x, f);
    double h = -dot(p, f, d) + 0.5 * dot(p, p, d);
    free(f);
    return h;
}

static void lt_prox_p(const double *hp, int d, const double *x, const double *v, double lam, double *p)
{
    double *f = malloc(sizeof(double) * d);
    lt_f(hp, d, x, f);
    for (int i = 0; i < d; i++) p[i] = (v[i] + lam * f[i]) / (1.0 + lam);
    free(f);
}

/* grad_x H = -(A^T p + eps (1 - tanh^2 x) * p) */
static void lt_grad_x(const double *hp, int d, const double *x, const double *p, double *g)
{
    const double *A = hp + 1;
    for (int c = 0; c < d; c++) {
        double s = 0.0;
        for (int a = 0; a < d; a++) s += A[a * d + c] * p[a];
        double th = tanh(x[c]);
        g[c] = -(s + hp[0] * (1.0 - th * th) * p[c]);
    }
}

/* ------------------------------------------------------------------ */
/* Isaacs' game (section 6.3, an unnamed example of Isaacs), d = 2:    */
/* scalar x (first player) and y (second player), dynamics             */
/* x' = 2 beta + sin(alpha), y' = -c(x,y) + cos(alpha), running cost 1, */
/* so that H(x,y,p,q) = -c(x,y) q + 2|p| - sqrt(p^2 + q^2) - 1 (the    */
/* section's closed form of the min-max over the controls).  Bump speed */
/* c(x,y) = b0 (1 + b1 exp(-b2 ((x - cx)^2 + (y - cy)^2)));            */
/* hp = [b0, b1, b2, cx, cy] (section 6.3: 2, 3, 4, 1, 1).  Initial    */
/* cost g = e(x) + h(y), e(x) = (a x)^2/2 - c0 convex, h(y) = -(b y)^2/2 */
/* concave; gp = [c0, a, b] (section 6.3: 1/2, 2.5, 1).                 */
/* ------------------------------------------------------------------ */

static double isaacs_c(const double *hp, double x, double y, double *cx, double *cy)
{
    double rx = x - hp[3], ry = y - hp[4];
    double e = exp(-hp[2] * (rx * rx + ry * ry));
    if (cx) *cx = hp[0] * hp[1] * e * (-2.0 * hp[2] * rx);
    if (cy) *cy = hp[0] * hp[1] * e * (-2.0 * hp[2] * ry);
    return hp[0] * (1.0 + hp[1] * e);
}

/* H(x, y, p, q) as defined above (callers pass the costate pair (p, -q)). */
double or_isaacs_H(const double *hp, double x, double y, double p, double q)
{
    return -isaacs_c(hp, x, y, NULL, NULL) * q + 2.0 * fabs(p) - sqrt(p * p + q * q) - 1.0;
}

/* e*(p) = sup_x p x - e(x) = p^2/(2 a^2) + c0. */
double or_saddle_estar(const double *gp, double p) { return p * p / (2.0 * gp[1] * gp[1]) + gp[0]; }

/* h_*(q) = inf_y q y - h(y) = -q^2/(2 b^2). */
double or_saddle_hstar(const double *gp, double q) { return -q * q / (2.0 * gp[2] * gp[2]); }

double or_saddle_g(const double *gp, double x, double y)
{
    return 0.5 * gp[1] * gp[1] * x * x - gp[0] - 0.5 * gp[2] * gp[2] * y * y;
}

static double shrink1(double v, double lam)
{
    double a = fabs(v) - lam;
    return a > 0.0 ? (v > 0.0 ? a : -a) : 0.0;
}

/* p-step at one node (maximisation over p of -delta H(x,y,p,-q) [- e*(p) at
 * the Hopf node 1] - |p - v|^2/(2 sigma)): the term +delta sqrt(p^2 + q^2)
 * is linearised at the current p (its gradient is taken as 0 at p = q = 0),
 * then the rest is solved exactly: a shrink by 2 sigma delta, scaled by
 * 1/(1 + sigma/a^2) when e* takes part. */
double or_isaacs_dual_p(const double *gp, double p_old, double q_old, double v, double sigma, double delta,
                        int first_hopf)
{
    double s = sqrt(p_old * p_old + q_old * q_old);
    double vv = v + sigma * delta * (s > 0.0 ? p_old / s : 0.0);
    if (!first_hopf) return shrink1(vv, 2.0 * sigma * delta);
    double r = 1.0 / (1.0 + sigma / (gp[1] * gp[1]));
    return shrink1(vv * r, 2.0 * sigma * delta * r);
}

/* q-step at one node (minimisation over q of -delta H(x,y,p,-q) [- h_*(-q)
 * at the Hopf node 1] + |q - u|^2/(2 sigma), with the new p): -delta H is
 * -delta c q + delta sqrt(p^2 + q^2) + const; the root term is linearised
 * at the current q, the linear and quadratic terms are exact. */
double or_isaacs_dual_q(const double *hp, const double *gp, double x, double y, double p_new, double q_old,
                        double u, double sigma, double delta, int first_hopf)
{
    double s = sqrt(p_new * p_new + q_old * q_old);
    double c = isaacs_c(hp, x, y, NULL, NULL);
    double uu = u + sigma * delta * c - sigma * delta * (s > 0.0 ? q_old / s : 0.0);
    return first_hopf ? uu / (1.0 + sigma / (gp[2] * gp[2])) : uu;
}

/* ------------------------------------------------------------------ */
/* Dispatch over the Hamiltonian families (control path).             */
/* ------------------------------------------------------------------ */

double or_H(const or_problem *pb, const double *x, const double *p, double s)
{
    (void)s;
    switch (pb->H) {
    case OR_H_CNORM: return cnorm_c(pb->hp, x) * norm2(p, pb->d);
    case OR_H_QUADROTOR: return quad_H(pb->hp, x, p);
    case OR_H_LINEAR_TANH: return lt_H(pb->hp, pb->d, x, p);
    case OR_H_PURSUIT_EVASION: {
        /* full state X = (x,y), full costate P = (p,-q) */
        double q[6];
        for (int i = 0; i < 6; i++) q[i] = -p[6 + i];
        return pe_H(pb->hp, x, x + 6, p, q);
    }
    }
    return NAN;
}

void or_grad_x_H(const or_problem *pb, const double *x, const double *p, double s, double *g)
{
    (void)s;
    int d = pb->d;
    switch (pb->H) {
    case OR_H_CNORM: {
        double np = norm2(p, d);
        cnorm_grad_c(pb->hp, x, d, g);
        for (int i = 0; i < d; i++) g[i] *= np;
        return;
    }
    case OR_H_QUADROTOR: quad_grad_x(pb->hp, x, p, g); return;
    case OR_H_LINEAR_TANH: lt_grad_x(pb->hp, d, x, p, g); return;
    case OR_H_PURSUIT_EVASION: {
        /* gradient of H_paper(X, P) in X: (-J_F(x)^T P_x, -J_F(y)^T P_y) */
        double gx[6], gy[6];
        pe_JFt(pb->hp[0], x, p, gx);
        pe_JFt(pb->hp[0], x + 6, p + 6, gy);
        for (int i = 0; i < 6; i++) { g[i] = -gx[i]; g[6 + i] = -gy[i]; }
        return;
    }
    }
}

/* argmin_p lam H(x,p,s) + |p - v|^2/2 for the control families. */
void or_prox_p(const or_problem *pb, const double *x, const double *v, double lam, double s, double *p)
{
    (void)s;
    switch (pb->H) {
    case OR_H_CNORM: or_shrink2(v, lam * cnorm_c(pb->hp, x), pb->d, p); return;
    case OR_H_QUADROTOR: quad_prox_p(pb->hp, x, v, lam, p); return;
    case OR_H_LINEAR_TANH: lt_prox_p(pb->hp, pb->d, x, v, lam, p); return;
    }
}

/* Game-path pieces, in the game variables (x, y, p, q). */
double or_game_H(const or_problem *pb, const double *x, const double *y, const double *p, const double *q)
{
    return pe_H(pb->hp, x, y, p, q);
}

void or_game_prox_p(const or_problem *pb, const double *x, const double *y, const double *q,
                    const double *v, double lam, double *p)
{
    (void)y; (void)q;
    pe_prox_p(pb->hp, x, v, lam, p);
}

void or_game_prox_q(const or_problem *pb, const double *x, const double *y, const double *p,
                    const double *v, double lam, double *q)
{
    (void)x; (void)p;
    pe_prox_q(pb->hp, y, v, lam, q);
}

void or_game_grad_x(const or_problem *pb, const double *x, const double *y, const double *p,
                    const double *q, double *g)
{
    (void)y; (void)q;
    pe_grad_x(pb->hp, x, p, g);
}

void or_game_grad_y(const or_problem *pb, const double *x, const double *y, const double *p,
                    const double *q, double *g)
{
    (void)x; (void)p;
    pe_grad_y(pb->hp, y, q, g);
}

/* ------------------------------------------------------------------ */
/* Initial costs g and their proximal maps.                           */
/* ------------------------------------------------------------------ */

/* Cholesky factor L of (I + tau Q_s), Q_s = (Q + Q^T)/2; lower, row-major. */
static int chol_I_tauQ(const double *Q, int d, double tau, double *L)
{
    for (int a = 0; a < d; a++)
        for (int c = 0; c < d; c++)
            L[a * d + c] = (a == c ? 1.0 : 0.0) + tau * 0.5 * (Q[a * d + c] + Q[c * d + a]);
    for (int c = 0; c < d; c++) {
        double s = L[c * d + c];
        for (int k = 0; k < c; k++) s -= L[c * d + k] * L[c * d + k];
        if (!(s > 0.0)) return -1;
        double lcc = sqrt(s);
        L[c * d + c] = lcc;
        for (int a = c + 1; a < d; a++) {
            double t = L[a * d + c];
            for (int k = 0; k < c; k++) t -= L[a * d + k] * L[c * d + k];
            L[a * d + c] = t / lcc;
        }
        for (int a = 0; a < c; a++) L[a * d + c] = 0.0;
    }
    return 0;
}

/* Solve L L^T out = v. */
static void chol_solve(const double *L, int d, const double *v, double *out)
{
    for (int a = 0; a < d; a++) {
        double s = v[a];
        for (int k = 0; k < a; k++) s -= L[a * d + k] * out[k];
        out[a] = s / L[a * d + a];
    }
    for (int a = d - 1; a >= 0; a--) {
        double s = out[a];
        for (int k = a + 1; k < d; k++) s -= L[k * d + a] * out[k];
        out[a] = s / L[a * d + a];
    }
}

double or_g(const or_problem *pb, const double *x0)
{
    int d = pb->d;
    switch (pb->g) {
    case OR_G_NORM: return norm2(x0, d) - pb->gp[0];
    case OR_G_QUAD_SHIFT: {
        double s = 0.0;
        for (int i = 0; i < d; i++) s += (x0[i] - pb->gp[1 + i]) * (x0[i] - pb->gp[1 + i]);
        return 0.5 * s - pb->gp[0];
    }
    case OR_G_QUAD_FORM: {
        const double *Q = pb->gp;
        double s = 0.0;
        for (int a = 0; a < d; a++)
            for (int c = 0; c < d; c++) s += x0[a] * 0.5 * (Q[a * d + c] + Q[c * d + a]) * x0[c];
        return 0.5 * s;
    }
    case OR_G_PAIR_DIST: {
        int dx = d - pb->d_y;
        double r[3] = { x0[0] - x0[dx], x0[1] - x0[dx + 1], x0[2] - x0[dx + 2] };
        return norm2(r, 3) - pb->gp[0];
    }
    }
    return NAN;
}

/* argmin_x tau g(x) + |x - v|^2/2 for the control path; `chol` is the
 * factor of I + tau Q_s for the quadratic form (else unused). */
static void prox_g(const or_problem *pb, const double *v, double tau, const double *chol, double *out)
{
    int d = pb->d;
    switch (pb->g) {
    case OR_G_NORM: or_shrink2(v, tau, d, out); return;
    case OR_G_QUAD_SHIFT:
        for (int i = 0; i < d; i++) out[i] = (v[i] + tau * pb->gp[1 + i]) / (1.0 + tau);
        return;
    case OR_G_QUAD_FORM: chol_solve(chol, d, v, out); return;
    }
}

/* Exported for tests: prox of tau g at v (builds its own factor). */
int or_prox_g(const or_problem *pb, const double *v, double tau, double *out)
{
    double *L = NULL;
    if (pb->g == OR_G_QUAD_FORM) {
        L = malloc(sizeof(double) * pb->d * pb->d);
        if (chol_I_tauQ(pb->gp, pb->d, tau, L)) { free(L); return -1; }
    }
    prox_g(pb, v, tau, L, out);
    free(L);
    return 0;
}

/* Convex conjugate g*(p) = sup_x <x,p> - g(x) (section 4.1, derivation of
 * eq. dischopf).  NORM: g = |x| - r gives g* = r on the unit ball, +inf
 * outside.  QUAD_SHIFT: g = |x - a|^2/2 - c0 gives g* = |p|^2/2 + <a,p> + c0.
 * Other initial costs: NAN (the Hopf path is not offered for them). */
double or_gstar(const or_problem *pb, const double *p)
{
    int d = pb->d;
    switch (pb->g) {
    case OR_G_NORM:
        /* the indicator of the unit ball; the slack covers the rounding of the clip that puts p on
         * the sphere, in the working precision (binary64, or the binary32 rounding variant) */
        return norm2(p, d) <= 1.0 + (sizeof(double) == 8 ? 1e-12 : 1e-5) ? pb->gp[0] : INFINITY;
    case OR_G_QUAD_SHIFT: return 0.5 * dot(p, p, d) + dot(pb->gp + 1, p, d) + pb->gp[0];
    }
    return NAN;
}

/* Hopf dual step at j = 1 (Algorithm 2; Appendix A.1.2):
 *   argmin_p  g*(p) + delta H(x_1, p, s_1) + |p - v|^2 / (2 sigma)
 *  - QUAD_SHIFT (any control family with a p-prox): sigma g*(p) + |p - v|^2/2
 *    = (1+sigma)/2 |p - w|^2 + const with w = (v - sigma a)/(1 + sigma), so p
 *    is the family's p-prox of w with step sigma delta/(1+sigma); for the
 *    eikonal family H = c(x)|p| that is shrink_2(w, sigma delta c/(1+sigma));
 *  - NORM, eikonal family: every term is a function of |p| along the
 *    direction of v, so p = v/|v| * clip(|v| - sigma delta c, 0, 1) (shrink,
 *    then the ball).
 * Returns -1 when the pair (H, g) has no Hopf step here. */
int or_hopf_prox1(const or_problem *pb, const double *x1, const double *v, double sigma, double delta,
                  double *out)
{
    int d = pb->d;
    if (pb->g == OR_G_QUAD_SHIFT && (pb->H == OR_H_CNORM || pb->H == OR_H_QUADROTOR)) {
        double *w = malloc(sizeof(double) * d);
        for (int i = 0; i < d; i++) w[i] = (v[i] - sigma * pb->gp[1 + i]) / (1.0 + sigma);
        or_prox_p(pb, x1, w, sigma * delta / (1.0 + sigma), delta, out);
        free(w);
        return 0;
    }
    if (pb->H != OR_H_CNORM) return -1;
    double c = cnorm_c(pb->hp, x1);
    if (pb->g == OR_G_NORM) {
        double nv = norm2(v, d);
        double r = nv - sigma * delta * c;
        if (r < 0.0) r = 0.0;
        if (r > 1.0) r = 1.0;
        for (int i = 0; i < d; i++) out[i] = nv > 0.0 ? v[i] / nv * r : 0.0;
        return 0;
    }
    return -1;
}

/* Game, node 0: pursuer block x0 <- argmin tau g(x, y0) + |x - v|^2/2 for
 * g = |r_P - r_E| - r: the position moves toward r_E by shrink_2, the
 * velocity is untouched (g does not depend on it). */
void or_game_prox_x0(const or_problem *pb, const double *v, const double *y0, double tau, double *out)
{
    int dx = pb->d - pb->d_y;
    double w[3] = { v[0] - y0[0], v[1] - y0[1], v[2] - y0[2] }, s[3];
    or_shrink2(w, tau, 3, s);
    for (int i = 0; i < 3; i++) out[i] = y0[i] + s[i];
    for (int i = 3; i < dx; i++) out[i] = v[i];
}

/* Game, node 0: evader block y0 <- argmin -tau g(x0, y) + |y - v|^2/2, the
 * prox of the concave -g ("stretch"): the position moves away from r_P by
 * tau; at v = r_P the direction e_1 is taken. */
void or_game_stretch_y0(const or_problem *pb, const double *v, const double *x0, double tau, double *out)
{
    int dy = pb->d_y;
    double w[3] = { v[0] - x0[0], v[1] - x0[1], v[2] - x0[2] };
    double nw = norm2(w, 3);
    if (nw > 0.0) {
        for (int i = 0; i < 3; i++) out[i] = x0[i] + w[i] * (1.0 + tau / nw);
    } else {
        out[0] = x0[0] + tau; out[1] = x0[1]; out[2] = x0[2];
    }
    for (int i = 3; i < dy; i++) out[i] = v[i];
}

/* ------------------------------------------------------------------ */
/* One query point: control path (Algorithm 1, Appendix A.1.1).       */
/* ------------------------------------------------------------------ */

typedef struct {
    double sigma, tau, theta, tol;
    int max_iter, fixed_iters;
    uint64_t seed;
    int N_max;
    int starts, restarts;        /* recipes (see the header comment); 1 and 0 = plain Algorithm 1 */
    double sigma_inc, value_tol;
} or_opts;

static int all_finite(const double *a, int n)
{
    for (int i = 0; i < n; i++)
        if (!isfinite(a[i])) return 0;
    return 1;
}

/* The value: the Lagrangian g(x_0) + sum_j <p_j, x_j - x_{j-1}> - delta sum_j H(x_j, p_j). */
static double control_value(const or_problem *pb, const double *x, const double *p, int N, double delta)
{
    int d = pb->d;
    double val = or_g(pb, x);
    for (int j = 1; j <= N; j++) {
        for (int i = 0; i < d; i++) val += p[j * d + i] * (x[j * d + i] - x[(j - 1) * d + i]);
        val -= delta * or_H(pb, &x[j * d], &p[j * d], j * delta);
    }
    return val;
}

/* One random start (seed) of Algorithm 1 with the cap/sigma recipe; x, p
 * (N+1 x d) receive the last iterate. */
static void control_run(const or_problem *pb, const or_opts *o, long pt, const double *xt, double t, int N,
                        uint64_t seed, double *x, double *p, double *phi, int *iters, int *status)
{
    int d = pb->d;
    double delta = t / N;
    size_t sz = (size_t)(N + 1) * d;
    double *z = calloc(sz, sizeof(double)), *xn = calloc(sz, sizeof(double)), *pn = calloc(sz, sizeof(double));
    double *v = calloc(d, sizeof(double)), *gr = calloc(d, sizeof(double));
    double sigma = o->sigma, tau = o->tau;
    const double st_product = o->sigma * o->tau;
    double *chol = NULL;
    if (pb->g == OR_G_QUAD_FORM) {
        chol = malloc(sizeof(double) * d * d);
        chol_I_tauQ(pb->gp, d, tau, chol);
    }

    /* random start (section 6 set-up) */
    memset(x, 0, sz * sizeof(double));
    memset(p, 0, sz * sizeof(double));
    for (int j = 0; j < N; j++)
        for (int i = 0; i < d; i++) x[j * d + i] = xt[i] + or_init_noise(seed, pt, OR_ARR_X, j, i);
    for (int i = 0; i < d; i++) x[N * d + i] = xt[i];
    for (int j = 1; j <= N; j++)
        for (int i = 0; i < d; i++) p[j * d + i] = or_init_noise(seed, pt, OR_ARR_P, j, i);
    memcpy(z, x, sz * sizeof(double));

    int k = 0, kp = 0, phase = 0, st = OR_PT_MAXITER;
    double prev_val = NAN;
    for (;;) {
        /* dual step: p_j <- prox_{sigma delta H(x_j,.)}(p_j + sigma (z_j - z_{j-1})) */
        for (int i = 0; i < d; i++) pn[i] = 0.0;
        for (int j = 1; j <= N; j++) {
            for (int i = 0; i < d; i++) v[i] = p[j * d + i] + sigma * (z[j * d + i] - z[(j - 1) * d + i]);
            or_prox_p(pb, &x[j * d], v, sigma * delta, j * delta, &pn[j * d]);
        }
        /* node 0: x_0 <- prox_{tau g}(x_0 - tau (D^T p)_0), (D^T p)_0 = -p_1 */
        for (int i = 0; i < d; i++) v[i] = x[i] + tau * pn[d + i];
        prox_g(pb, v, tau, chol, xn);
        /* nodes 1..N-1: one gradient step on -delta H plus the coupling term */
        for (int j = 1; j < N; j++) {
            or_grad_x_H(pb, &x[j * d], &pn[j * d], j * delta, gr);
            for (int i = 0; i < d; i++)
                xn[j * d + i] = x[j * d + i] - tau * (pn[j * d + i] - pn[(j + 1) * d + i]) + tau * delta * gr[i];
        }
        for (int i = 0; i < d; i++) xn[N * d + i] = x[N * d + i];

        double rx = 0.0, rp = 0.0;
        for (size_t a = 0; a < sz; a++) {
            rx += (xn[a] - x[a]) * (xn[a] - x[a]);
            rp += (pn[a] - p[a]) * (pn[a] - p[a]);
        }
        for (size_t a = 0; a < sz; a++) z[a] = xn[a] + o->theta * (xn[a] - x[a]);
        memcpy(x, xn, sz * sizeof(double));
        memcpy(p, pn, sz * sizeof(double));
        k++;
        kp++;
        if (!isfinite(rx + rp)) { st = OR_PT_NONFINITE; break; }
        int small = (rx < o->tol) && (rp < o->tol);
        if (!o->fixed_iters && small) { st = OR_PT_CONVERGED; break; }
        if (o->fixed_iters) {
            if (k >= o->max_iter) { st = small ? OR_PT_CONVERGED : OR_PT_MAXITER; break; }
            continue;
        }
        /* value-change rule, after the first cap */
        if (phase >= 1 && o->value_tol > 0.0) {
            double val = control_value(pb, x, p, N, delta);
            if (isfinite(prev_val) && fabs(val - prev_val) <= o->value_tol * fmax(fabs(val), 1.0)) {
                st = OR_PT_VALUE_STALLED;
                break;
            }
            prev_val = val;
        }
        if (kp >= o->max_iter) {
            if (phase < o->restarts) {
                /* cap reached: raise sigma, keep sigma tau, continue from this iterate */
                phase++;
                kp = 0;
                sigma += o->sigma_inc;
                tau = st_product / sigma;
                prev_val = NAN;
                if (chol) chol_I_tauQ(pb->gp, d, tau, chol);
                continue;
            }
            st = OR_PT_MAXITER;
            break;
        }
    }
    double val = control_value(pb, x, p, N, delta);
    if (!isfinite(val) || !all_finite(x, (int)sz) || !all_finite(p, (int)sz)) st = OR_PT_NONFINITE;
    *phi = val;
    *iters = k;
    *status = st;
    free(z); free(xn); free(pn); free(v); free(gr); free(chol);
}

static int rank_of(int st, double phi)
{
    if (st == OR_PT_CONVERGED || st == OR_PT_VALUE_STALLED) return 0;
    return isfinite(phi) ? 1 : 2;
}

static void solve_control_point(const or_problem *pb, const or_opts *o, long pt, const double *xt,
                                double t, int N, double *phi, int *iters, int *status,
                                double *xtraj, double *ptraj)
{
    int d = pb->d;
    size_t sz = (size_t)(N + 1) * d;
    double *x = calloc(sz, sizeof(double)), *p = calloc(sz, sizeof(double));
    int starts = o->starts > 1 ? o->starts : 1;
    int best_rank = 3;
    double best_phi = NAN;
    for (int s = 0; s < starts; s++) {
        double ph;
        int it, st;
        control_run(pb, o, pt, xt, t, N, o->seed + (uint64_t)s, x, p, &ph, &it, &st);
        int r = rank_of(st, ph);
        if (r < best_rank || (r == best_rank && r < 2 && ph < best_phi)) {
            best_rank = r;
            best_phi = ph;
            *phi = ph;
            *iters = it;
            *status = st;
            if (xtraj) memcpy(xtraj, x, sz * sizeof(double));
            if (ptraj) memcpy(ptraj, p, sz * sizeof(double));
        }
    }
    free(x); free(p);
}

/* ------------------------------------------------------------------ */
/* One query point: Hopf formulation (Algorithm 2, Appendix A.1.2).   */
/* Arrays keep nodes 0..N so outputs line up with the Lax path; node  */
/* 0 does not take part and stays zero.                               */
/* ------------------------------------------------------------------ */

static void solve_hopf_point(const or_problem *pb, const or_opts *o, long pt, const double *xt,
                             double t, int N, double *phi, int *iters, int *status,
                             double *xtraj, double *ptraj)
{
    int d = pb->d;
    double delta = t / N;
    size_t sz = (size_t)(N + 1) * d;
    double *x = calloc(sz, sizeof(double)), *p = calloc(sz, sizeof(double)), *z = calloc(sz, sizeof(double));
    double *xn = calloc(sz, sizeof(double)), *pn = calloc(sz, sizeof(double));
    double *v = calloc(d, sizeof(double)), *gr = calloc(d, sizeof(double));

    /* random start: x_j (1 <= j < N) near x, x_N = x, p_j (1 <= j <= N) near 0, z = x */
    for (int j = 1; j < N; j++)
        for (int i = 0; i < d; i++) x[j * d + i] = xt[i] + or_init_noise(o->seed, pt, OR_ARR_X, j, i);
    for (int i = 0; i < d; i++) x[N * d + i] = xt[i];
    for (int j = 1; j <= N; j++)
        for (int i = 0; i < d; i++) p[j * d + i] = or_init_noise(o->seed, pt, OR_ARR_P, j, i);
    memcpy(z, x, sz * sizeof(double));

    int k = 0, st = OR_PT_MAXITER;
    for (;;) {
        /* p-update, (D^T z)_1 = z_1, (D^T z)_j = z_j - z_{j-1} */
        for (int i = 0; i < d; i++) v[i] = p[d + i] + o->sigma * z[d + i];
        or_hopf_prox1(pb, &x[d], v, o->sigma, delta, &pn[d]);
        for (int j = 2; j <= N; j++) {
            for (int i = 0; i < d; i++) v[i] = p[j * d + i] + o->sigma * (z[j * d + i] - z[(j - 1) * d + i]);
            or_prox_p(pb, &x[j * d], v, o->sigma * delta, j * delta, &pn[j * d]);
        }
        /* x-update, j = 1..N-1: (D p)_j = p_j - p_{j+1}, one gradient step on -delta H */
        for (int j = 1; j < N; j++) {
            or_grad_x_H(pb, &x[j * d], &pn[j * d], j * delta, gr);
            for (int i = 0; i < d; i++)
                xn[j * d + i] = x[j * d + i] - o->tau * (pn[j * d + i] - pn[(j + 1) * d + i])
                                + o->tau * delta * gr[i];
        }
        for (int i = 0; i < d; i++) xn[N * d + i] = x[N * d + i];

        double rx = 0.0, rp = 0.0;
        for (size_t a = d; a < sz; a++) {
            rx += (xn[a] - x[a]) * (xn[a] - x[a]);
            rp += (pn[a] - p[a]) * (pn[a] - p[a]);
        }
        for (size_t a = d; a < sz; a++) z[a] = xn[a] + o->theta * (xn[a] - x[a]);
        memcpy(x, xn, sz * sizeof(double));
        memcpy(p, pn, sz * sizeof(double));
        k++;
        if (!isfinite(rx + rp)) { st = OR_PT_NONFINITE; break; }
        int small = (rx < o->tol) && (rp < o->tol);
        if (!o->fixed_iters && small) { st = OR_PT_CONVERGED; break; }
        if (k >= o->max_iter) { st = small ? OR_PT_CONVERGED : OR_PT_MAXITER; break; }
    }

    /* value (Algorithm 2 fval):
       -g*(p_1) + <p_N, x> + sum_{j<N} <p_j - p_{j+1}, x_j> - delta sum_j H(x_j, p_j) */
    double val = -or_gstar(pb, &p[d]) + dot(&p[N * d], xt, d);
    for (int j = 1; j < N; j++)
        for (int i = 0; i < d; i++) val += (p[j * d + i] - p[(j + 1) * d + i]) * x[j * d + i];
    for (int j = 1; j <= N; j++) val -= delta * or_H(pb, &x[j * d], &p[j * d], j * delta);
    if (!isfinite(val) || !all_finite(x, (int)sz) || !all_finite(p, (int)sz)) st = OR_PT_NONFINITE;
    *phi = val;
    *iters = k;
    *status = st;
    if (xtraj) memcpy(xtraj, x, sz * sizeof(double));
    if (ptraj) memcpy(ptraj, p, sz * sizeof(double));
    free(x); free(p); free(z); free(xn); free(pn); free(v); free(gr);
}

/* ------------------------------------------------------------------ */
/* One query point: weighted Euler discretisations (forward Euler,     */
/* trapezoid; backward Euler at wl = 0, wr = 1), eikonal and quadrotor. */
/* ------------------------------------------------------------------ */

/* The Lagrangian of the weighted saddle at (x, p). */
static double mix_value(const or_problem *pb, const double *x, const double *p, int N, double delta, double wl,
                        double wr)
{
    int d = pb->d;
    double val = or_g(pb, x);
    for (int j = 1; j <= N; j++) {
        for (int i = 0; i < d; i++) val += p[j * d + i] * (x[j * d + i] - x[(j - 1) * d + i]);
        val -= delta * (wl * or_H(pb, &x[(j - 1) * d], &p[j * d], (j - 1) * delta)
                        + wr * or_H(pb, &x[j * d], &p[j * d], j * delta));
    }
    return val;
}

static void solve_mix_point(const or_problem *pb, const or_opts *o, long pt, const double *xt, double t, int N,
                            double wl, double wr, double *phi, int *iters, int *status, double *xtraj, double *ptraj)
{
    int d = pb->d;
    double delta = t / N;
    size_t sz = (size_t)(N + 1) * d;
    double *x = calloc(sz, sizeof(double)), *p = calloc(sz, sizeof(double)), *z = calloc(sz, sizeof(double));
    double *xn = calloc(sz, sizeof(double)), *pn = calloc(sz, sizeof(double));
    double *v = calloc(d, sizeof(double)), *ga = calloc(d, sizeof(double)), *gb = calloc(d, sizeof(double));

    /* random start, as in Algorithm 1: x_j (j < N) near x, x_N = x, p_j (j >= 1) near 0, z = x */
    for (int j = 0; j < N; j++)
        for (int i = 0; i < d; i++) x[j * d + i] = xt[i] + or_init_noise(o->seed, pt, OR_ARR_X, j, i);
    for (int i = 0; i < d; i++) x[N * d + i] = xt[i];
    for (int j = 1; j <= N; j++)
        for (int i = 0; i < d; i++) p[j * d + i] = or_init_noise(o->seed, pt, OR_ARR_P, j, i);
    memcpy(z, x, sz * sizeof(double));

    int k = 0, st = OR_PT_MAXITER;
    for (;;) {
        /* p-step: the prox of the interval's weighted Hamiltonians (eikonal: a
           shrink by sigma delta times the weighted speed; quadrotor: a linear solve) */
        for (int i = 0; i < d; i++) pn[i] = 0.0;
        for (int j = 1; j <= N; j++) {
            for (int i = 0; i < d; i++) v[i] = p[j * d + i] + o->sigma * (z[j * d + i] - z[(j - 1) * d + i]);
            if (pb->H == OR_H_QUADROTOR) {
                quad_prox_p_mix(pb->hp, &x[(j - 1) * d], &x[j * d], wl, wr, v, o->sigma * delta, &pn[j * d]);
            } else {
                double c_eff = wl * cnorm_c(pb->hp, &x[(j - 1) * d]) + wr * cnorm_c(pb->hp, &x[j * d]);
                or_shrink2(v, o->sigma * delta * c_eff, d, &pn[j * d]);
            }
        }
        /* node 0: proximal-gradient step (gradient of -delta wl H(x_0, p_1), prox of g) */
        or_grad_x_H(pb, &x[0], &pn[d], 0.0, ga);
        for (int i = 0; i < d; i++) v[i] = x[i] + o->tau * pn[d + i] + o->tau * delta * wl * ga[i];
        prox_g(pb, v, o->tau, NULL, xn);
        /* nodes 1..N-1: x_j is the right end of interval j (weight wr, costate p_j)
           and the left end of interval j+1 (weight wl, costate p_{j+1}) */
        for (int j = 1; j < N; j++) {
            or_grad_x_H(pb, &x[j * d], &pn[j * d], j * delta, ga);
            or_grad_x_H(pb, &x[j * d], &pn[(j + 1) * d], j * delta, gb);
            for (int i = 0; i < d; i++)
                xn[j * d + i] = x[j * d + i] - o->tau * (pn[j * d + i] - pn[(j + 1) * d + i])
                                + o->tau * delta * (wr * ga[i] + wl * gb[i]);
        }
        for (int i = 0; i < d; i++) xn[N * d + i] = x[N * d + i];

        double rx = 0.0, rp = 0.0;
        for (size_t a = 0; a < sz; a++) {
            rx += (xn[a] - x[a]) * (xn[a] - x[a]);
            rp += (pn[a] - p[a]) * (pn[a] - p[a]);
        }
        for (size_t a = 0; a < sz; a++) z[a] = xn[a] + o->theta * (xn[a] - x[a]);
        memcpy(x, xn, sz * sizeof(double));
        memcpy(p, pn, sz * sizeof(double));
        k++;
        if (!isfinite(rx + rp)) { st = OR_PT_NONFINITE; break; }
        int small = (rx < o->tol) && (rp < o->tol);
        if (!o->fixed_iters && small) { st = OR_PT_CONVERGED; break; }
        if (k >= o->max_iter) { st = small ? OR_PT_CONVERGED : OR_PT_MAXITER; break; }
    }
    double val = mix_value(pb, x, p, N, delta, wl, wr);
    if (!isfinite(val) || !all_finite(x, (int)sz) || !all_finite(p, (int)sz)) st = OR_PT_NONFINITE;
    *phi = val;
    *iters = k;
    *status = st;
    if (xtraj) memcpy(xtraj, x, sz * sizeof(double));
    if (ptraj) memcpy(ptraj, p, sz * sizeof(double));
    free(x); free(p); free(z); free(xn); free(pn); free(v); free(ga); free(gb);
}

/* ------------------------------------------------------------------ */
/* One query point: game path (Algorithm 3, Appendix A.2.1), with the  */
/* recipes of section 6 that the paper applies to a game (sigma raised */
/* at the cap, value-change stop after the first cap; one start).      */
/* ------------------------------------------------------------------ */

/* The game value: g(x_0, y_0) + sum_j (<p_j, x_j - x_{j-1}> - <q_j, y_j - y_{j-1}>) - delta sum_j H. */
static double game_value(const or_problem *pb, const double *x, const double *y, const double *p, const double *q,
                         int N, double delta)
{
    int d = pb->d, dy = pb->d_y, dx = d - dy;
    double x0y0[64];
    for (int i = 0; i < dx; i++) x0y0[i] = x[i];
    for (int i = 0; i < dy; i++) x0y0[dx + i] = y[i];
    double val = or_g(pb, x0y0);
    for (int j = 1; j <= N; j++) {
        for (int i = 0; i < dx; i++) val += p[j * dx + i] * (x[j * dx + i] - x[(j - 1) * dx + i]);
        for (int i = 0; i < dy; i++) val -= q[j * dy + i] * (y[j * dy + i] - y[(j - 1) * dy + i]);
        val -= delta * or_game_H(pb, &x[j * dx], &y[j * dy], &p[j * dx], &q[j * dy]);
    }
    return val;
}

static void solve_game_point(const or_problem *pb, const or_opts *o, long pt, const double *xt,
                             double t, int N, double *phi, int *iters, int *status,
                             double *xtraj, double *ptraj)
{
    int d = pb->d, dy = pb->d_y, dx = d - dy;
    double delta = t / N;
    size_t sx = (size_t)(N + 1) * dx, sy = (size_t)(N + 1) * dy;
    double *x = calloc(sx, 8), *p = calloc(sx, 8), *z = calloc(sx, 8), *xn = calloc(sx, 8), *pn = calloc(sx, 8);
    double *y = calloc(sy, 8), *q = calloc(sy, 8), *w = calloc(sy, 8), *yn = calloc(sy, 8), *qn = calloc(sy, 8);
    double v[64], gr[64];
    double sigma = o->sigma, tau = o->tau;
    const double st_product = o->sigma * o->tau;

    for (int j = 0; j < N; j++) {
        for (int i = 0; i < dx; i++) x[j * dx + i] = xt[i] + or_init_noise(o->seed, pt, OR_ARR_X, j, i);
        for (int i = 0; i < dy; i++) y[j * dy + i] = xt[dx + i] + or_init_noise(o->seed, pt, OR_ARR_Y, j, i);
    }
    for (int i = 0; i < dx; i++) x[N * dx + i] = xt[i];
    for (int i = 0; i < dy; i++) y[N * dy + i] = xt[dx + i];
    for (int j = 1; j <= N; j++) {
        for (int i = 0; i < dx; i++) p[j * dx + i] = or_init_noise(o->seed, pt, OR_ARR_P, j, i);
        for (int i = 0; i < dy; i++) q[j * dy + i] = or_init_noise(o->seed, pt, OR_ARR_Q, j, i);
    }
    memcpy(z, x, sx * 8);
    memcpy(w, y, sy * 8);

    int k = 0, kp = 0, phase = 0, st = OR_PT_MAXITER;
    double prev_val = NAN;
    for (;;) {
        /* p block (maximiser's costate): uses x^k, y^k, q^k */
        for (int i = 0; i < dx; i++) pn[i] = 0.0;
        for (int j = 1; j <= N; j++) {
            for (int i = 0; i < dx; i++) v[i] = p[j * dx + i] + sigma * (z[j * dx + i] - z[(j - 1) * dx + i]);
            or_game_prox_p(pb, &x[j * dx], &y[j * dy], &q[j * dy], v, sigma * delta, &pn[j * dx]);
        }
        /* q block: uses p^{k+1} */
        for (int i = 0; i < dy; i++) qn[i] = 0.0;
        for (int j = 1; j <= N; j++) {
            for (int i = 0; i < dy; i++) v[i] = q[j * dy + i] + sigma * (w[j * dy + i] - w[(j - 1) * dy + i]);
            or_game_prox_q(pb, &x[j * dx], &y[j * dy], &pn[j * dx], v, sigma * delta, &qn[j * dy]);
        }
        /* x block: x_0 by the prox of g(., y_0^k); x_j by a descent step */
        for (int i = 0; i < dx; i++) v[i] = x[i] + tau * pn[dx + i];
        or_game_prox_x0(pb, v, y, tau, xn);
        for (int j = 1; j < N; j++) {
            or_game_grad_x(pb, &x[j * dx], &y[j * dy], &pn[j * dx], &qn[j * dy], gr);
            for (int i = 0; i < dx; i++)
                xn[j * dx + i] = x[j * dx + i] - tau * (pn[j * dx + i] - pn[(j + 1) * dx + i])
                                 + tau * delta * gr[i];
        }
        for (int i = 0; i < dx; i++) xn[N * dx + i] = x[N * dx + i];
        /* y block (maximiser): y_0 by the prox of -g(x_0^{k+1}, .); y_j by an
         * ascent step on the Lagrangian */
        for (int i = 0; i < dy; i++) v[i] = y[i] + tau * qn[dy + i];
        or_game_stretch_y0(pb, v, xn, tau, yn);
        for (int j = 1; j < N; j++) {
            or_game_grad_y(pb, &xn[j * dx], &y[j * dy], &pn[j * dx], &qn[j * dy], gr);
            for (int i = 0; i < dy; i++)
                yn[j * dy + i] = y[j * dy + i] - tau * (qn[j * dy + i] - qn[(j + 1) * dy + i])
                                 - tau * delta * gr[i];
        }
        for (int i = 0; i < dy; i++) yn[N * dy + i] = y[N * dy + i];

        double rx = 0, rp = 0, ry = 0, rq = 0;
        for (size_t a = 0; a < sx; a++) {
            rx += (xn[a] - x[a]) * (xn[a] - x[a]);
            rp += (pn[a] - p[a]) * (pn[a] - p[a]);
        }
        for (size_t a = 0; a < sy; a++) {
            ry += (yn[a] - y[a]) * (yn[a] - y[a]);
            rq += (qn[a] - q[a]) * (qn[a] - q[a]);
        }
        for (size_t a = 0; a < sx; a++) z[a] = xn[a] + o->theta * (xn[a] - x[a]);
        for (size_t a = 0; a < sy; a++) w[a] = yn[a] + o->theta * (yn[a] - y[a]);
        memcpy(x, xn, sx * 8); memcpy(p, pn, sx * 8);
        memcpy(y, yn, sy * 8); memcpy(q, qn, sy * 8);
        k++;
        kp++;
        if (!isfinite(rx + rp + ry + rq)) { st = OR_PT_NONFINITE; break; }
        int small = rx < o->tol && rp < o->tol && ry < o->tol && rq < o->tol;
        if (!o->fixed_iters && small) { st = OR_PT_CONVERGED; break; }
        if (o->fixed_iters) {
            if (k >= o->max_iter) { st = small ? OR_PT_CONVERGED : OR_PT_MAXITER; break; }
            continue;
        }
        /* value-change rule, after the first cap */
        if (phase >= 1 && o->value_tol > 0.0) {
            double val = game_value(pb, x, y, p, q, N, delta);
            if (isfinite(prev_val) && fabs(val - prev_val) <= o->value_tol * fmax(fabs(val), 1.0)) {
                st = OR_PT_VALUE_STALLED;
                break;
            }
            prev_val = val;
        }
        if (kp >= o->max_iter) {
            if (phase < o->restarts) {
                /* cap reached: raise sigma, keep sigma tau, continue from this iterate */
                phase++;
                kp = 0;
                sigma += o->sigma_inc;
                tau = st_product / sigma;
                prev_val = NAN;
                continue;
            }
            st = OR_PT_MAXITER;
            break;
        }
    }

    double val = game_value(pb, x, y, p, q, N, delta);
    if (!isfinite(val) || !all_finite(x, (int)sx) || !all_finite(y, (int)sy) ||
        !all_finite(p, (int)sx) || !all_finite(q, (int)sy))
        st = OR_PT_NONFINITE;
    *phi = val;
    *iters = k;
    *status = st;
    /* trajectories per node: state (x_j, y_j); multipliers (p_j, q_j) */
    for (int j = 0; j <= N; j++) {
        if (xtraj) {
            for (int i = 0; i < dx; i++) xtraj[j * d + i] = x[j * dx + i];
            for (int i = 0; i < dy; i++) xtraj[j * d + dx + i] = y[j * dy + i];
        }
        if (ptraj) {
            for (int i = 0; i < dx; i++) ptraj[j * d + i] = p[j * dx + i];
            for (int i = 0; i < dy; i++) ptraj[j * d + dx + i] = q[j * dy + i];
        }
    }
    free(x); free(p); free(z); free(xn); free(pn);
    free(y); free(q); free(w); free(yn); free(qn);
}

/* ------------------------------------------------------------------ */
/* One query point of Isaacs' game: Algorithm 4 (hopf = 1; no node 0,   */
/* z_0 = w_0 = 0) or Algorithm 3 (hopf = 0; node 0 by the prox of e and */
/* the prox of -h).  Blocks p, q, x, y in that order.                  */
/* ------------------------------------------------------------------ */

static void solve_isaacs_point(const or_problem *pb, const or_opts *o, long pt, const double *xt, double t, int N,
                               int hopf, double *phi, int *iters, int *status, double *xtraj, double *ptraj)
{
    const double *hp = pb->hp, *gp = pb->gp;
    double delta = t / N, sg = o->sigma, ta = o->tau, th = o->theta;
    size_t n1 = (size_t)N + 1;
    double *x = calloc(n1, 8), *y = calloc(n1, 8), *p = calloc(n1, 8), *q = calloc(n1, 8);
    double *z = calloc(n1, 8), *w = calloc(n1, 8), *xn = calloc(n1, 8), *yn = calloc(n1, 8);
    double *pn = calloc(n1, 8), *qn = calloc(n1, 8);
    int j0 = hopf ? 1 : 0;

    /* random start: free nodes near (x, y), costates near 0, node N = (x, y) */
    for (int j = j0; j < N; j++) {
        x[j] = xt[0] + or_init_noise(o->seed, pt, OR_ARR_X, j, 0);
        y[j] = xt[1] + or_init_noise(o->seed, pt, OR_ARR_Y, j, 0);
    }
    x[N] = xt[0];
    y[N] = xt[1];
    for (int j = 1; j <= N; j++) {
        p[j] = or_init_noise(o->seed, pt, OR_ARR_P, j, 0);
        q[j] = or_init_noise(o->seed, pt, OR_ARR_Q, j, 0);
    }
    memcpy(z, x, n1 * 8);
    memcpy(w, y, n1 * 8);

    int k = 0, st = OR_PT_MAXITER;
    for (;;) {
        /* p and q, node by node (q uses the new p of its node) */
        for (int j = 1; j <= N; j++) {
            int first = hopf && j == 1;
            double v = p[j] + sg * (z[j] - z[j - 1]);
            pn[j] = or_isaacs_dual_p(gp, p[j], q[j], v, sg, delta, first);
            double u = q[j] + sg * (w[j] - w[j - 1]);
            qn[j] = or_isaacs_dual_q(hp, gp, x[j], y[j], pn[j], q[j], u, sg, delta, first);
        }
        /* x: descent; with H(x,y,p,-q) = c(x,y) q + ..., grad_x H = q dc/dx */
        if (!hopf) xn[0] = (x[0] + ta * pn[1]) / (1.0 + ta * gp[1] * gp[1]);
        for (int j = 1; j < N; j++) {
            double cx;
            isaacs_c(hp, x[j], y[j], &cx, NULL);
            xn[j] = x[j] - ta * (pn[j] - pn[j + 1]) + ta * delta * qn[j] * cx;
        }
        xn[N] = x[N];
        /* y: ascent, at the new x */
        if (!hopf) yn[0] = (y[0] + ta * qn[1]) / (1.0 + ta * gp[2] * gp[2]);
        for (int j = 1; j < N; j++) {
            double cy;
            isaacs_c(hp, xn[j], y[j], NULL, &cy);
            yn[j] = y[j] - ta * (qn[j] - qn[j + 1]) - ta * delta * qn[j] * cy;
        }
        yn[N] = y[N];

        double rx = 0, ry = 0, rp = 0, rq = 0;
        for (int j = 0; j <= N; j++) {
            rx += (xn[j] - x[j]) * (xn[j] - x[j]);
            ry += (yn[j] - y[j]) * (yn[j] - y[j]);
            rp += (pn[j] - p[j]) * (pn[j] - p[j]);
            rq += (qn[j] - q[j]) * (qn[j] - q[j]);
        }
        for (int j = j0; j <= N; j++) {
            z[j] = xn[j] + th * (xn[j] - x[j]);
            w[j] = yn[j] + th * (yn[j] - y[j]);
        }
        memcpy(x, xn, n1 * 8); memcpy(y, yn, n1 * 8);
        memcpy(p, pn, n1 * 8); memcpy(q, qn, n1 * 8);
        k++;
        if (!isfinite(rx + ry + rp + rq)) { st = OR_PT_NONFINITE; break; }
        int small = rx < o->tol && ry < o->tol && rp < o->tol && rq < o->tol;
        if (!o->fixed_iters && small) { st = OR_PT_CONVERGED; break; }
        if (k >= o->max_iter) { st = small ? OR_PT_CONVERGED : OR_PT_MAXITER; break; }
    }

    double val;
    if (hopf) {
        /* -e*(p_1) - h_*(-q_1) + <p_N,x> - <q_N,y> + sum_{j<N} ((p_j - p_{j+1}) x_j - (q_j - q_{j+1}) y_j) */
        val = -or_saddle_estar(gp, p[1]) - or_saddle_hstar(gp, -q[1]) + p[N] * xt[0] - q[N] * xt[1];
        for (int j = 1; j < N; j++) val += (p[j] - p[j + 1]) * x[j] - (q[j] - q[j + 1]) * y[j];
    } else {
        val = or_saddle_g(gp, x[0], y[0]);
        for (int j = 1; j <= N; j++) val += p[j] * (x[j] - x[j - 1]) - q[j] * (y[j] - y[j - 1]);
    }
    for (int j = 1; j <= N; j++) val -= delta * or_isaacs_H(hp, x[j], y[j], p[j], -q[j]);
    if (!isfinite(val) || !all_finite(x, (int)n1) || !all_finite(y, (int)n1) || !all_finite(p, (int)n1) ||
        !all_finite(q, (int)n1))
        st = OR_PT_NONFINITE;
    *phi = val;
    *iters = k;
    *status = st;
    for (int j = 0; j <= N; j++) {
        if (xtraj) { xtraj[2 * j] = x[j]; xtraj[2 * j + 1] = y[j]; }
        if (ptraj) { ptraj[2 * j] = p[j]; ptraj[2 * j + 1] = q[j]; }
    }
    free(x); free(y); free(p); free(q); free(z); free(w); free(xn); free(yn); free(pn); free(qn);
}

/* ------------------------------------------------------------------ */
/* Batch driver.                                                       */
/* ------------------------------------------------------------------ */

/*
 * Solve n independent query points.  x is [n][d] (row-major), t and N are
 * [n].  Outputs phi, iters, status are [n]; x_traj and p_traj (may be NULL)
 * are [n][N_max+1][d], nodes beyond a point's N left untouched.  ids (may
 * be NULL, meaning 0..n-1) gives each point's index in the full workload;
 * it selects the point's random start.  Points are distributed over
 * n_threads OpenMP threads (n_threads <= 0: the runtime default); each point
 * is solved sequentially.
 * Returns 0, or -1 for an unsupported problem.
 */
typedef struct {
    int starts, restarts;
    double sigma_inc, value_tol;
} or_recipe;

static int solve_batch(const or_problem *pb, long n, const double *x, const double *t, const int *N,
                       double sigma, double tau, double theta, double tol, int max_iter, int fixed_iters,
                       uint64_t seed, int N_max, const int64_t *ids, double *phi, int *iters, int *status,
                       double *x_traj, double *p_traj, int n_threads, int hopf, const or_recipe *recipe,
                       const double *mix)
{
    int game = pb->d_y > 0;
    int isaacs = game && pb->H == OR_H_ISAACS && pb->g == OR_G_SADDLE_QUAD && pb->d == 2 && pb->d_y == 1;
    if (game && !isaacs && !(pb->H == OR_H_PURSUIT_EVASION && pb->g == OR_G_PAIR_DIST)) return -1;
    if (!game && (pb->H == OR_H_ISAACS || pb->g == OR_G_SADDLE_QUAD)) return -1;
    if (!game && (pb->H == OR_H_PURSUIT_EVASION || pb->g == OR_G_PAIR_DIST)) return -1;
    if (hopf && !isaacs && (game || !((pb->H == OR_H_CNORM && (pb->g == OR_G_NORM || pb->g == OR_G_QUAD_SHIFT)) ||
                                      (pb->H == OR_H_QUADROTOR && pb->g == OR_G_QUAD_SHIFT))))
        return -1;
    if (mix && (game || hopf || recipe ||
                !((pb->H == OR_H_CNORM && (pb->g == OR_G_NORM || pb->g == OR_G_QUAD_SHIFT)) ||
                  (pb->H == OR_H_QUADROTOR && pb->g == OR_G_QUAD_SHIFT))))
        return -1;
    or_opts o = { sigma, tau, theta, tol, max_iter, fixed_iters, seed, N_max, 1, 0, 0.0, 0.0 };
    if (recipe) {
        o.starts = recipe->starts;
        o.restarts = recipe->restarts;
        o.sigma_inc = recipe->sigma_inc;
        o.value_tol = recipe->value_tol;
        /* games: the sigma and value-change recipes only (one start), Algorithm 3 of the pursuit-evasion game */
        if ((game && (isaacs || o.starts > 1)) || hopf || fixed_iters || o.restarts < 0 || o.sigma_inc < 0.0 ||
            o.value_tol < 0.0)
            return -1;
    }
    int d = pb->d;
#ifdef _OPENMP
    int nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#else
    int nt = 1;
    (void)n_threads;
#endif
    (void)nt;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
    for (long i = 0; i < n; i++) {
        int Ni = N[i];
        double ti = t[i];
        int bad = !(ti > 0.0) || !isfinite(ti) || Ni < 1 || Ni > N_max || !all_finite(&x[i * d], d);
        if (bad) {
            phi[i] = NAN;
            iters[i] = 0;
            status[i] = OR_PT_BADINPUT;
            continue;
        }
        double *xt_out = x_traj ? &x_traj[(size_t)i * (N_max + 1) * d] : NULL;
        double *pt_out = p_traj ? &p_traj[(size_t)i * (N_max + 1) * d] : NULL;
        long id = ids ? (long)ids[i] : i;
        if (isaacs)
            solve_isaacs_point(pb, &o, id, &x[i * d], ti, Ni, hopf, &phi[i], &iters[i], &status[i], xt_out, pt_out);
        else if (game)
            solve_game_point(pb, &o, id, &x[i * d], ti, Ni, &phi[i], &iters[i], &status[i], xt_out, pt_out);
        else if (hopf)
            solve_hopf_point(pb, &o, id, &x[i * d], ti, Ni, &phi[i], &iters[i], &status[i], xt_out, pt_out);
        else if (mix)
            solve_mix_point(pb, &o, id, &x[i * d], ti, Ni, mix[0], mix[1], &phi[i], &iters[i], &status[i], xt_out,
                            pt_out);
        else
            solve_control_point(pb, &o, id, &x[i * d], ti, Ni, &phi[i], &iters[i], &status[i], xt_out, pt_out);
    }
    return 0;
}

/* Lax formulation (Algorithm 1; Algorithm 3 for games). */
int or_solve(const or_problem *pb, long n, const double *x, const double *t, const int *N,
             double sigma, double tau, double theta, double tol, int max_iter, int fixed_iters,
             uint64_t seed, int N_max, const int64_t *ids, double *phi, int *iters, int *status,
             double *x_traj, double *p_traj, int n_threads)
{
    return solve_batch(pb, n, x, t, N, sigma, tau, theta, tol, max_iter, fixed_iters, seed, N_max, ids, phi, iters,
                       status, x_traj, p_traj, n_threads, 0, NULL, NULL);
}

/* Hopf formulation (Algorithm 2), eikonal family with NORM or QUAD_SHIFT g. */
int or_solve_hopf(const or_problem *pb, long n, const double *x, const double *t, const int *N,
                  double sigma, double tau, double theta, double tol, int max_iter, int fixed_iters,
                  uint64_t seed, int N_max, const int64_t *ids, double *phi, int *iters, int *status,
                  double *x_traj, double *p_traj, int n_threads)
{
    return solve_batch(pb, n, x, t, N, sigma, tau, theta, tol, max_iter, fixed_iters, seed, N_max, ids, phi, iters,
                       status, x_traj, p_traj, n_threads, 1, NULL, NULL);
}

/* Algorithm 1 with the robustness recipes (tolerance mode); Algorithm 3 of the
 * pursuit-evasion game with the sigma and value-change recipes (starts = 1). */
int or_solve_recipe(const or_problem *pb, long n, const double *x, const double *t, const int *N,
                    double sigma, double tau, double theta, double tol, int max_iter, uint64_t seed, int N_max,
                    const int64_t *ids, int starts, int restarts, double sigma_inc, double value_tol,
                    double *phi, int *iters, int *status, double *x_traj, double *p_traj, int n_threads)
{
    or_recipe r = { starts, restarts, sigma_inc, value_tol };
    return solve_batch(pb, n, x, t, N, sigma, tau, theta, tol, max_iter, 0, seed, N_max, ids, phi, iters,
                       status, x_traj, p_traj, n_threads, 0, &r, NULL);
}

/* Weighted Euler discretisations (forward Euler wl = 1, wr = 0; trapezoid
 * wl = wr = 1/2; backward Euler wl = 0, wr = 1), eikonal and quadrotor families. */
int or_solve_mix(const or_problem *pb, long n, const double *x, const double *t, const int *N,
                 double sigma, double tau, double theta, double tol, int max_iter, int fixed_iters,
                 uint64_t seed, int N_max, const int64_t *ids, double wl, double wr, double *phi, int *iters,
                 int *status, double *x_traj, double *p_traj, int n_threads)
{
    double w[2] = { wl, wr };
    return solve_batch(pb, n, x, t, N, sigma, tau, theta, tol, max_iter, fixed_iters, seed, N_max, ids, phi, iters,
                       status, x_traj, p_traj, n_threads, 0, NULL, w);
}
