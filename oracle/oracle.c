/*
 * CPU oracle for the swept time-space decomposition hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no source, header, table or helper with the
 * HIP path.
 *
 * What it computes is the plain, slow, obviously correct definition: one full
 * explicit timestep over the whole periodic grid per loop iteration, exactly
 * the "classic" decomposition of Magee & Niemeyer (arXiv 1612.02495, Sec. 4.4).
 * The swept rule reorders *where and when* these same updates are evaluated
 * and does not change the numerical scheme (Sec. 2), so the plain timestepper
 * is the reference the swept result must reproduce.
 *
 * Precision and operation order (IEEE-754, round to nearest even; build with
 * -ffp-contract=off and no -ffast-math, so the only fused multiply-adds are
 * the fma() calls written out, each a*b + c rounded once):
 *
 *   Heat (Sec. 4.1, Eq. HeatDisc; Appendix, final FTCS form):
 *       Fo = (alpha*dt)/(dx*dx), c = 1 - 2*Fo   (computed once, in double)
 *       T_i^{m+1} = Fo*(T_{i+1}^m + T_{i-1}^m) + c*T_i^m
 *                 = fma(Fo, T_{i+1}^m + T_{i-1}^m, c*T_i^m)
 *
 *   Kuramoto-Sivashinsky (Sec. 4.1, Eq. KSDisc; Appendix, RK2 midpoint):
 *       with a=u_{i+1}, b=u_{i-1}, aa=u_{i+2}, bb=u_{i-2}, o=u_i, the right-
 *       hand side is f = -g with
 *       g = (a - b)(a + b)/(4dx)                     (u u_x = (u^2/2)_x)
 *         + ((a + b) - 2o)/dx^2                      (u_xx)
 *         + ((aa + bb) - 4(a + b) + 6o)/dx^4         (u_xxxx)
 *       and each RK2 stage u + h f is formed as u - h g, the step h folded
 *       into the coefficients h/(4dx), h/dx^2, h/dx^4 (each the double
 *       product of h and the inverse):
 *       S1 = a + b, S2 = aa + bb,
 *       hg = fma(h/dx^4, fma(6, o, fma(-4, S1, S2)),
 *                fma(h/dx^2, fma(-2, o, S1), (h/(4dx)) * ((a - b) * S1)))
 *       predictor  u^{m+1/2}_i = u^m_i - hg(u^m)_i      with h = dt/2, for all i, then
 *       final      u^{m+1}_i   = u^m_i - hg(u^{m+1/2})_i  with h = dt.
 *     The inverses 1/(4dx), 1/dx^2 and 1/dx^4 = (1/dx^2)^2 are formed once and
 *     multiplied in, as Sec. 5 (division avoidance) describes.  The printed
 *     "+2u_i" in the u_xx numerator is read as "-2u_i" (the central second
 *     difference; with "+" the term is not a derivative and sum(u) would not be
 *     conserved).  Every sum is symmetric in the two sides and the flux term
 *     antisymmetric, so the step maps -u(-x) exactly to the negated mirror of
 *     the step of u(x).
 *
 *   Periodic boundaries: neighbour i+k is (i+k) mod n (Sec. 4.1; Appendix).
 *
 * The float entry points run the same order in single precision, with the
 * constants formed in double and rounded once to float.
 *
 * Heat adjoint (not in the paper; the derivation is plain calculus on the
 * discrete scheme above): for J = 1/2 ||u_T - y||^2 with u_{m+1} = A(alpha) u_m,
 *   lambda_T = u_T - y,  lambda_m = A^T lambda_{m+1}  (A is symmetric here),
 *   dJ/du_0 = lambda_0,
 *   dJ/dalpha = (dt/dx^2) * sum_{m<T} sum_i lambda_{m+1,i} (u_{m,i-1} + u_{m,i+1} - 2 u_{m,i}).
 * Forward states are recomputed from checkpoints every K steps.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL -1
#define ORACLE_ENOMEM -3

static int64_t wrap(int64_t i, int64_t n) {
    int64_t r = i % n;
    return r < 0 ? r + n : r;
}

/* ---------------------------------------------------------------- heat -- */

static void heat_step_f64(const double* u, double* v, int64_t n, double fo, double c) {
    for (int64_t i = 0; i < n; ++i) {
        double left = u[wrap(i - 1, n)];
        double right = u[wrap(i + 1, n)];
        v[i] = fma(fo, right + left, c * u[i]);
    }
}

static void heat_step_f32(const float* u, float* v, int64_t n, float fo, float c) {
    for (int64_t i = 0; i < n; ++i) {
        float left = u[wrap(i - 1, n)];
        float right = u[wrap(i + 1, n)];
        v[i] = fmaf(fo, right + left, c * u[i]);
    }
}

int oracle_heat_f64(double* u, int64_t n, double alpha, double dt, double dx, int64_t steps) {
    if (!u || n < 1 || steps < 0) return ORACLE_EINVAL;
    double fo = (alpha * dt) / (dx * dx);
    double c = 1.0 - 2.0 * fo;
    double* v = (double*)malloc((size_t)n * sizeof(double));
    if (!v) return ORACLE_ENOMEM;
    double* cur = u;
    double* nxt = v;
    for (int64_t m = 0; m < steps; ++m) {
        heat_step_f64(cur, nxt, n, fo, c);
        double* t = cur; cur = nxt; nxt = t;
    }
    if (cur != u) memcpy(u, cur, (size_t)n * sizeof(double));
    free(v);
    return ORACLE_OK;
}

int oracle_heat_f32(float* u, int64_t n, double alpha, double dt, double dx, int64_t steps) {
    if (!u || n < 1 || steps < 0) return ORACLE_EINVAL;
    double fo_d = (alpha * dt) / (dx * dx);
    float fo = (float)fo_d;
    float c = (float)(1.0 - 2.0 * fo_d);
    float* v = (float*)malloc((size_t)n * sizeof(float));
    if (!v) return ORACLE_ENOMEM;
    float* cur = u;
    float* nxt = v;
    for (int64_t m = 0; m < steps; ++m) {
        heat_step_f32(cur, nxt, n, fo, c);
        float* t = cur; cur = nxt; nxt = t;
    }
    if (cur != u) memcpy(u, cur, (size_t)n * sizeof(float));
    free(v);
    return ORACLE_OK;
}

/* --------------------------------------------- all host cores (OpenMP) -- */
/*
 * The same timesteppers with the loop over grid points of each step split
 * over host threads (OpenMP, static schedule).  Every point is updated from
 * the previous step's values by the same expression as above, and no value
 * is summed across points, so the result is bit for bit that of the
 * single-thread entry points for any thread count.  For the CPU-baseline
 * timing on all host cores.  nthreads <= 0 takes the OpenMP default
 * (OMP_NUM_THREADS, else the host's cores); *used receives the count.
 */
#include <omp.h>

int oracle_heat_f64_mt(double* u, int64_t n, double alpha, double dt, double dx, int64_t steps, int nthreads,
                       int* used) {
    if (!u || n < 1 || steps < 0) return ORACLE_EINVAL;
    double fo = (alpha * dt) / (dx * dx);
    double c = 1.0 - 2.0 * fo;
    double* v = (double*)malloc((size_t)n * sizeof(double));
    if (!v) return ORACLE_ENOMEM;
    int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
    if (used) *used = nt;
    double* cur = u;
    double* nxt = v;
    for (int64_t m = 0; m < steps; ++m) {
#pragma omp parallel for num_threads(nt) schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double left = cur[wrap(i - 1, n)];
            double right = cur[wrap(i + 1, n)];
            nxt[i] = fma(fo, right + left, c * cur[i]);
        }
        double* t = cur; cur = nxt; nxt = t;
    }
    if (cur != u) memcpy(u, cur, (size_t)n * sizeof(double));
    free(v);
    return ORACLE_OK;
}

/* ----------------------------------------------- heat, insulated rod -- */
/*
 * The rod with insulated ends of Sec. 4.1 (Appendix, "insulated boundary
 * conditions at both ends"): n nodes, the same interior update, and mirror
 * ghosts about the end nodes, u_{-1} = u_1 and u_n = u_{n-2}.  The printed
 * ghost relations are garbled; the right-hand one (ghost n+1 equals node n-1
 * in 1-based numbering) is a mirror about the end node, and the left-hand one
 * is read the same way.  n >= 2.
 */
static void heat_ins_step_f64(const double* u, double* v, int64_t n, double fo, double c) {
    for (int64_t i = 0; i < n; ++i) {
        double left = i == 0 ? u[1] : u[i - 1];
        double right = i == n - 1 ? u[n - 2] : u[i + 1];
        v[i] = fma(fo, right + left, c * u[i]);
    }
}

static void heat_ins_step_f32(const float* u, float* v, int64_t n, float fo, float c) {
    for (int64_t i = 0; i < n; ++i) {
        float left = i == 0 ? u[1] : u[i - 1];
        float right = i == n - 1 ? u[n - 2] : u[i + 1];
        v[i] = fmaf(fo, right + left, c * u[i]);
    }
}

int oracle_heat_insulated_f64(double* u, int64_t n, double alpha, double dt, double dx, int64_t steps) {
    if (!u || n < 2 || steps < 0) return ORACLE_EINVAL;
    double fo = (alpha * dt) / (dx * dx);
    double c = 1.0 - 2.0 * fo;
    double* v = (double*)malloc((size_t)n * sizeof(double));
    if (!v) return ORACLE_ENOMEM;
    double* cur = u;
    double* nxt = v;
    for (int64_t m = 0; m < steps; ++m) {
        heat_ins_step_f64(cur, nxt, n, fo, c);
        double* t = cur; cur = nxt; nxt = t;
    }
    if (cur != u) memcpy(u, cur, (size_t)n * sizeof(double));
    free(v);
    return ORACLE_OK;
}

int oracle_heat_insulated_f32(float* u, int64_t n, double alpha, double dt, double dx, int64_t steps) {
    if (!u || n < 2 || steps < 0) return ORACLE_EINVAL;
    double fo_d = (alpha * dt) / (dx * dx);
    float fo = (float)fo_d;
    float c = (float)(1.0 - 2.0 * fo_d);
    float* v = (float*)malloc((size_t)n * sizeof(float));
    if (!v) return ORACLE_ENOMEM;
    float* cur = u;
    float* nxt = v;
    for (int64_t m = 0; m < steps; ++m) {
        heat_ins_step_f32(cur, nxt, n, fo, c);
        float* t = cur; cur = nxt; nxt = t;
    }
    if (cur != u) memcpy(u, cur, (size_t)n * sizeof(float));
    free(v);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------ KS -- */

typedef struct {
    double i4dx, idx2, idx4, dt, dth;
    double pnl, p2, p4; /* predictor (h = dt/2): h/(4dx), h/dx^2, h/dx^4 */
    double fnl, f2, f4; /* final (h = dt) */
} ks_consts;

static ks_consts ks_make(double dt, double dx) {
    ks_consts k;
    k.i4dx = 1.0 / (4.0 * dx);
    k.idx2 = 1.0 / (dx * dx);
    k.idx4 = k.idx2 * k.idx2;
    k.dt = dt;
    k.dth = 0.5 * dt;
    k.pnl = k.dth * k.i4dx;
    k.p2 = k.dth * k.idx2;
    k.p4 = k.dth * k.idx4;
    k.fnl = k.dt * k.i4dx;
    k.f2 = k.dt * k.idx2;
    k.f4 = k.dt * k.idx4;
    return k;
}

/* h g at point i of the ring v, with cnl = h/(4dx), c2 = h/dx^2, c4 = h/dx^4 */
static double ks_hg_f64(const double* v, int64_t n, int64_t i, double cnl, double c2, double c4) {
    double bb = v[wrap(i - 2, n)];
    double b = v[wrap(i - 1, n)];
    double o = v[i];
    double a = v[wrap(i + 1, n)];
    double aa = v[wrap(i + 2, n)];
    double s1 = a + b, s2 = aa + bb;
    double flux = (a - b) * s1;
    double d2 = fma(-2.0, o, s1);
    double d4 = fma(6.0, o, fma(-4.0, s1, s2));
    return fma(c4, d4, fma(c2, d2, cnl * flux));
}

static float ks_hg_f32(const float* v, int64_t n, int64_t i, float cnl, float c2, float c4) {
    float bb = v[wrap(i - 2, n)];
    float b = v[wrap(i - 1, n)];
    float o = v[i];
    float a = v[wrap(i + 1, n)];
    float aa = v[wrap(i + 2, n)];
    float s1 = a + b, s2 = aa + bb;
    float flux = (a - b) * s1;
    float d2 = fmaf(-2.0f, o, s1);
    float d4 = fmaf(6.0f, o, fmaf(-4.0f, s1, s2));
    return fmaf(c4, d4, fmaf(c2, d2, cnl * flux));
}

int oracle_ks_f64(double* u, int64_t n, double dt, double dx, int64_t steps) {
    if (!u || n < 1 || steps < 0) return ORACLE_EINVAL;
    ks_consts k = ks_make(dt, dx);
    double* up = (double*)malloc((size_t)n * sizeof(double));
    if (!up) return ORACLE_ENOMEM;
    for (int64_t m = 0; m < steps; ++m) {
        for (int64_t i = 0; i < n; ++i) up[i] = u[i] - ks_hg_f64(u, n, i, k.pnl, k.p2, k.p4);
        for (int64_t i = 0; i < n; ++i) u[i] = u[i] - ks_hg_f64(up, n, i, k.fnl, k.f2, k.f4);
    }
    free(up);
    return ORACLE_OK;
}

int oracle_ks_f32(float* u, int64_t n, double dt, double dx, int64_t steps) {
    if (!u || n < 1 || steps < 0) return ORACLE_EINVAL;
    ks_consts k = ks_make(dt, dx);
    float pnl = (float)k.pnl, p2 = (float)k.p2, p4 = (float)k.p4;
    float fnl = (float)k.fnl, f2 = (float)k.f2, f4 = (float)k.f4;
    float* up = (float*)malloc((size_t)n * sizeof(float));
    if (!up) return ORACLE_ENOMEM;
    for (int64_t m = 0; m < steps; ++m) {
        for (int64_t i = 0; i < n; ++i) up[i] = u[i] - ks_hg_f32(u, n, i, pnl, p2, p4);
        for (int64_t i = 0; i < n; ++i) u[i] = u[i] - ks_hg_f32(up, n, i, fnl, f2, f4);
    }
    free(up);
    return ORACLE_OK;
}

int oracle_ks_f64_mt(double* u, int64_t n, double dt, double dx, int64_t steps, int nthreads, int* used) {
    if (!u || n < 1 || steps < 0) return ORACLE_EINVAL;
    ks_consts k = ks_make(dt, dx);
    double* up = (double*)malloc((size_t)n * sizeof(double));
    if (!up) return ORACLE_ENOMEM;
    int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
    if (used) *used = nt;
    for (int64_t m = 0; m < steps; ++m) {
#pragma omp parallel num_threads(nt)
        {
#pragma omp for schedule(static)
            for (int64_t i = 0; i < n; ++i) up[i] = u[i] - ks_hg_f64(u, n, i, k.pnl, k.p2, k.p4);
#pragma omp for schedule(static)
            for (int64_t i = 0; i < n; ++i) u[i] = u[i] - ks_hg_f64(up, n, i, k.fnl, k.f2, k.f4);
        }
    }
    free(up);
    return ORACLE_OK;
}

/* ------------------------------------------------------- heat adjoint -- */

/* Neumaier-compensated accumulator: keeps the reference sums of the
 * objective and of dJ/dalpha accurate to a few ulps regardless of length. */
typedef struct { double s, c; } acc_t;
static void acc_add(acc_t* a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static double acc_get(const acc_t* a) { return a->s + a->c; }

/*
 * u0, y: n values each.  Outputs: g_u0 (n values), *g_alpha, *J.
 * Checkpoints every `ckpt` steps (0 = choose ~sqrt(steps)).
 */
int oracle_heat_adjoint_f64(const double* u0, const double* y, int64_t n, double alpha, double dt,
                            double dx, int64_t steps, int64_t ckpt, double* g_u0, double* g_alpha,
                            double* J) {
    if (!u0 || !y || !g_u0 || !g_alpha || !J || n < 1 || steps < 0) return ORACLE_EINVAL;
    double fo = (alpha * dt) / (dx * dx);
    double c = 1.0 - 2.0 * fo;
    double dfo = dt / (dx * dx); /* d Fo / d alpha */
    int64_t K = ckpt;
    if (K <= 0) {
        K = (int64_t)ceil(sqrt((double)(steps > 0 ? steps : 1)));
        if (K < 1) K = 1;
    }
    int64_t nseg = steps > 0 ? (steps + K - 1) / K : 0;
    size_t nb = (size_t)n * sizeof(double);
    double* ck = (double*)malloc(nb * (size_t)(nseg > 0 ? nseg : 1));
    double* seg = (double*)malloc(nb * (size_t)(K + 1));
    double* lam = (double*)malloc(nb);
    double* tmp = (double*)malloc(nb);
    if (!ck || !seg || !lam || !tmp) {
        free(ck); free(seg); free(lam); free(tmp);
        return ORACLE_ENOMEM;
    }
    /* forward: store the state at the start of every segment */
    memcpy(tmp, u0, nb);
    for (int64_t s = 0; s < nseg; ++s) {
        memcpy(ck + (size_t)s * n, tmp, nb);
        int64_t len = (s == nseg - 1) ? steps - s * K : K;
        for (int64_t m = 0; m < len; ++m) {
            heat_step_f64(tmp, lam, n, fo, c);
            memcpy(tmp, lam, nb);
        }
    }
    /* tmp = u_T */
    acc_t jacc = {0.0, 0.0};
    for (int64_t i = 0; i < n; ++i) {
        double d = tmp[i] - y[i];
        lam[i] = d;
        acc_add(&jacc, 0.5 * d * d);
    }
    acc_t gacc = {0.0, 0.0};
    for (int64_t s = nseg - 1; s >= 0; --s) {
        int64_t len = (s == nseg - 1) ? steps - s * K : K;
        memcpy(seg, ck + (size_t)s * n, nb);
        for (int64_t m = 0; m < len; ++m) heat_step_f64(seg + (size_t)m * n, seg + (size_t)(m + 1) * n, n, fo, c);
        for (int64_t m = len - 1; m >= 0; --m) {
            const double* um = seg + (size_t)m * n;
            /* dJ/dalpha contribution of step m: <lambda_{m+1}, dA/dalpha u_m> */
            for (int64_t i = 0; i < n; ++i) {
                double lap = (um[wrap(i - 1, n)] + um[wrap(i + 1, n)]) - 2.0 * um[i];
                acc_add(&gacc, lam[i] * lap);
            }
            /* lambda_m = A^T lambda_{m+1}; A is symmetric for the periodic stencil */
            heat_step_f64(lam, tmp, n, fo, c);
            memcpy(lam, tmp, nb);
        }
    }
    memcpy(g_u0, lam, nb);
    *g_alpha = dfo * acc_get(&gacc);
    *J = acc_get(&jacc);
    free(ck); free(seg); free(lam); free(tmp);
    return ORACLE_OK;
}

/* ------------------------------------------------------- KS adjoint -- */
/*
 * Reverse sweep of the periodic KS RK2 scheme above for
 * J = 1/2 ||u_T - y||^2 (not in the paper; plain calculus on the discrete
 * scheme).  One step is q = u + (dt/2) f(u), u' = u + dt f(q), so with
 * lambda' = dJ/du':
 *   mu     = dt * Jf(q)^T lambda'                    (= dJ/dq)
 *   lambda = lambda' + mu + (dt/2) * Jf(u)^T mu      (= dJ/du)
 * where Jf(v) is the Jacobian of f at v.  Its transpose applied to w, at j,
 * collects the derivatives of f_{j-2} .. f_{j+2} with respect to v_j:
 *   df_{j-1}/dv_j = -( 2 v_j/(4dx) + 1/dx^2 - 4/dx^4)
 *   df_{j+1}/dv_j = -(-2 v_j/(4dx) + 1/dx^2 - 4/dx^4)
 *   df_j/dv_j     = -(-2/dx^2 + 6/dx^4)
 *   df_{j+-2}/dv_j = -1/dx^4
 * with 2 v_j/(4dx) formed as v_j * (1/(2dx)), 1/(2dx) = 2 * (1/(4dx)) (the
 * same rounding as (2 v_j) * (1/(4dx))), and the sum taken in the order
 * w_{j-1}, w_{j+1}, w_j, w_{j-2}, w_{j+2}: the first product rounded, each
 * later one fused into the running sum.  The update of lambda is
 * fma(dt/2, Jf(u)^T mu, lambda' + mu).
 * Forward states are recomputed from checkpoints every `ckpt` steps.
 */
static void ks_jt_f64(const double* v, const double* w, double* out, int64_t n, const ks_consts* k) {
    double c1 = k->idx2 - 4.0 * k->idx4;
    double c0 = -(6.0 * k->idx4 - 2.0 * k->idx2);
    double c2 = -k->idx4;
    double i2dx = 2.0 * k->i4dx;
    for (int64_t j = 0; j < n; ++j) {
        double s = v[j] * i2dx;
        double dm = -(s + c1);  /* df_{j-1}/dv_j */
        double dp = -(c1 - s);  /* df_{j+1}/dv_j */
        double acc = dm * w[wrap(j - 1, n)];
        acc = fma(dp, w[wrap(j + 1, n)], acc);
        acc = fma(c0, w[j], acc);
        acc = fma(c2, w[wrap(j - 2, n)], acc);
        out[j] = fma(c2, w[wrap(j + 2, n)], acc);
    }
}

int oracle_ks_adjoint_f64(const double* u0, const double* y, int64_t n, double dt, double dx, int64_t steps,
                          int64_t ckpt, double* g_u0, double* J) {
    if (!u0 || !y || !g_u0 || !J || n < 5 || steps < 0) return ORACLE_EINVAL;
    ks_consts k = ks_make(dt, dx);
    int64_t K = ckpt;
    if (K <= 0) {
        K = 1;
        while (K * K < steps) ++K;
    }
    int64_t nck = steps / K + 1;
    double* cks = (double*)malloc((size_t)(nck * n) * sizeof(double));
    double* seg = (double*)malloc((size_t)((K + 1) * n) * sizeof(double));
    double* q = (double*)malloc((size_t)n * sizeof(double));
    double* lam = (double*)malloc((size_t)n * sizeof(double));
    double* mu = (double*)malloc((size_t)n * sizeof(double));
    double* t1 = (double*)malloc((size_t)n * sizeof(double));
    if (!cks || !seg || !q || !lam || !mu || !t1) {
        free(cks); free(seg); free(q); free(lam); free(mu); free(t1);
        return ORACLE_ENOMEM;
    }
    /* forward, keeping u at steps 0, K, 2K, ... */
    memcpy(seg, u0, (size_t)n * sizeof(double));
    for (int64_t m = 0; m < steps; ++m) {
        if (m % K == 0) memcpy(cks + (m / K) * n, seg, (size_t)n * sizeof(double));
        for (int64_t i = 0; i < n; ++i) q[i] = seg[i] - ks_hg_f64(seg, n, i, k.pnl, k.p2, k.p4);
        for (int64_t i = 0; i < n; ++i) t1[i] = seg[i] - ks_hg_f64(q, n, i, k.fnl, k.f2, k.f4);
        memcpy(seg, t1, (size_t)n * sizeof(double));
    }
    acc_t ja = {0.0, 0.0};
    for (int64_t i = 0; i < n; ++i) {
        double r = seg[i] - y[i];
        lam[i] = r;
        acc_add(&ja, 0.5 * r * r);
    }
    *J = acc_get(&ja);
    /* reverse, segment by segment */
    for (int64_t s0 = ((steps - 1) / K) * K; steps > 0 && s0 >= 0; s0 -= K) {
        int64_t s1 = s0 + K < steps ? s0 + K : steps;
        memcpy(seg, cks + (s0 / K) * n, (size_t)n * sizeof(double));
        for (int64_t m = s0; m < s1 - 1; ++m) {
            double* u = seg + (m - s0) * n;
            for (int64_t i = 0; i < n; ++i) q[i] = u[i] - ks_hg_f64(u, n, i, k.pnl, k.p2, k.p4);
            for (int64_t i = 0; i < n; ++i) u[n + i] = u[i] - ks_hg_f64(q, n, i, k.fnl, k.f2, k.f4);
        }
        for (int64_t m = s1 - 1; m >= s0; --m) {
            double* u = seg + (m - s0) * n;
            for (int64_t i = 0; i < n; ++i) q[i] = u[i] - ks_hg_f64(u, n, i, k.pnl, k.p2, k.p4);
            ks_jt_f64(q, lam, mu, n, &k);
            for (int64_t i = 0; i < n; ++i) mu[i] = k.dt * mu[i];
            ks_jt_f64(u, mu, t1, n, &k);
            for (int64_t i = 0; i < n; ++i) lam[i] = fma(k.dth, t1[i], lam[i] + mu[i]);
        }
    }
    memcpy(g_u0, lam, (size_t)n * sizeof(double));
    free(cks); free(seg); free(q); free(lam); free(mu); free(t1);
    return ORACLE_OK;
}
