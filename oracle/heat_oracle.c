/*
 * heat_oracle.c -- FP64 CPU reference for the implicit-Euler heat solver and
 * its discrete adjoint.  TEST INFRASTRUCTURE ONLY: called by the test suite,
 * the smoke check and the CPU-baseline timing; never by the product path.
 * Shares no code with the GPU library.
 *
 * What it computes (the paper's Sec. 4.2-4.3 and App. D.2-D.3, with the sign
 * convention A = I + dt*L+, L+ positive semidefinite, which is the paper's
 * A = I - dt*L with L = -L+):
 *
 *   face conductance   c_f = 2 a_p a_q / (a_p + a_q) / h_d^2       (Prop. 1, eq. fv_stencil)
 *   operator           (L+ x)_p = beta_p x_p + sum_{interior faces f=(p,q)} c_f (x_p - x_q)
 *                      boundary faces carry no term (zero flux), except that
 *                      - with lateral periodicity the x and y faces wrap around
 *                        (circular padding, App. D.2), so cell 0 and cell n-1 of
 *                        a row share a face;
 *                      - with a Robin back face the rows k = nz-1 carry the sink
 *                        beta_p = h/dz (App. D.2, "Symmetry, sign, and diagonal
 *                        dominance"); every other row has beta_p = 0
 *   state equation     A T^n = T^{n-1} + dt q^n,   T^0 = 0          (eq. state_eq plus a source)
 *   observation        S^n = T^n restricted to the plane k = 0      (the projector Pi of eq. nefty_obj)
 *   adjoint            A mu^n = mu^{n+1} + Pi^T g^n,  mu^{N+1} = 0  (eq. adjoint_eq; A symmetric)
 *   gradient           dJ/da_p = -dt sum_n sum_{f ni p} dc_f/da_p (T_p-T_q)(mu_p-mu_q)
 *                      dc_f/da_p = 2 a_q^2 / (a_p + a_q)^2 / h_d^2   (eq. grad_assembly and the
 *                      harmonic-mean derivative of App. D.3; the Robin sink
 *                      does not depend on alpha and adds nothing)
 *   source sensitivity dJ/dq^n = dt * mu^n on k = 0
 *
 * By default every linear solve is a plain Jacobi-preconditioned conjugate
 * gradient in FP64, run to a tight relative residual (1e-13 by default), so
 * the result is the exact discrete trajectory up to that tolerance.  The
 * paper's own inner solver can be chosen instead: K plain Jacobi sweeps
 * x <- D^-1 (b - R x), A = D + R, started from the previous time level's
 * state (eq. jacobi_iter, App. D.2); the adjoint solves take the same K
 * sweeps from mu^{n+1} (App. D.3 uses the same inner solver both ways).
 * Nothing is fused or blocked: each step is one function.
 *
 * Layout: volumes are [nz][ny][nx], x fastest; k = 0 is the top face.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* The grid, its boundary closure and the inner solver. */
typedef struct {
    int nx, ny, nz;
    double hx, hy, hz;
    int periodic;   /* 1: the lateral x and y faces wrap around (needs nx, ny >= 3); 0: zero flux */
    double beta;    /* Robin sink rate h/dz on the back-face rows k = nz-1; 0: adiabatic back face */
    int jacobi_k;   /* 0: Jacobi-PCG to rtol; K > 0: K Jacobi sweeps per solve */
} orc_grid;

static long long ng_of(const orc_grid *g) { return (long long)g->nx * g->ny * g->nz; }

static long long idx(const orc_grid *g, int i, int j, int k) {
    return (long long)i + (long long)g->nx * ((long long)j + (long long)g->ny * k);
}

/* Harmonic-mean face conductance (Prop. 1) divided by the squared spacing. */
static double conductance(double ap, double aq, double h) {
    return 2.0 * ap * aq / (ap + aq) / (h * h);
}

/* Derivative of the conductance with respect to the first argument. */
static double dconductance(double ap, double aq, double h) {
    return 2.0 * aq * aq / ((ap + aq) * (ap + aq)) / (h * h);
}

/* Index of the cell one step from (i, j, k) along axis d (0: x, 1: y, 2: z)
 * in direction s (-1 or +1), or -1 where that side of the cell is a boundary
 * face. Lateral periodicity wraps x and y; z never wraps. */
static long long neighbour(const orc_grid *g, int i, int j, int k, int d, int s) {
    if (d == 0) {
        i += s;
        if (i < 0 || i >= g->nx) {
            if (!g->periodic) return -1;
            i = (i + g->nx) % g->nx;
        }
    } else if (d == 1) {
        j += s;
        if (j < 0 || j >= g->ny) {
            if (!g->periodic) return -1;
            j = (j + g->ny) % g->ny;
        }
    } else {
        k += s;
        if (k < 0 || k >= g->nz) return -1;
    }
    return idx(g, i, j, k);
}

static double spacing(const orc_grid *g, int d) { return d == 0 ? g->hx : d == 1 ? g->hy : g->hz; }

/* Robin sink of the row of cell (.., .., k): beta on the back face, else 0. */
static double sink(const orc_grid *g, int k) { return k == g->nz - 1 ? g->beta : 0.0; }

/* Runs BODY once for every interior face (p, q) of the grid, with h the
 * spacing across it: q is the +x, +y or +z neighbour of p (wrapped where
 * the lateral faces are periodic). */
#define FOR_EACH_FACE(g, BODY)                                                  \
    for (int k = 0; k < (g)->nz; ++k)                                           \
        for (int j = 0; j < (g)->ny; ++j)                                       \
            for (int i = 0; i < (g)->nx; ++i)                                   \
                for (int d = 0; d < 3; ++d) {                                   \
                    long long p = idx((g), i, j, k);                            \
                    long long q = neighbour((g), i, j, k, d, +1);               \
                    if (q < 0) continue;                                        \
                    double h = spacing((g), d);                                 \
                    BODY                                                        \
                }

/* y = A x = x + dt * L+ x, written per cell over its (up to) six faces. */
void orc_apply_A(const orc_grid *g, const double *alpha, double dt, const double *x, double *y) {
    const int nx = g->nx, ny = g->ny, nz = g->nz;
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                long long p = idx(g, i, j, k);
                double ap = alpha[p], s = sink(g, k) * x[p];
                for (int d = 0; d < 3; ++d)
                    for (int sg = -1; sg <= 1; sg += 2) {
                        long long q = neighbour(g, i, j, k, d, sg);
                        if (q >= 0) s += conductance(ap, alpha[q], spacing(g, d)) * (x[p] - x[q]);
                    }
                y[p] = x[p] + dt * s;
            }
}

/* Diagonal of A: D_p = 1 + dt * (beta_p + sum of the conductances of p's interior faces). */
void orc_diagonal(const orc_grid *g, const double *alpha, double dt, double *d) {
    const int nx = g->nx, ny = g->ny, nz = g->nz;
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                long long p = idx(g, i, j, k);
                double ap = alpha[p], s = sink(g, k);
                for (int dd = 0; dd < 3; ++dd)
                    for (int sg = -1; sg <= 1; sg += 2) {
                        long long q = neighbour(g, i, j, k, dd, sg);
                        if (q >= 0) s += conductance(ap, alpha[q], spacing(g, dd));
                    }
                d[p] = 1.0 + dt * s;
            }
}

/* y = R x with R = A - D the off-diagonal part of A: (R x)_p = -dt sum_{q ~ p} c_pq x_q. */
void orc_apply_R(const orc_grid *g, const double *alpha, double dt, const double *x, double *y) {
    const int nx = g->nx, ny = g->ny, nz = g->nz;
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                long long p = idx(g, i, j, k);
                double ap = alpha[p], s = 0.0;
                for (int d = 0; d < 3; ++d)
                    for (int sg = -1; sg <= 1; sg += 2) {
                        long long q = neighbour(g, i, j, k, d, sg);
                        if (q >= 0) s += conductance(ap, alpha[q], spacing(g, d)) * x[q];
                    }
                y[p] = -dt * s;
            }
}

/*
 * K Jacobi sweeps on A x = b from the x passed in (eq. jacobi_iter):
 * x <- D^-1 (b - R x), R x formed from the whole previous iterate before
 * any entry of x changes.
 */
void orc_jacobi(const orc_grid *g, const double *alpha, double dt, const double *dg,
                const double *b, double *x, int K) {
    const long long n = ng_of(g);
    double *rx = malloc(sizeof(double) * n);
    for (int kappa = 0; kappa < K; ++kappa) {
        orc_apply_R(g, alpha, dt, x, rx);
#pragma omp parallel for schedule(static)
        for (long long i = 0; i < n; ++i) x[i] = (b[i] - rx[i]) / dg[i];
    }
    free(rx);
}

static double dot(long long n, const double *a, const double *b) {
    double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (long long i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/*
 * Jacobi-preconditioned CG for A x = b, starting from the x passed in.
 * Stops when ||r||_2 <= rtol * ||b||_2 (r the recursively updated residual)
 * or after max_iter iterations.  ||b|| = 0 gives x = 0 and 0 iterations.
 * Returns the iteration count, or -1 if max_iter was reached first.
 * *rel_out receives the final ||r|| / ||b||.
 */
int orc_pcg(const orc_grid *g, const double *alpha, double dt, const double *dg,
            const double *b, double *x, double rtol, int max_iter, double *rel_out) {
    const long long n = ng_of(g);
    double bb = dot(n, b, b);
    if (bb == 0.0) {
        memset(x, 0, sizeof(double) * (size_t)n);
        if (rel_out) *rel_out = 0.0;
        return 0;
    }
    double *r = malloc(sizeof(double) * n), *z = malloc(sizeof(double) * n);
    double *p = malloc(sizeof(double) * n), *q = malloc(sizeof(double) * n);
    orc_apply_A(g, alpha, dt, x, q);
#pragma omp parallel for schedule(static)
    for (long long i = 0; i < n; ++i) {
        r[i] = b[i] - q[i];
        z[i] = r[i] / dg[i];
        p[i] = z[i];
    }
    double rz = dot(n, r, z);
    double rr = dot(n, r, r);
    const double bnorm = sqrt(bb);
    int it = 0, status = 0;
    while (sqrt(rr) > rtol * bnorm) {
        if (it == max_iter) { status = -1; break; }
        orc_apply_A(g, alpha, dt, p, q);
        double a = rz / dot(n, p, q);
#pragma omp parallel for schedule(static)
        for (long long i = 0; i < n; ++i) {
            x[i] += a * p[i];
            r[i] -= a * q[i];
            z[i] = r[i] / dg[i];
        }
        double rz_new = dot(n, r, z);
        double beta = rz_new / rz;
        rz = rz_new;
#pragma omp parallel for schedule(static)
        for (long long i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        rr = dot(n, r, r);
        ++it;
    }
    if (rel_out) *rel_out = sqrt(rr) / bnorm;
    free(r); free(z); free(p); free(q);
    return status < 0 ? -1 : it;
}

/* The configured inner solver on A x = b from the x passed in: Jacobi-PCG
 * (returns its iterations, or -1 without convergence) or K Jacobi sweeps
 * (returns K). */
static int inner_solve(const orc_grid *g, const double *alpha, double dt, const double *dg,
                       const double *b, double *x, double rtol, int max_iter) {
    if (g->jacobi_k > 0) {
        orc_jacobi(g, alpha, dt, dg, b, x, g->jacobi_k);
        return g->jacobi_k;
    }
    return orc_pcg(g, alpha, dt, dg, b, x, rtol, max_iter, NULL);
}

/*
 * Forward sweep.  src is the top-face source per step, [nsteps][ny][nx]
 * (q^n = src[n-1]).  T0 may be NULL (T^0 = 0).  Outputs:
 *   S      [nsteps][ny][nx]  surface temperature of T^1..T^N
 *   T_all  [nsteps][ng]      every state T^1..T^N (may be NULL)
 *   iters  [nsteps]          inner-solver iterations per step (may be NULL)
 * Returns 0, or -1 if some step did not converge.
 */
int orc_forward(const orc_grid *g, const double *alpha, const double *src, const double *T0,
                double dt, int nsteps, double rtol, int max_iter,
                double *S, double *T_all, int *iters) {
    const long long n = ng_of(g), nxy = (long long)g->nx * g->ny;
    double *dg = malloc(sizeof(double) * n), *b = malloc(sizeof(double) * n);
    double *x = malloc(sizeof(double) * n);
    orc_diagonal(g, alpha, dt, dg);
    if (T0) memcpy(x, T0, sizeof(double) * n); else memset(x, 0, sizeof(double) * n);
    int status = 0;
    for (int s = 1; s <= nsteps; ++s) {
        /* b = T^{s-1} + dt q^s, the source living on the k = 0 plane */
        memcpy(b, x, sizeof(double) * n);
        for (long long c = 0; c < nxy; ++c) b[c] += dt * src[(long long)(s - 1) * nxy + c];
        /* warm start from T^{s-1}, which is already in x */
        int it = inner_solve(g, alpha, dt, dg, b, x, rtol, max_iter);
        if (it < 0) status = -1;
        if (iters) iters[s - 1] = it;
        memcpy(S + (long long)(s - 1) * nxy, x, sizeof(double) * nxy);
        if (T_all) memcpy(T_all + (long long)(s - 1) * n, x, sizeof(double) * n);
    }
    free(dg); free(b); free(x);
    return status;
}

/* G_p += scale * sum_{f ni p} dc_f/da_p (T_p - T_q)(mu_p - mu_q), visiting each face once. */
static void accumulate_gradient(const orc_grid *g, const double *alpha, const double *T,
                                const double *mu, double scale, double *G) {
    FOR_EACH_FACE(g, {
        double w = (T[p] - T[q]) * (mu[p] - mu[q]);
        G[p] += scale * dconductance(alpha[p], alpha[q], h) * w;
        G[q] += scale * dconductance(alpha[q], alpha[p], h) * w;
    })
}

/*
 * Adjoint sweep over a stored forward trajectory T_all [nsteps][ng] with
 * surface weights gs = dJ/dS, [nsteps][ny][nx].  Outputs:
 *   G     [ng]              dJ/dalpha (overwritten)
 *   dq    [nsteps][ny][nx]  dJ/dq^n = dt mu^n on k = 0 (may be NULL)
 *   mu1   [ng]              mu^1 = dJ/dT^0 (may be NULL)
 *   iters [nsteps]          iterations of the solve producing mu^n, at index n-1 (may be NULL)
 */
int orc_adjoint(const orc_grid *g, const double *alpha, double dt, int nsteps,
                const double *T_all, const double *gs, double rtol, int max_iter,
                double *G, double *dq, double *mu1, int *iters) {
    const long long n = ng_of(g), nxy = (long long)g->nx * g->ny;
    double *dg = malloc(sizeof(double) * n), *c = malloc(sizeof(double) * n);
    double *mu = calloc((size_t)n, sizeof(double));
    orc_diagonal(g, alpha, dt, dg);
    memset(G, 0, sizeof(double) * n);
    int status = 0;
    for (int s = nsteps; s >= 1; --s) {
        /* c = mu^{s+1} + Pi^T g^s; mu holds mu^{s+1} and is the warm start */
        memcpy(c, mu, sizeof(double) * n);
        for (long long e = 0; e < nxy; ++e) c[e] += gs[(long long)(s - 1) * nxy + e];
        int it = inner_solve(g, alpha, dt, dg, c, mu, rtol, max_iter);
        if (it < 0) status = -1;
        if (iters) iters[s - 1] = it;
        accumulate_gradient(g, alpha, T_all + (long long)(s - 1) * n, mu, -dt, G);
        if (dq) for (long long e = 0; e < nxy; ++e) dq[(long long)(s - 1) * nxy + e] = dt * mu[e];
    }
    if (mu1) memcpy(mu1, mu, sizeof(double) * n);
    free(dg); free(c); free(mu);
    return status;
}

/*
 * Tangent-linear model: the directional derivative of the surface series in
 * the direction v of alpha.  Differentiating A T^n = T^{n-1} + dt q^n gives
 *   A dT^n = dT^{n-1} - dt (d(L+ T^n)/dalpha) v,   dT^0 = 0,
 * where ((d(L+ T)/dalpha) v)_p = sum_{f=(p,q)} (dc_f/da_p v_p + dc_f/da_q v_q)(T_p - T_q).
 * Output dS [nsteps][ny][nx] = dT^n on k = 0.
 */
int orc_tlm(const orc_grid *g, const double *alpha, const double *v, double dt, int nsteps,
            const double *T_all, double rtol, int max_iter, double *dS) {
    const long long n = ng_of(g), nxy = (long long)g->nx * g->ny;
    double *dg = malloc(sizeof(double) * n), *b = malloc(sizeof(double) * n);
    double *dT = calloc((size_t)n, sizeof(double));
    orc_diagonal(g, alpha, dt, dg);
    int status = 0;
    for (int s = 1; s <= nsteps; ++s) {
        const double *T = T_all + (long long)(s - 1) * n;
        memcpy(b, dT, sizeof(double) * n);
        FOR_EACH_FACE(g, {
            double dc = dconductance(alpha[p], alpha[q], h) * v[p] + dconductance(alpha[q], alpha[p], h) * v[q];
            double f = dc * (T[p] - T[q]);
            b[p] -= dt * f;
            b[q] += dt * f;
        })
        if (inner_solve(g, alpha, dt, dg, b, dT, rtol, max_iter) < 0) status = -1;
        memcpy(dS + (long long)(s - 1) * nxy, dT, sizeof(double) * nxy);
    }
    free(dg); free(b); free(dT);
    return status;
}

/* Number of OpenMP threads the oracle runs with (for reporting). */
int orc_num_threads(void) {
    int t = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            extern int omp_get_num_threads(void);
            t = omp_get_num_threads();
#endif
        }
    }
    return t;
}

/* Use n OpenMP threads from now on (n >= 1; for timing the oracle on one core). */
void orc_set_num_threads(int n) {
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
