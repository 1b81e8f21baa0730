/*
 * Plain CPU FP64 oracle for the MG-MLQMC per-sample path.
 *
 * TEST INFRASTRUCTURE ONLY: called by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark; never by the product path.  Written from
 * the paper's statement of the method; shares no code with the GPU library.
 *
 * Every routine is the plain definition: loops in the paper's order, no
 * blocking, fusion or reordering.  Pinned by the CPU tests (closed forms,
 * invariants, brute force, library routines); see oracle.h for conventions.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif
#ifndef M_SQRT2
#define M_SQRT2 1.41421356237309504880
#endif

/* ======================================================================
 * Section 3.2: rank-1 lattice rule t_n = {n z / N}, turned into a lattice
 * sequence by visiting n in base-2 radical-inverse order, plus a random shift
 * {t + Delta}.  Points live in 64-bit fixed point: the integer x stands for
 * x / 2^64 in [0,1), so "mod 1" is wrap-around of unsigned arithmetic.
 * ====================================================================== */
uint32_t oracle_bitrev32(uint32_t v)
{
    uint32_t r = 0;
    for (int b = 0; b < 32; ++b) {
        r = (r << 1) | (v & 1u);
        v >>= 1;
    }
    return r;
}

void oracle_lattice_x(const uint32_t *z, int s, const uint64_t *delta,
                      uint64_t n, uint64_t *x)
{
    uint32_t rn = oracle_bitrev32((uint32_t)n);
    for (int j = 0; j < s; ++j) {
        /* {rev(n) z_j / 2^32} in 32-bit fixed point */
        uint32_t k = (uint32_t)((uint64_t)rn * (uint64_t)z[j]);
        /* {t + Delta} in 64-bit fixed point */
        x[j] = ((uint64_t)k << 32) + delta[j];
    }
}

double oracle_unit(uint64_t x)
{
    /* midpoint of the 2^-52-wide cell containing x / 2^64: never 0 or 1 */
    return (2.0 * (double)(x >> 12) + 1.0) * 0x1p-53;
}

/* Phi(y) - u, evaluated so that it keeps full relative accuracy near the
 * root: through erf in the central region (u - 1/2 is exact there) and
 * through erfc in the lower tail. */
static double phi_minus_u(double y, double u)
{
    if (u >= 0.25)
        return 0.5 * erf(y / M_SQRT2) - (u - 0.5);
    return 0.5 * erfc(-y / M_SQRT2) - u;
}

double oracle_norminv(double u)
{
    if (!(u > 0.0 && u < 1.0))
        return NAN;
    if (u == 0.5)
        return 0.0;
    if (u > 0.5)                      /* Phi^-1(u) = -Phi^-1(1-u), 1-u exact */
        return -oracle_norminv(1.0 - u);
    /* u in (0, 1/2): root in (-40, 0).  Bisection to a narrow bracket ... */
    double lo = -40.0, hi = 0.0;
    for (int it = 0; it < 40; ++it) {
        double mid = 0.5 * (lo + hi);
        if (phi_minus_u(mid, u) < 0.0)
            lo = mid;
        else
            hi = mid;
    }
    /* ... then Halley's iteration on g(y) = Phi(y) - u, g' = phi, g'' = -y phi */
    double y = 0.5 * (lo + hi);
    for (int it = 0; it < 50; ++it) {
        double g = phi_minus_u(y, u);
        double pdf = exp(-0.5 * y * y) / sqrt(2.0 * M_PI);
        double t = g / pdf;
        double step = t / (1.0 + 0.5 * y * t);
        double ynew = y - step;
        if (ynew == y || fabs(step) <= 1e-17 * fabs(y))
            return ynew;
        y = ynew;
    }
    return y;
}

void oracle_points(const uint32_t *z, int s, const uint64_t *delta,
                   int64_t n_begin, int64_t n_end, uint64_t *x, double *y)
{
    for (int64_t n = n_begin; n < n_end; ++n) {
        uint64_t *xr = x + (n - n_begin) * s;
        oracle_lattice_x(z, s, delta, (uint64_t)n, xr);
        if (y)
            for (int j = 0; j < s; ++j)
                y[(n - n_begin) * s + j] = oracle_norminv(oracle_unit(xr[j]));
    }
}

/* ======================================================================
 * Section 5: truncated KL expansion of a zero-mean Gaussian field with the
 * separable exponential covariance sigma^2 exp(-|x1-x1'|/lam - |x2-x2'|/lam).
 * The 1-D kernel exp(-|x-t|/lam) on [0,1] has eigenfunctions
 * sin(w x) + lam w cos(w x), eigenvalues 2 lam / (1 + lam^2 w^2), where w
 * solves (lam^2 w^2 - 1) sin w = 2 lam w cos w; one root per ((k-1)pi, k pi).
 * ====================================================================== */
static double kl_char(double lam, double w)
{
    return (lam * lam * w * w - 1.0) * sin(w) - 2.0 * lam * w * cos(w);
}

double oracle_kl_root(double lam, int k)
{
    double lo = (k - 1) * M_PI, hi = k * M_PI;
    /* sign just right of (k-1)pi: negative for k = 1, (-1)^k otherwise */
    int lo_positive = (k % 2 == 0);
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi)
            break;
        double f = kl_char(lam, mid);
        if (f == 0.0)
            return mid;
        if ((f > 0.0) == lo_positive)
            lo = mid;
        else
            hi = mid;
    }
    return 0.5 * (lo + hi);
}

double oracle_kl_theta(double lam, double w)
{
    return 2.0 * lam / (1.0 + lam * lam * w * w);
}

double oracle_kl_psi(double lam, double w, double x)
{
    /* ||sin wx + lam w cos wx||^2 over [0,1] = (1 + lam^2 w^2)/2 + lam at a root */
    double norm2 = 0.5 * (1.0 + lam * lam * w * w) + lam;
    return (sin(w * x) + lam * w * cos(w * x)) / sqrt(norm2);
}

typedef struct {
    double theta;
    int i, j;
} kl_pair;

static int kl_pair_cmp(const void *pa, const void *pb)
{
    const kl_pair *a = (const kl_pair *)pa, *b = (const kl_pair *)pb;
    if (a->theta > b->theta) return -1;   /* descending eigenvalue */
    if (a->theta < b->theta) return 1;
    if (a->i != b->i) return a->i < b->i ? -1 : 1;   /* ties: i ascending */
    return (a->j > b->j) - (a->j < b->j);
}

int oracle_kl_modes(double lam, int s, int *mi, int *mj, double *theta)
{
    /* The top s products theta_i theta_j only involve 1-D indices <= s. */
    int p = s;
    double *th = (double *)malloc(sizeof(double) * p);
    kl_pair *all = (kl_pair *)malloc(sizeof(kl_pair) * (size_t)p * p);
    if (!th || !all) {
        free(th);
        free(all);
        return -1;
    }
    for (int k = 1; k <= p; ++k)
        th[k - 1] = oracle_kl_theta(lam, oracle_kl_root(lam, k));
    for (int i = 1; i <= p; ++i)
        for (int j = 1; j <= p; ++j) {
            kl_pair *q = &all[(size_t)(i - 1) * p + (j - 1)];
            q->theta = th[i - 1] * th[j - 1];
            q->i = i;
            q->j = j;
        }
    qsort(all, (size_t)p * p, sizeof(kl_pair), kl_pair_cmp);
    for (int m = 0; m < s; ++m) {
        mi[m] = all[m].i;
        mj[m] = all[m].j;
        if (theta)
            theta[m] = all[m].theta;
    }
    free(th);
    free(all);
    return 0;
}

/* ---- problem handle ------------------------------------------------------ */
struct oracle_problem {
    int n0, num_levels, s, g0;
    double lam, sigma;
    int mu0, mu1, mu2, max_iters;
    double rtol;
    int pmax;        /* largest 1-D index used by the kept modes */
    double *w;       /* [pmax] roots */
    double *coef;    /* [s] sigma sqrt(theta_i theta_j) */
    int *mi, *mj;    /* [s] 1-based */
};

static int ilog2(int v)
{
    int r = 0;
    while ((1 << r) < v)
        ++r;
    return r;
}

oracle_problem *oracle_problem_new(int n0, int num_levels, int s,
                                   double corr_len, double sigma2,
                                   int mu0, int mu1, int mu2,
                                   double rtol, int max_iters)
{
    if (n0 < 2 || (n0 & (n0 - 1)) || num_levels < 1 || s < 1 || corr_len <= 0)
        return NULL;
    oracle_problem *P = (oracle_problem *)calloc(1, sizeof(*P));
    P->n0 = n0;
    P->num_levels = num_levels;
    P->s = s;
    P->g0 = ilog2(n0) - 1;
    P->lam = corr_len;
    P->sigma = sqrt(sigma2);
    P->mu0 = mu0;
    P->mu1 = mu1;
    P->mu2 = mu2;
    P->rtol = rtol;
    P->max_iters = max_iters;
    P->mi = (int *)malloc(sizeof(int) * s);
    P->mj = (int *)malloc(sizeof(int) * s);
    double *th2 = (double *)malloc(sizeof(double) * s);
    oracle_kl_modes(corr_len, s, P->mi, P->mj, th2);
    P->pmax = 0;
    for (int m = 0; m < s; ++m) {
        if (P->mi[m] > P->pmax) P->pmax = P->mi[m];
        if (P->mj[m] > P->pmax) P->pmax = P->mj[m];
    }
    P->w = (double *)malloc(sizeof(double) * P->pmax);
    for (int k = 1; k <= P->pmax; ++k)
        P->w[k - 1] = oracle_kl_root(corr_len, k);
    P->coef = (double *)malloc(sizeof(double) * s);
    for (int m = 0; m < s; ++m)
        P->coef[m] = P->sigma * sqrt(th2[m]);
    free(th2);
    return P;
}

void oracle_problem_free(oracle_problem *P)
{
    if (!P)
        return;
    free(P->w);
    free(P->coef);
    free(P->mi);
    free(P->mj);
    free(P);
}

int oracle_finest_mg_level(const oracle_problem *P, int k)
{
    return P->g0 + k;
}

int64_t oracle_field_size(const oracle_problem *P, int k)
{
    int64_t tot = 0;
    for (int g = 0; g <= P->g0 + k; ++g) {
        int64_t n = (int64_t)2 << g;
        tot += n * n;
    }
    return tot;
}

/* z(x) = sigma sum_m sqrt(theta_m) psi_m(x) y_m  (truncated KL, eq. truncatedKL)
 * at every cell centre of every multigrid level */
void oracle_field(const oracle_problem *P, const double *y, int k, double *z)
{
    int G = P->g0 + k;
    int64_t off = 0;
    for (int g = 0; g <= G; ++g) {
        int n = 2 << g;
        /* psi_i at the n cell-centre coordinates, i = 1..pmax */
        double *ps = (double *)malloc(sizeof(double) * P->pmax * n);
        for (int i = 0; i < P->pmax; ++i)
            for (int c = 0; c < n; ++c)
                ps[i * n + c] = oracle_kl_psi(P->lam, P->w[i], (c + 0.5) / n);
        for (int jc = 0; jc < n; ++jc)
            for (int ic = 0; ic < n; ++ic) {
                double acc = 0.0;
                for (int m = 0; m < P->s; ++m)
                    acc += P->coef[m] * ps[(P->mi[m] - 1) * n + ic] *
                           ps[(P->mj[m] - 1) * n + jc] * y[m];
                z[off + ic + (int64_t)n * jc] = acc;
            }
        free(ps);
        off += (int64_t)n * n;
    }
}

/* ======================================================================
 * Section 6 problem -div(a grad u) = f on [0,1]^2, u = 0 on the boundary,
 * discretised with cell-centred finite volumes: interior face weight is the
 * harmonic mean 2 a_P a_N / (a_P + a_N); a wall face has the cell value at
 * distance h/2, i.e. weight 2 a_P and no neighbour.
 * ====================================================================== */
static double hmean(double ap, double an)
{
    return 2.0 * ap * an / (ap + an);
}

/* unscaled stencil of cell (i,j): neighbour weights (0 at walls), diagonal */
static void stencil(int n, const double *a, int i, int j, double *wE,
                    double *wW, double *wN, double *wS, double *diag)
{
    double ap = a[i + n * j];
    double d = 0.0;
    *wE = *wW = *wN = *wS = 0.0;
    if (i + 1 < n) { *wE = hmean(ap, a[i + 1 + n * j]); d += *wE; } else d += 2.0 * ap;
    if (i > 0)     { *wW = hmean(ap, a[i - 1 + n * j]); d += *wW; } else d += 2.0 * ap;
    if (j + 1 < n) { *wN = hmean(ap, a[i + n * (j + 1)]); d += *wN; } else d += 2.0 * ap;
    if (j > 0)     { *wS = hmean(ap, a[i + n * (j - 1)]); d += *wS; } else d += 2.0 * ap;
    *diag = d;
}

static double nbr(int n, const double *u, int i, int j)
{
    if (i < 0 || j < 0 || i >= n || j >= n)
        return 0.0;
    return u[i + n * j];
}

/* (A u)_P = h^-2 times the net flux out of cell P, summed face by face: an
 * interior face contributes w_f (u_P - u_N), a wall face 2 a_P u_P.  Summing
 * the differences, rather than D u_P minus the neighbour terms, keeps the
 * rounding error proportional to the fluxes instead of to a_P u_P / h^2. */
void oracle_apply(int n, const double *a, const double *u, double *out)
{
    double inv_h2 = (double)n * (double)n;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            double ap = a[i + n * j], up = u[i + n * j], v = 0.0;
            v += i + 1 < n ? hmean(ap, a[i + 1 + n * j]) * (up - u[i + 1 + n * j]) : 2.0 * ap * up;
            v += i > 0 ? hmean(ap, a[i - 1 + n * j]) * (up - u[i - 1 + n * j]) : 2.0 * ap * up;
            v += j + 1 < n ? hmean(ap, a[i + n * (j + 1)]) * (up - u[i + n * (j + 1)]) : 2.0 * ap * up;
            v += j > 0 ? hmean(ap, a[i + n * (j - 1)]) * (up - u[i + n * (j - 1)]) : 2.0 * ap * up;
            out[i + n * j] = inv_h2 * v;
        }
}

/* Cholesky factorisation of the SPD pentadiagonal matrix h^2 A in band
 * storage (half bandwidth n, lexicographic order), then two triangular
 * solves with right-hand side h^2 f. */
int oracle_direct_solve(int n, const double *a, const double *f, double *u)
{
    int64_t M = (int64_t)n * n, bw = n;
    /* L[p][d] = L(p, p-d), d = 0..bw */
    double *L = (double *)calloc((size_t)M * (bw + 1), sizeof(double));
    double *Ab = (double *)calloc((size_t)M * (bw + 1), sizeof(double));
    if (!L || !Ab) {
        free(L);
        free(Ab);
        return -1;
    }
#define BAND(X, p, q) X[(size_t)(p) * (bw + 1) + ((p) - (q))]
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            double wE, wW, wN, wS, d;
            stencil(n, a, i, j, &wE, &wW, &wN, &wS, &d);
            int64_t p = i + (int64_t)n * j;
            BAND(Ab, p, p) = d;
            if (i > 0) BAND(Ab, p, p - 1) = -wW;
            if (j > 0) BAND(Ab, p, p - n) = -wS;
        }
    int status = 0;
    for (int64_t p = 0; p < M && status == 0; ++p) {
        int64_t q0 = p - bw < 0 ? 0 : p - bw;
        for (int64_t q = q0; q <= p; ++q) {
            double sum = BAND(Ab, p, q);
            for (int64_t t = q0; t < q; ++t)
                sum -= BAND(L, p, t) * BAND(L, q, t);
            if (q == p) {
                if (!(sum > 0.0)) {
                    status = -1;
                    break;
                }
                BAND(L, p, p) = sqrt(sum);
            } else {
                BAND(L, p, q) = sum / BAND(L, q, q);
            }
        }
    }
    if (status == 0) {
        double h2 = 1.0 / ((double)n * (double)n);
        /* L v = h^2 f */
        for (int64_t p = 0; p < M; ++p) {
            double sum = h2 * f[p];
            int64_t q0 = p - bw < 0 ? 0 : p - bw;
            for (int64_t q = q0; q < p; ++q)
                sum -= BAND(L, p, q) * u[q];
            u[p] = sum / BAND(L, p, p);
        }
        /* L^T u = v */
        for (int64_t p = M - 1; p >= 0; --p) {
            double sum = u[p];
            int64_t q1 = p + bw >= M ? M - 1 : p + bw;
            for (int64_t q = p + 1; q <= q1; ++q)
                sum -= BAND(L, q, p) * u[q];
            u[p] = sum / BAND(L, p, p);
        }
    }
#undef BAND
    free(L);
    free(Ab);
    return status;
}

/* Neumaier's compensated summation */
typedef struct {
    double s, c;
} ksum;

static void ksum_add(ksum *k, double v)
{
    double t = k->s + v;
    if (fabs(k->s) >= fabs(v))
        k->c += (k->s - t) + v;
    else
        k->c += (v - t) + k->s;
    k->s = t;
}

void oracle_qoi(int n, const double *u, double *q_mean, double *q_ctr)
{
    ksum k = {0.0, 0.0};
    for (int64_t p = 0; p < (int64_t)n * n; ++p)
        ksum_add(&k, u[p]);
    *q_mean = (k.s + k.c) / ((double)n * (double)n);
    int c = n / 2;
    *q_ctr = 0.25 * (u[(c - 1) + n * (c - 1)] + u[c + n * (c - 1)] +
                     u[(c - 1) + n * c] + u[c + n * c]);
}

/* ======================================================================
 * Section 4: multigrid correction scheme, V-cycle and full multigrid.
 * Smoother: red-black Gauss-Seidel (red = (i+j) even).  Restriction: mean of
 * the 4 fine cells.  Prolongation: bilinear (9,3,3,1)/16 with odd reflection
 * of the coarse values across the Dirichlet walls.  Coarsest grid (2x2):
 * exact solve.  FMG interpolation: the same bilinear prolongation.
 * ====================================================================== */
typedef struct {
    const oracle_problem *P;
    int G;
    const double *a[32];   /* coefficient on level g */
    double *e[32];         /* V-cycle iterate / correction on level g */
    double *f[32];         /* right-hand side on level g */
    double *r[32];         /* residual scratch on level g */
    int *trace, *marks, cap, len;
} fmg_state;

static void trace_visit(fmg_state *S, int g)
{
    if (!S->trace)
        return;
    if (S->len > 0 && S->trace[S->len - 1] == g)
        return;                            /* consecutive repeat: same node */
    if (S->len < S->cap) {
        S->trace[S->len] = g;
        if (S->marks)
            S->marks[S->len] = 0;
    }
    S->len++;
}

static void trace_mark(fmg_state *S)
{
    if (S->trace && S->marks && S->len > 0 && S->len <= S->cap)
        S->marks[S->len - 1] = 1;
}

static void rb_sweep(int n, const double *a, const double *f, double *u, int colour)
{
    double h2 = 1.0 / ((double)n * (double)n);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            if (((i + j) & 1) != colour)
                continue;
            double wE, wW, wN, wS, d;
            stencil(n, a, i, j, &wE, &wW, &wN, &wS, &d);
            double v = h2 * f[i + n * j] + wE * nbr(n, u, i + 1, j) +
                       wW * nbr(n, u, i - 1, j) + wN * nbr(n, u, i, j + 1) +
                       wS * nbr(n, u, i, j - 1);
            u[i + n * j] = v / d;
        }
}

static void residual(int n, const double *a, const double *f, const double *u, double *r)
{
    oracle_apply(n, a, u, r);
    for (int64_t p = 0; p < (int64_t)n * n; ++p)
        r[p] = f[p] - r[p];
}

static void restrict_mean(int nc, const double *r, double *fc)
{
    int n = 2 * nc;
    for (int J = 0; J < nc; ++J)
        for (int I = 0; I < nc; ++I)
            fc[I + nc * J] = 0.25 * (r[2 * I + n * (2 * J)] + r[2 * I + 1 + n * (2 * J)] +
                                     r[2 * I + n * (2 * J + 1)] + r[2 * I + 1 + n * (2 * J + 1)]);
}

/* coarse value with odd reflection across each wall crossed */
static double coarse_odd(int nc, const double *e, int I, int J)
{
    double sgn = 1.0;
    if (I < 0) { I = 0; sgn = -sgn; }
    if (I >= nc) { I = nc - 1; sgn = -sgn; }
    if (J < 0) { J = 0; sgn = -sgn; }
    if (J >= nc) { J = nc - 1; sgn = -sgn; }
    return sgn * e[I + nc * J];
}

/* out = P e (add == 0) or out += P e (add == 1) */
static void prolong(int nc, const double *e, double *out, int add)
{
    int n = 2 * nc;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            int I = i / 2, J = j / 2;
            int sx = (i % 2) ? 1 : -1, sy = (j % 2) ? 1 : -1;
            double v = (9.0 * coarse_odd(nc, e, I, J) + 3.0 * coarse_odd(nc, e, I + sx, J) +
                        3.0 * coarse_odd(nc, e, I, J + sy) + coarse_odd(nc, e, I + sx, J + sy)) /
                       16.0;
            if (add)
                out[i + n * j] += v;
            else
                out[i + n * j] = v;
        }
}

/* V(mu1, mu2) on level g for A_g u = f, u updated in place */
static void vcycle(fmg_state *S, int g, double *u, const double *f)
{
    int n = 2 << g;
    trace_visit(S, g);
    if (g == 0) {
        oracle_direct_solve(n, S->a[0], f, u);
        return;
    }
    for (int it = 0; it < S->P->mu1; ++it) {
        rb_sweep(n, S->a[g], f, u, 0);
        rb_sweep(n, S->a[g], f, u, 1);
    }
    residual(n, S->a[g], f, u, S->r[g]);
    restrict_mean(n / 2, S->r[g], S->f[g - 1]);
    memset(S->e[g - 1], 0, sizeof(double) * (n / 2) * (n / 2));
    vcycle(S, g - 1, S->e[g - 1], S->f[g - 1]);
    trace_visit(S, g);
    prolong(n / 2, S->e[g - 1], u, 1);
    for (int it = 0; it < S->P->mu2; ++it) {
        rb_sweep(n, S->a[g], f, u, 1);
        rb_sweep(n, S->a[g], f, u, 0);
    }
}

/* The transfer operators, one red-black half-sweep and one V-cycle, exported
 * so that the tests can pin each of them against dense matrices built from
 * their definitions. */
void oracle_restrict(int nc, const double *r, double *fc)
{
    restrict_mean(nc, r, fc);
}

void oracle_prolong(int nc, const double *e, double *out, int add)
{
    prolong(nc, e, out, add);
}

void oracle_rb_sweep(int n, const double *a, const double *f, double *u, int colour)
{
    rb_sweep(n, a, f, u, colour);
}

int oracle_vcycle(const oracle_problem *P, int g, const double *a_all, double *u,
                  const double *f)
{
    fmg_state S;
    memset(&S, 0, sizeof(S));
    S.P = P;
    S.G = g;
    int64_t off = 0;
    int ok = 1;
    for (int l = 0; l <= g; ++l) {
        int64_t m = (int64_t)(2 << l) * (2 << l);
        S.a[l] = a_all + off;
        S.e[l] = (double *)calloc(m, sizeof(double));
        S.f[l] = (double *)calloc(m, sizeof(double));
        S.r[l] = (double *)calloc(m, sizeof(double));
        ok &= S.e[l] && S.f[l] && S.r[l];
        off += m;
    }
    if (ok)
        vcycle(&S, g, u, f);
    for (int l = 0; l <= g; ++l) {
        free(S.e[l]);
        free(S.f[l]);
        free(S.r[l]);
    }
    return ok ? 0 : -1;
}

static double dot(int64_t m, const double *x, const double *y)
{
    ksum k = {0.0, 0.0};
    for (int64_t p = 0; p < m; ++p)
        ksum_add(&k, x[p] * y[p]);
    return k.s + k.c;
}

static double norm2(int64_t m, const double *v)
{
    return sqrt(dot(m, v, v));
}

/* rtol mode, one FMG stage on level g: solve A_g x = 1 from the interpolated
 * initial guess x to ||1 - A x||_2 / ||1||_2 <= rtol.  The paper runs a
 * fixed number of V-cycles per stage and says nothing about iterating to a
 * tolerance; this mode is flexible preconditioned conjugate gradients with one
 * V(mu1, mu2) cycle from a zero initial guess as the preconditioner z = B r
 * (Notay, SIAM J. Sci. Comput. 22 (2000): beta = (z, r - r_old) / (z_old,
 * r_old)), and the residual is recomputed from x at every step.  Returns the
 * number of preconditioner applications; *relres gets the final ratio;
 * *bad = 1 if the stage stopped above rtol: at max_iters, or because four
 * steps in a row did not bring the ratio 10% below its best value so far
 * (the accuracy a computed FP64 residual can show is bounded below by
 * rounding; iterating on does not lower it). */
static int stage_refine(fmg_state *S, int g, double *x, const double *ones, double *relres,
                        int *bad)
{
    int n = 2 << g;
    int64_t m = (int64_t)n * n;
    double *r = (double *)malloc(sizeof(double) * m);
    double *r_old = (double *)malloc(sizeof(double) * m);
    double *z = (double *)malloc(sizeof(double) * m);
    double *p = (double *)calloc(m, sizeof(double));
    double *q = (double *)malloc(sizeof(double) * m);
    double nf = norm2(m, ones), rz_old = 0.0;
    int it = 0;
    residual(n, S->a[g], ones, x, r);
    double rho = norm2(m, r) / nf;
    double best = rho;                                 /* last 10% improvement */
    int since = 0;                                     /* steps since then */
    *bad = 0;
    while (rho > S->P->rtol) {
        if (it >= S->P->max_iters || since >= 4) {
            *bad = 1;
            break;
        }
        memset(z, 0, sizeof(double) * m);
        vcycle(S, g, z, r);                            /* z = B r */
        double rz = dot(m, r, z);
        double beta = it == 0 ? 0.0 : (rz - dot(m, r_old, z)) / rz_old;
        for (int64_t i = 0; i < m; ++i)
            p[i] = z[i] + beta * p[i];
        oracle_apply(n, S->a[g], p, q);                /* q = A p */
        double alpha = rz / dot(m, p, q);
        for (int64_t i = 0; i < m; ++i)
            x[i] += alpha * p[i];
        memcpy(r_old, r, sizeof(double) * m);
        residual(n, S->a[g], ones, x, r);
        rho = norm2(m, r) / nf;
        rz_old = rz;
        ++it;
        if (rho < 0.9 * best) {
            best = rho;
            since = 0;
        } else {
            ++since;
        }
    }
    *relres = rho;
    free(r);
    free(r_old);
    free(z);
    free(p);
    free(q);
    return it;
}

int oracle_fmg(const oracle_problem *P, int G, const double *a_all,
               double *qoi, int *iters, double *relres, double *u_out,
               int *trace, int *marks, int trace_cap, int *trace_len)
{
    fmg_state S;
    memset(&S, 0, sizeof(S));
    S.P = P;
    S.G = G;
    S.trace = trace;
    S.marks = marks;
    S.cap = trace_cap;
    double *sol[32];
    double *ones[32];
    int64_t off = 0;
    for (int g = 0; g <= G; ++g) {
        int64_t m = (int64_t)(2 << g) * (2 << g);
        S.a[g] = a_all + off;
        S.e[g] = (double *)calloc(m, sizeof(double));
        S.f[g] = (double *)calloc(m, sizeof(double));
        S.r[g] = (double *)calloc(m, sizeof(double));
        sol[g] = (double *)calloc(m, sizeof(double));
        ones[g] = (double *)malloc(sizeof(double) * m);
        for (int64_t p = 0; p < m; ++p)
            ones[g][p] = 1.0;
        off += m;
    }
    int noconv = 0;

    /* initial descent of the FMG figure: problem set-up on every level */
    for (int g = G; g > 0; --g)
        trace_visit(&S, g);
    /* stage 0: exact solve on the coarsest grid */
    vcycle(&S, 0, sol[0], ones[0]);
    trace_mark(&S);
    for (int g = 0; g <= G; ++g) {
        int n = 2 << g;
        int64_t m = (int64_t)n * n;
        if (g > 0) {
            /* nested iteration: interpolated coarse solution as initial guess */
            trace_visit(&S, g);
            prolong(n / 2, sol[g - 1], sol[g], 0);
            if (P->rtol > 0.0) {
                double rho;
                int bad;
                int it = stage_refine(&S, g, sol[g], ones[g], &rho, &bad);
                noconv |= bad;
                if (relres) relres[g] = rho;
                if (iters) iters[g] = it;
            } else {
                for (int c = 0; c < P->mu0; ++c)
                    vcycle(&S, g, sol[g], ones[g]);
                if (iters) iters[g] = P->mu0;
                if (relres) relres[g] = -1.0;
            }
            trace_mark(&S);
        } else {
            if (iters) iters[0] = 0;
            if (relres) {
                if (P->rtol > 0.0) {
                    residual(n, S.a[0], ones[0], sol[0], S.r[0]);
                    relres[0] = norm2(m, S.r[0]) / norm2(m, ones[0]);
                } else {
                    relres[0] = -1.0;
                }
            }
        }
        if (qoi)
            oracle_qoi(n, sol[g], &qoi[2 * g], &qoi[2 * g + 1]);
    }
    if (u_out)
        memcpy(u_out, sol[G], sizeof(double) * (2 << G) * (2 << G));
    if (trace_len)
        *trace_len = S.len;
    for (int g = 0; g <= G; ++g) {
        free(S.e[g]);
        free(S.f[g]);
        free(S.r[g]);
        free(sol[g]);
        free(ones[g]);
    }
    return noconv;
}

/* ---- one sample / a batch ------------------------------------------------ */
int oracle_sample_from_field(const oracle_problem *P, int k, const double *z,
                             int method, double *qoi, int *iters, double *relres)
{
    int G = P->g0 + k;
    int64_t M = oracle_field_size(P, k);
    double *a = (double *)malloc(sizeof(double) * M);
    for (int64_t p = 0; p < M; ++p)
        a[p] = exp(z[p]);                 /* lognormal coefficient a = exp(z) */
    int status = 0;
    if (method == 0) {
        double *q_all = (double *)malloc(sizeof(double) * 2 * (G + 1));
        int *it_all = (int *)malloc(sizeof(int) * (G + 1));
        double *rr_all = (double *)malloc(sizeof(double) * (G + 1));
        status = oracle_fmg(P, G, a, q_all, it_all, rr_all, NULL, NULL, NULL, 0, NULL);
        for (int l = 0; l <= k; ++l) {
            qoi[2 * l] = q_all[2 * (P->g0 + l)];
            qoi[2 * l + 1] = q_all[2 * (P->g0 + l) + 1];
            if (iters) iters[l] = it_all[P->g0 + l];
            if (relres) relres[l] = rr_all[P->g0 + l];
        }
        free(q_all);
        free(it_all);
        free(rr_all);
    } else {
        int64_t off = 0;
        for (int g = 0; g <= G; ++g) {
            int n = 2 << g;
            int64_t m = (int64_t)n * n;
            if (g >= P->g0) {
                int l = g - P->g0;
                double *f = (double *)malloc(sizeof(double) * m);
                double *u = (double *)malloc(sizeof(double) * m);
                for (int64_t p = 0; p < m; ++p)
                    f[p] = 1.0;
                if (oracle_direct_solve(n, a + off, f, u) != 0)
                    status = -1;
                oracle_qoi(n, u, &qoi[2 * l], &qoi[2 * l + 1]);
                if (iters) iters[l] = 0;
                if (relres) relres[l] = -1.0;
                free(f);
                free(u);
            }
            off += m;
        }
    }
    free(a);
    return status;
}

int oracle_sample(const oracle_problem *P, int k, const double *y, int method,
                  double *qoi)
{
    int64_t M = oracle_field_size(P, k);
    double *z = (double *)malloc(sizeof(double) * M);
    oracle_field(P, y, k, z);
    int st = oracle_sample_from_field(P, k, z, method, qoi, NULL, NULL);
    free(z);
    return st;
}

int oracle_batch(const oracle_problem *P, int k, int B, const double *y,
                 int method, double *qoi, int nthreads)
{
    int bad = 0;
#ifdef _OPENMP
    if (nthreads <= 0)
        nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads) reduction(+ : bad)
#endif
    for (int b = 0; b < B; ++b)
        bad += oracle_sample(P, k, y + (int64_t)b * P->s, method,
                             qoi + (int64_t)b * (k + 1) * 2) != 0;
    (void)nthreads;
    return bad;
}
