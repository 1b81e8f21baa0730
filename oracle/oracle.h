/*
 * Plain CPU FP64 oracle for the multigrid multilevel (quasi-)Monte Carlo
 * per-sample path (Robbe, Nuyens, Vandewalle, "Recycling samples in the
 * multigrid multilevel (quasi-)Monte Carlo method").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this code; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code with the GPU library.
 *
 * Conventions (readings of the paper that are fixed here):
 *  - Multigrid level g has n_g = 2^(g+1) cells per side on [0,1]^2 (g = 0 is
 *    the 2x2 coarsest grid).  Cell (i,j), i fastest, has centre
 *    ((i+1/2)/n, (j+1/2)/n); flat index p = i + n*j.
 *  - MLMC level l of a hierarchy with n0 cells on level 0 is multigrid level
 *    g0 + l with g0 = log2(n0) - 1.
 *  - A field on levels 0..G is stored level after level ("level-major"),
 *    each level n_g*n_g values.
 */
#ifndef MLMC_ORACLE_H
#define MLMC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- Section 3.2: randomly shifted rank-1 lattice sequence ------------- */
uint32_t oracle_bitrev32(uint32_t v);
/* x_j = (bitrev32(n) * z_j mod 2^32) * 2^32 + delta_j  (mod 2^64), j < s */
void oracle_lattice_x(const uint32_t *z, int s, const uint64_t *delta,
                      uint64_t n, uint64_t *x);
/* u = (2 floor(x / 2^12) + 1) 2^-53, strictly inside (0,1) */
double oracle_unit(uint64_t x);
/* inverse standard normal CDF by bracketing + Halley on Phi(y) = u */
double oracle_norminv(double u);
/* points n_begin..n_end-1 of one shift: x [B][s] and y = Phi^-1(u) [B][s] */
void oracle_points(const uint32_t *z, int s, const uint64_t *delta,
                   int64_t n_begin, int64_t n_end, uint64_t *x, double *y);

/* ---- Section 5: KL expansion, exponential covariance on [0,1] ---------- */
/* k-th root (k >= 1) of (lam^2 w^2 - 1) sin w - 2 lam w cos w in ((k-1)pi, k pi) */
double oracle_kl_root(double lam, int k);
double oracle_kl_theta(double lam, double w);        /* 2 lam / (1 + lam^2 w^2) */
double oracle_kl_psi(double lam, double w, double x); /* normalised eigenfunction */
/* ordered 2-D mode table: top s products theta_i theta_j, ties by i ascending.
 * mi, mj are 1-based 1-D indices; theta receives theta_i * theta_j. */
int oracle_kl_modes(double lam, int s, int *mi, int *mj, double *theta);

/* ---- problem handle ------------------------------------------------------ */
typedef struct oracle_problem oracle_problem;
oracle_problem *oracle_problem_new(int n0, int num_levels, int s,
                                   double corr_len, double sigma2,
                                   int mu0, int mu1, int mu2,
                                   double rtol, int max_iters);
void oracle_problem_free(oracle_problem *P);
int oracle_finest_mg_level(const oracle_problem *P, int k);  /* G for MLMC level k */
int64_t oracle_field_size(const oracle_problem *P, int k);  /* sum_{g<=G} n_g^2 */

/* z (not exp(z)) at the cell centres of every multigrid level 0..G(k),
 * level-major, by direct summation of the truncated KL expansion */
void oracle_field(const oracle_problem *P, const double *y, int k, double *z);

/* ---- Section 6 discretisation (cell-centred finite volumes) ------------- */
/* out = A u with A = h^-2 [sum_faces w (u_P - u_nbr) + sum_walls 2 a_P u_P] */
void oracle_apply(int n, const double *a, const double *u, double *out);
/* band Cholesky solve of A u = f; returns 0 or -1 if not positive definite */
int oracle_direct_solve(int n, const double *a, const double *f, double *u);
/* Q_mean = n^-2 sum u ; Q_ctr = mean of the 4 cells touching (1/2,1/2) */
void oracle_qoi(int n, const double *u, double *q_mean, double *q_ctr);

/* ---- Section 4: full multigrid with all coarse solutions kept ---------- */
/* a_all: exp(z) on levels 0..G (level-major).  f = 1 on every level.
 * qoi [G+1][2]: QoI of the solution at the end of every FMG stage.
 * iters[G+1], relres[G+1]: per stage iterations (mu0 with fixed cycles; in
 * rtol mode the flexible-CG steps, one V-cycle each) and the final
 * ||f - A u||_2 / ||f||_2 (relres only computed when rtol > 0, else -1).
 * u_out: final solution on level G (n_G^2), may be NULL.
 * trace/marks: visited levels (consecutive repeats merged) and 1 where the
 * stage solution is recorded; may be NULL.  Returns 0, or 1 if some stage
 * hit max_iters before reaching rtol. */
int oracle_fmg(const oracle_problem *P, int G, const double *a_all,
               double *qoi, int *iters, double *relres, double *u_out,
               int *trace, int *marks, int trace_cap, int *trace_len);

/* The pieces of the V-cycle, for the tests that pin them one by one:
 * fc = R r, the mean of the four children (fine grid 2nc x 2nc);
 * out = P e (add = 0) or out += P e (add = 1), bilinear (9,3,3,1)/16 with
 * coarse values reflected oddly across the walls;
 * one Gauss-Seidel half-sweep over the cells of one colour
 * (0 = red = (i+j) even, 1 = black) for A u = f;
 * one V(mu1, mu2) cycle on multigrid level g for A_g u = f, u updated in
 * place, a_all the coefficients of levels 0..g (level-major), mu1 and mu2
 * from the problem.  Returns 0, or -1 if out of memory. */
void oracle_restrict(int nc, const double *r, double *fc);
void oracle_prolong(int nc, const double *e, double *out, int add);
void oracle_rb_sweep(int n, const double *a, const double *f, double *u, int colour);
int oracle_vcycle(const oracle_problem *P, int g, const double *a_all, double *u,
                  const double *f);

/* ---- one sample / a batch ------------------------------------------------ */
/* method 0: FMG (fixed cycles or rtol, as configured); 1: direct solve per level.
 * qoi [k+1][2] for MLMC levels 0..k.  Returns 0 / nonzero as oracle_fmg. */
int oracle_sample_from_field(const oracle_problem *P, int k, const double *z,
                             int method, double *qoi, int *iters,
                             double *relres);
int oracle_sample(const oracle_problem *P, int k, const double *y, int method,
                  double *qoi);
/* B samples y [B][s] -> qoi [B][k+1][2]; OpenMP over samples with nthreads
 * (<= 0: runtime default).  Returns the number of samples that did not
 * converge. */
int oracle_batch(const oracle_problem *P, int k, int B, const double *y,
                 int method, double *qoi, int nthreads);

#ifdef __cplusplus
}
#endif
#endif
