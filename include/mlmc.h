/*
 * mlmc.h -- C ABI of the MI355X (gfx950) library for the per-sample hot path
 * of the multigrid multilevel (quasi-)Monte Carlo method with sample
 * recycling (Robbe, Nuyens, Vandewalle).
 *
 * Problem (Section 1, eq. PDE; Section 6 "Discretization"):
 *   -div(a(x,y) grad u(x,y)) = 1 on D = [0,1]^2, u = 0 on the boundary,
 *   a = exp(z), z a zero-mean Gaussian field given by its truncated KL
 *   expansion (Section 5, eq. truncatedKL) with the separable exponential
 *   covariance sigma^2 exp(-|x1-x1'|/lambda - |x2-x2'|/lambda).
 * Per sample: points (Section 3.2) -> KL field on every grid of the
 * hierarchy -> full multigrid (Section 4, figure FMG) -> the QoI of every FMG
 * stage, i.e. of every level l <= k, recycled into the level differences
 * F_l - F_{l-1} (Section 3.2, eq. Upsilon-reuse) -> estimators.
 *
 * Grids.  Multigrid level g has n_g = 2^(g+1) cells per side (g = 0 is 2x2,
 * solved exactly).  MLMC level l has n0 * 2^l cells per side, i.e. it is
 * multigrid level g0 + l with g0 = log2(n0) - 1.  Cell (i,j) of an n x n grid
 * has centre ((i+1/2)/n, (j+1/2)/n) and flat index i + n*j (i fastest).
 * A per-sample field over levels 0..G is stored level after level.
 *
 * Discretisation: cell-centred finite volumes; an interior face carries the
 * harmonic mean 2 a_P a_N / (a_P + a_N), a boundary face 2 a_P (the cell value
 * at distance h/2 from the wall).  Smoother: red-black Gauss-Seidel, red =
 * (i+j) even, red first before the coarse-grid correction, black first after.
 * Restriction: mean of the four children.  Prolongation and FMG
 * interpolation: bilinear (9,3,3,1)/16 with odd reflection across walls.
 *
 * Conventions for every entry point:
 *  - Return value: mlmc_status, 0 on success, negative on error.  No C++
 *    exception or longjmp crosses the ABI.
 *  - Pointers named *_dev are device pointers on the context's device; all
 *    other pointers are host pointers.  The caller owns every buffer it
 *    passes; the context owns its own workspace (allocated at create).
 *  - Calls that take a stream enqueue their work on that hipStream_t (NULL =
 *    the default stream) and return without waiting, except where stated.
 *  - Argument errors (MLMC_E_INVAL) are detected before any GPU work is
 *    enqueued and leave every output untouched.
 *  - A context must not be used by two host threads at once; calls that
 *    share a context are ordered by the host, and their device work is
 *    ordered by the streams the caller passes.
 */
#ifndef MLMC_H
#define MLMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MLMC_OK = 0,
    MLMC_E_INVAL = -1,   /* invalid argument; nothing was written */
    MLMC_E_NOMEM = -2,   /* device memory (HBM) budget exceeded */
    MLMC_E_HIP = -3,     /* a HIP runtime call failed; see mlmc_last_error */
    MLMC_E_NOCONV = -4,  /* refinement stopped above rtol; outputs written */
    MLMC_E_STATE = -5    /* context unusable (e.g. earlier HIP failure) */
} mlmc_status;

enum { MLMC_FP64 = 0, MLMC_MIXED = 1 };

/* QoI selection (Section 6 "Quantity of interest" and its readings):
 * MEAN   = n^-2 sum_P u_P (midpoint rule for the mean of u),
 * CENTER = mean of the four cells touching (1/2,1/2) (a grid vertex). */
enum { MLMC_QOI_MEAN = 1u, MLMC_QOI_CENTER = 2u };

enum { MLMC_POINTS_LATTICE = 0, MLMC_POINTS_EXPLICIT = 1 };

/* Covariance of the Gaussian field z (Section 5):
 * SEPARABLE_EXP  exp(-|x1-x1'|/lambda - |x2-x2'|/lambda), KL eigenpairs from
 *                the 1-D characteristic equation (products of 1-D modes);
 * MATERN         isotropic Matern, eq. matern, smoothness nu, rho = |x-x'|/lambda;
 *                KL eigenpairs by the Nystrom method on the nystrom_q^2
 *                midpoint nodes of the unit square, eigenfunctions at the cell
 *                centres by the Nystrom interpolation formula. */
enum { MLMC_FIELD_SEPARABLE_EXP = 0, MLMC_FIELD_MATERN = 1 };

typedef struct mlmc_ctx_s *mlmc_ctx;

typedef struct {
    int32_t n0;           /* cells per side on MLMC level 0; power of two >= 2 */
    int32_t num_levels;   /* MLMC levels 0..num_levels-1; finest n0 * 2^(L) <= 4096 */
    int32_t s;            /* number of KL terms (stochastic dimension), 1..4096 */
    double corr_len;      /* correlation length lambda > 0 */
    double sigma2;        /* pointwise variance sigma^2 >= 0 of the full field z */
    int32_t mu0;          /* V-cycles per FMG stage (fixed-cycle mode), >= 1 */
    int32_t mu1, mu2;     /* pre-/post-smoothing red-black sweeps, >= 0, sum >= 1 */
    double rtol;          /* 0: fixed mu0 cycles.  > 0: every stage iterates
                             V-cycle-preconditioned flexible CG until
                             ||f-Au||_2/||f||_2 <= rtol, max_iters steps, or
                             four steps in a row that do not bring the ratio
                             10% below its best value (the FP64 rounding
                             floor, about eps * condition) */
    int32_t max_iters;    /* refinement cap per stage when rtol > 0 (>= 1) */
    int32_t precision;    /* MLMC_FP64, or MLMC_MIXED (field from bf16 digit
                             products on the matrix cores, see mlmc_field;
                             a = exp(z) kept in FP32 for FP32 V-cycles and in
                             FP64 for the residual of the FP64 refinement;
                             needs rtol > 0) */
    uint32_t qoi_mask;    /* non-empty subset of MLMC_QOI_MEAN | MLMC_QOI_CENTER;
                             nq = number of bits, QoI q in increasing bit order */
    int32_t num_shifts;   /* R, number of random shifts (>= 1 if shifts given) */
    const uint32_t *genvec;  /* host [s]: generating vector z mod 2^32 (odd
                                entries give full projections); NULL disables
                                lattice points.  Copied at create. */
    const uint64_t *shifts;  /* host [num_levels][num_shifts][s]: shift
                                Delta_l^(r)_j as 64-bit fixed point (value / 2^64);
                                NULL disables lattice points.  Copied at create. */
    int64_t max_batch;    /* samples of the finest level solved at once; sizes
                             the workspace (coarser levels run larger chunks) */
    int32_t field_kind;   /* MLMC_FIELD_* */
    double nu;            /* MATERN: smoothness, 0 < nu <= 8 */
    int32_t nystrom_q;    /* MATERN: quadrature nodes per side, 4..96 (0: 32);
                             s <= nystrom_q^2 */
} mlmc_config;

/* A set of samples, all with finest MLMC level `level` (Algorithm 1,
 * SampleAndSolve: the solve yields every level tau <= level).
 * LATTICE (Section 3.2, and the lattice sequence of Section 6 "QMC method"):
 *   point n of shift r is x_j = (bitrev32(n) z_j mod 2^32) 2^32 + Delta_{level,r,j}
 *   (mod 2^64), u_j = (2 floor(x_j / 2^12) + 1) 2^-53, y_j = Phi^-1(u_j).
 *   Samples are ordered shift-major: b = (r - shift_begin) * (n_end - n_begin)
 *   + (n - n_begin), B = (shift_end - shift_begin) * (n_end - n_begin).
 *   Requires 0 <= n_begin <= n_end <= 2^32 and
 *   0 <= shift_begin < shift_end <= num_shifts.
 * EXPLICIT (plain Monte Carlo or any caller-chosen y): y_dev [B][s] FP64 on the
 *   device, B = n_end - n_begin, shift_end - shift_begin must be 1 (the
 *   replica index is only a label). */
typedef struct {
    int32_t kind;
    int32_t level;
    int32_t shift_begin, shift_end;
    int64_t n_begin, n_end;
    const double *y_dev;
} mlmc_points;

typedef struct {
    int64_t samples;          /* B */
    int32_t max_iters_used;   /* rtol mode: largest refinement count of any
                                 stage of any sample; fixed mode: mu0 */
    double max_rel_residual;  /* rtol mode: largest final ||f-Au||/||f||;
                                 fixed mode: -1 */
    int64_t not_converged;    /* rtol mode: samples with a stage that stopped
                                 above rtol (max_iters or stalled) */
} mlmc_solve_info;

/* Create a context on `device`: validates cfg, builds the KL mode table and
 * basis (analytic 1-D eigenpairs, Section 5 with the exponential kernel; or,
 * for MATERN, the Nystrom eigenpairs: the weighted covariance matrix of the
 * nodes formed on the device, its symmetric eigendecomposition by rocSOLVER,
 * the interpolation formula evaluated at every cell centre of every level as
 * one FP64 matrix-core product), MATERN needs device >= 0;
 * uploads generating vector and shifts, allocates the workspace for
 * max_batch finest-level samples.  E_NOMEM if it does not fit in free HBM.
 * Synchronous.  device < 0 creates a host-only context that makes no HIP
 * call: mlmc_kl_modes, mlmc_fmg_trace, mlmc_field_size and mlmc_num_qoi work,
 * the GPU entry points return MLMC_E_STATE. */
mlmc_status mlmc_create(const mlmc_config *cfg, int device, mlmc_ctx *out);

/* Free the context and its device memory.  Synchronises the device first.
 * NULL is accepted. */
mlmc_status mlmc_destroy(mlmc_ctx ctx);

/* Values per sample of a field over MG levels 0..G(level), i.e.
 * sum_{g <= g0+level} n_g^2; 0 for an invalid level. */
int64_t mlmc_field_size(mlmc_ctx ctx, int32_t level);

/* Number of QoIs selected by qoi_mask (1 or 2); 0 for a NULL context. */
int32_t mlmc_num_qoi(mlmc_ctx ctx);

/* Section 3.2: the points of `pts`.  x_dev [B][s] receives the shifted lattice
 * points in 64-bit fixed point (LATTICE only; NULL to skip), y_dev [B][s] the
 * normals y = Phi^-1(u) (NULL to skip; EXPLICIT copies the input). */
mlmc_status mlmc_points_gen(mlmc_ctx ctx, const mlmc_points *pts,
                            uint64_t *x_dev, double *y_dev, void *hip_stream);

/* Section 5, eq. truncatedKL: z(x) = sigma sum_{m<s} sqrt(theta_m) psi_m(x) y_m
 * at the cell centres of every MG level 0..G(level) of every sample, as one
 * dense product Y [B][s] x basis [s][M].  z_dev [B][M], M = mlmc_field_size
 * (sample-major, levels in order).  FP64 context: FP64 product on the matrix
 * cores.  MIXED context: the product the MIXED solve uses, with every sample
 * row of Y and every cell column of the basis scaled by a power of two
 * 2^E > max |entry| and written as five bf16 digits, the fifteen digit
 * products of weight 2^0 .. 2^-32 on the matrix cores summed exactly and
 * folded into FP64; |error| <= 2 s 2^(E_y + E_b - 38) per cell, without
 * rounding bias, returned as double. */
mlmc_status mlmc_field(mlmc_ctx ctx, const mlmc_points *pts, double *z_dev,
                       void *hip_stream);

/* mlmc_field for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same z, bit for bit, with the points' staging (Y for lattice points) and,
 * in a MIXED context, their digits and scale exponents held in a static
 * device array of the library (32 MiB per GPU, resolved once per device at
 * mlmc_create and held until the process ends) instead of the context's
 * workspace.  The call allocates nothing.  E_INVAL if the set needs more
 * than the 32 MiB: 8 B s per lattice sample, plus in a MIXED context 10 B
 * per padded sample row and mode (rows padded to 64, modes to 32) and 4 B
 * per padded row, each part rounded up to 256 bytes.  Every call on a GPU
 * shares that GPU's array: calls whose device work overlaps (on different
 * streams or host threads) race; calls ordered on one stream do not. */
mlmc_status mlmc_field_static(mlmc_ctx ctx, const mlmc_points *pts, double *z_dev,
                              void *hip_stream);

/* The hot path for one set of samples (Algorithm 1, SampleAndSolve body):
 * field (unless z_dev is given) -> a = exp(z) -> FMG from the 2x2 grid up to
 * level g0+pts->level, recording the QoI at the end of every stage that is an
 * MLMC level (Section 4, the circled solutions of the FMG figure) -> level
 * differences.
 *   z_dev    [B][M] or NULL: log-coefficient to use instead of computing it.
 *   qoi_dev  [B][level+1][nq] or NULL: F_l of every sample and level.
 *   sums_dev [R_b][nq][level+1][2] or NULL, R_b = shift_end - shift_begin:
 *            sum over the samples of shift r of (F_l - F_{l-1}) and of its
 *            square (F_{-1} = 0), compensated FP64 sums.
 *   info     host, optional; filling it synchronises the stream.
 * Returns MLMC_E_NOCONV (outputs still written) if info was requested and
 * some sample has a stage that stopped above rtol.
 * With rtol == 0 (fixed cycles) and info == NULL the call only enqueues
 * kernels on hip_stream (no host synchronisation, no allocation, no memset),
 * so it may be captured into a HIP graph and replayed: a replay recomputes
 * the points, the field and the solve into the same qoi_dev and sums_dev.
 * The context's workspace is shared by every call on it, so replays and
 * other calls on the context must not overlap.  With rtol > 0 the host reads
 * the convergence flags after every refinement step on grids >= 64^2, and
 * the call cannot be captured. */
mlmc_status mlmc_fmg_solve(mlmc_ctx ctx, const mlmc_points *pts,
                           const double *z_dev, double *qoi_dev,
                           double *sums_dev, mlmc_solve_info *info,
                           void *hip_stream);

/* Estimator input (Section 3.2, eqs. MLQMC, Upsilon-reuse, MGMLQMC):
 * sums[k][r][q][l][2] as produced by mlmc_fmg_solve for the samples of shift r
 * with finest level k (entries with l > k are ignored), n_per_level[k] = N_k
 * samples per shift with finest level k. */
typedef struct {
    int32_t num_levels;       /* L + 1 */
    int32_t num_shifts;       /* R >= 1 */
    int32_t nq;               /* 1 or 2 */
    int32_t reuse;            /* 1: recycle coarse solutions (MG-MLQMC) */
    const int64_t *n_per_level;
    const double *sums;
} mlmc_est_input;

/* Estimator outputs (host arrays, caller-allocated):
 *   upsilon     [nq][L+1][R]  Upsilon_{l,r} (eq. Upsilon-reuse, or its
 *                             no-recycling form 1/N_l sum over level-l samples)
 *   upsilon_bar [nq][L+1]     mean over shifts (eq. Upsilon-reuse-bar)
 *   var_level   [nq][L+1]     R >= 2: sum_r (Upsilon_{l,r}-bar)^2 / (R(R-1))
 *                             (eq. sample_variances); R = 1 without reuse:
 *                             s_l^2 / N_l (eq. vardecomp); R = 1 with reuse: NaN
 *   q_shift     [nq][R]       Q_r = sum_l Upsilon_{l,r}
 *   q_bar       [nq]          mean over shifts (eq. MLQMC / MGMLQMC)
 *   var_q       [nq]          eq. varovershifts / var_of_mgmlqmc (R >= 2);
 *                             sum of var_level (R = 1, no reuse); NaN otherwise */
typedef struct {
    double *upsilon;
    double *upsilon_bar;
    double *var_level;
    double *q_shift;
    double *q_bar;
    double *var_q;
} mlmc_est_output;

/* Host-only and synchronous; touches no GPU.  Levels without samples at or
 * above them (sum_{i>=l} N_i = 0) give Upsilon = 0. */
mlmc_status mlmc_estimate(const mlmc_est_input *in, mlmc_est_output *out);

/* The ordered 2-D KL mode table (descending theta_i theta_j, ties by i
 * ascending): i_out, j_out [s] 1-based 1-D indices, theta_out [s] products.
 * MATERN: i_out = j_out = 0, theta_out the s largest Nystrom eigenvalues,
 * descending.  Any output may be NULL.  Host-only. */
mlmc_status mlmc_kl_modes(mlmc_ctx ctx, int32_t *i_out, int32_t *j_out,
                          double *theta_out);

/* The level-visit sequence of the FMG schedule the library runs for finest
 * MLMC level `level` (Section 4, figure FMG): levels[len] are multigrid levels,
 * marks[len] is 1 where a stage solution is recorded.  Consecutive repeats
 * are merged; the initial descent G..1 (problem set-up) is included.  In rtol
 * mode the schedule depends on convergence, so E_INVAL.  Host-only; writes at
 * most cap entries and the full length to *len. */
mlmc_status mlmc_fmg_trace(mlmc_ctx ctx, int32_t level, int32_t *levels,
                           int32_t *marks, int64_t cap, int64_t *len);

/* Live timing of one kernel kind, for measuring the path against its
 * roofline.  Between mlmc_profile_begin and mlmc_profile_end every launch of
 * that kind is bracketed by HIP events on the stream it is launched on, and
 * its algorithmic HBM bytes and flops are accumulated:
 *   SMOOTH   one red-black colour on n^2 cells: a (n^2) + u of the other colour
 *            (n^2/2) + f of the colour (n^2/2, absent when f = 1) read, u of the
 *            colour (n^2/2) written, per sample
 *   RESTRICT residual + restriction: a, u (and f) read on n^2, f_c and the
 *            cleared coarse iterate written on n^2/4
 *   PROLONG  coarse-grid correction: e_c (n^2/4) read, u read and written;
 *            FMG interpolation: e_c read, u written
 *   FIELD    dense product: 2 B s M flops; Y, basis and the output once
 *   QOI, COARSE, POINTS, SUMS: their inputs and outputs once
 * Host-synchronous at end.  At most one kind is profiled at a time. */
enum {
    MLMC_KERNEL_POINTS = 0, MLMC_KERNEL_FIELD = 1, MLMC_KERNEL_SMOOTH = 2,
    MLMC_KERNEL_RESTRICT = 3, MLMC_KERNEL_PROLONG = 4, MLMC_KERNEL_COARSE = 5,
    MLMC_KERNEL_QOI = 6, MLMC_KERNEL_SUMS = 7,
    MLMC_KERNEL_PRE = 8,   /* fused tile pass: mu1 sweeps + residual + restriction;
                              bytes a, u (unless zero or interpolated start), f
                              (unless f = 1) read on n^2, u written on n^2,
                              coarse f written on n^2/4 (+ coarse u read on n^2/4
                              when interpolating) */
    MLMC_KERNEL_POST = 9,  /* fused tile pass: prolongation + correction + mu2
                              sweeps; bytes e_c (n^2/4), a, u, f (unless 1) read,
                              u written */
    MLMC_KERNEL_LDS = 10,  /* LDS-resident hierarchy (up to 16^2 with fixed
                              cycles, 32^2 with rtol): a of all its grids
                              read, f of its top grid read (V-cycle mode), u of
                              its top grid written */
    MLMC_KERNEL_REFINE = 11 /* rtol mode on grids >= 64^2, one flexible-CG step
                              after the V-cycle, per cell of the samples still
                              iterating: dots (z, r, r_old read), p with
                              (p, A p) (a, z, previous p read; p written), x
                              with the new residual (FP64 a, x, p read; x, r
                              written): 24 + 9 w bytes, w the V-cycle word
                              size (24 + 7 w at a stage's first step, which
                              has no r_old or previous p).  The PRE, POST and
                              LDS passes of a refinement step count only the
                              samples still iterating, too */
};
typedef struct {
    int64_t launches;
    double total_ms;      /* sum of the event-measured launch durations */
    double bytes;         /* sum of algorithmic HBM bytes over the launches */
    double flops;         /* sum of algorithmic flops over the launches */
} mlmc_profile_result;
mlmc_status mlmc_profile_begin(mlmc_ctx ctx, int32_t kernel_kind);
mlmc_status mlmc_profile_end(mlmc_ctx ctx, mlmc_profile_result *out);

/* ---- Pass kinds of the large grids and their autotuner -------------------
 * Every V-cycle level above the LDS-resident grids runs one pre pass (mu1
 * red-black sweeps, residual, restriction) and one post pass (prolongation,
 * correction, mu2 sweeps) per cycle, each in one of these kinds:
 *   MLMC_PASS_TILE32  32 x 32 cells and a halo per 256-thread workgroup
 *   MLMC_PASS_TILE16  16 x 16 cells per 128-thread workgroup (four times the
 *                     workgroups: for batches too small to fill the chip)
 *   MLMC_PASS_STREAM  rows streamed through LDS, one sample per workgroup
 *                     of n/2 threads (at least 256; 2 or 4 samples per
 *                     workgroup on 64^2 and 32^2, so that they fill a
 *                     wavefront); FP64 and FP32 V-cycles, 32 <= n <= 2048
 * All kinds give the bits of the same global sweep order, so the choice
 * changes only the time.  The choice is kept per context for each grid side
 * n and batch class c: chunks of Bc samples with 4^(c-1) < Bc <= 4^c (c = 0
 * for one sample), c < MLMC_BATCH_CLASSES (the last class takes every larger
 * chunk).  A new context starts from defaults measured on MI355X, a rule in
 * c, the number of 32 x 32 tiles of the pass, t = 4^c (n/32)^2, and the
 * lanes of a streaming pass, 4^c n/2: TILE16 for t <= 256, TILE32
 * otherwise; STREAM takes the pre and the post pass once it has at least
 * 131072 lanes and t >= 65536 (FP64 V-cycles: t >= 16384 when n <= 64) and
 * the smallest chunk of the class, 4^(c-1) + 1 samples, fills 256
 * workgroups, with FP64 V-cycles up to 1024^2 only.  mlmc_autotune replaces
 * the defaults by what it measures.  A server's slots take the first slot's
 * table. */
enum { MLMC_PASS_TILE32 = 0, MLMC_PASS_TILE16 = 1, MLMC_PASS_STREAM = 2 };
enum { MLMC_BATCH_CLASSES = 10 };
typedef struct {
    int32_t n;             /* grid side of the pass (cells per side) */
    int32_t batch_class;   /* c above */
    int32_t pre, post;     /* MLMC_PASS_* */
    double pre_ms, post_ms;  /* one launch as measured by mlmc_autotune (at
                                min(4^c, capacity) samples); 0 if not measured */
} mlmc_tune_entry;
/* Measures every allowed kind of both passes on every tile grid of levels
 * <= level, for every batch class up to the level's chunk capacity, at the
 * class's largest and smallest chunk, on the context's own workspace (its
 * contents are overwritten; stream-ordered on hip_stream, synchronous on
 * return), and installs per pass the kind whose larger ratio to the fastest
 * kind at the two sizes is smallest.  Solves
 * already enqueued on other streams must have finished.  E_INVAL for a level
 * out of range, E_STATE for a host-only context. */
mlmc_status mlmc_autotune(mlmc_ctx ctx, int32_t level, void *hip_stream);
/* The context's table: one entry per tile grid (coarsest first) and batch
 * class; writes at most max_entries and the full count to *count (host). */
mlmc_status mlmc_tuning_get(mlmc_ctx ctx, mlmc_tune_entry *out, int32_t max_entries,
                            int32_t *count);
/* Installs the kinds of `count` entries (a saved table, or a forced choice);
 * E_INVAL, before any change, if an entry names a grid that is not a tile
 * grid of the context, a class out of range or a kind the grid does not
 * support. */
mlmc_status mlmc_tuning_set(mlmc_ctx ctx, const mlmc_tune_entry *in, int32_t count);

/* ---- Serving loop: continuous batching of solve requests ----------------
 * A server owns num_slots copies of one configuration, each with its own HIP
 * stream, workspace for slot_samples samples and a host thread; the HBM
 * footprint is fixed at create (E_NOMEM if the slots do not fit).  Requests
 * (level, lattice-point range, shift range) join one FIFO queue.  A free slot
 * takes the oldest request and packs behind it every queued request of the
 * same level that still fits (continuous batching: requests arriving while
 * other batches run are admitted as slots free up), generates their points,
 * solves the batch (Algorithm 1's SampleAndSolve, all levels <= level) and
 * copies the QoIs to the host; batches of different levels run concurrently
 * on the slots' streams.  Every sample's result is bitwise the same
 * alone and in any batch. */
typedef struct mlmc_server_s *mlmc_server;

typedef struct {
    int32_t level;                  /* finest MLMC level */
    int32_t shift_begin, shift_end; /* shifts [shift_begin, shift_end) */
    int64_t n_begin, n_end;         /* lattice points [n_begin, n_end) */
    uint64_t tag;                   /* caller's label, returned with the result */
    double *qoi_out;                /* host [B][level+1][nq], B = samples of the
                                       request in lattice order (shift-major);
                                       caller-owned, written before the result
                                       is reported, kept valid until then */
    double *sums_out;               /* host [shift_end-shift_begin][nq][level+1][2]
                                       or NULL: per shift of the request, the
                                       compensated FP64 sums of F_l - F_{l-1}
                                       and of its square over its samples
                                       (Section 3.2, eq. Upsilon-reuse; F_{-1} =
                                       0), bitwise those mlmc_fmg_solve returns
                                       for the same points in one chunk; same
                                       lifetime as qoi_out */
} mlmc_request;

typedef struct {
    uint64_t tag;
    int32_t status;                 /* MLMC_OK, or the solve's error */
    int32_t level;
    int64_t samples;
    int64_t batch_samples;          /* samples of the batch it was solved in */
    double queued_ms;               /* submit -> its batch starts */
    double latency_ms;              /* submit -> QoIs on the host */
    int64_t not_converged;          /* rtol mode: samples of the request with a
                                       stage that stopped above rtol (then
                                       status is MLMC_E_NOCONV, outputs written) */
    double max_rel_residual;        /* rtol mode: largest final ||f-Au||/||f||
                                       of the request's samples; -1 otherwise */
} mlmc_result;

typedef struct {
    int64_t requests, samples;      /* completed */
    int64_t batches;
    double p50_ms, p99_ms, max_ms;  /* latency of the completed requests */
    double busy_s;                  /* first submit -> last completion */
} mlmc_server_stats;

/* cfg as for mlmc_create (cfg->max_batch is replaced by slot_samples; lattice
 * points required).  Each slot's workspace holds slot_samples samples of the
 * finest level; a batch of a coarser level may hold more, as many as fit the
 * same HBM footprint (mlmc_server_capacity).  The KL tables are held once and
 * shared by the slots.  E_INVAL for num_slots < 1, slot_samples < 1 or
 * device < 0. */
mlmc_status mlmc_server_create(const mlmc_config *cfg, int device, int32_t num_slots,
                               int64_t slot_samples, mlmc_server *out);
/* Finishes the queued and running requests, then frees everything. */
mlmc_status mlmc_server_destroy(mlmc_server srv);
/* Thread-safe, non-blocking.  E_INVAL (nothing queued) for a bad range, a
 * level outside the configuration, more samples than a slot holds at that
 * level, or a NULL qoi_out.  Every batch is solved with per-sample
 * convergence flags, so a request's result reports its unconverged samples
 * (rtol mode) with status MLMC_E_NOCONV. */
mlmc_status mlmc_server_submit(mlmc_server srv, const mlmc_request *req);
/* Up to max_results completed results, oldest first; waits up to wait_ms for
 * the first one (0: no wait).  *count receives the number written. */
mlmc_status mlmc_server_poll(mlmc_server srv, mlmc_result *out, int32_t max_results,
                             int32_t wait_ms, int32_t *count);
/* Samples of finest level `level` that one batch (one slot's workspace)
 * holds; 0 for a NULL server or a level outside the configuration. */
int64_t mlmc_server_capacity(mlmc_server srv, int32_t level);
/* Counters and latency percentiles of everything completed so far. */
mlmc_status mlmc_server_stats_get(mlmc_server srv, mlmc_server_stats *out);

const char *mlmc_status_str(mlmc_status st);
/* Text of the last error on ctx (empty string if none); NULL ctx gives the
 * last error of a failed mlmc_create on this thread. */
const char *mlmc_last_error(mlmc_ctx ctx);

#ifdef __cplusplus
}
#endif
#endif /* MLMC_H */
