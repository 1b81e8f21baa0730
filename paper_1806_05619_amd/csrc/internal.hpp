// Internal declarations of the MI355X MG-MLQMC library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "mlmc.h"

namespace mlmc {

// Host-side helpers shared by the C entry points (host.hip) and the serving
// loop (server.hip).
mlmc_status create_ctx(const mlmc_config *cfg, int device, mlmc_ctx parent, mlmc_ctx *out);
// samples of finest MLMC level k that one pass over the workspace holds
int64_t level_capacity(mlmc_ctx c, int k);
// mlmc_fmg_solve, and per sample (host arrays of B entries, either may be
// NULL): sample_bad[b] = 1 if a stage of sample b stopped above rtol,
// sample_rho[b] = the largest final residual ratio of its stages (-1 with
// fixed cycles).  Asking for either synchronises the stream, as info does.
mlmc_status fmg_solve_ex(mlmc_ctx ctx, const mlmc_points *pts, const double *z_dev,
                         double *qoi_dev, double *sums_dev, mlmc_solve_info *info,
                         void *hip_stream, int32_t *sample_bad, double *sample_rho);

constexpr int kMaxMgLevels = 12;   // n_g = 2^(g+1) <= 4096
constexpr int kBlock = 256;
constexpr int kLdsMaxLevel = 4;    // grids up to 32^2 run LDS-resident (one workgroup per sample)
constexpr int kLdsMaxLevelFixed = 3;   // fixed-cycle mode: up to 16^2; 32^2 runs the tile passes

// Offset (in cells) of multigrid level g inside a level-major per-sample
// field: sum_{g' < g} 4^(g'+1) = 4 (4^g - 1) / 3.
__host__ __device__ inline int64_t level_offset(int g) { return 4 * (((int64_t)1 << (2 * g)) - 1) / 3; }
__host__ __device__ inline int64_t level_cells(int g) { return (int64_t)4 << (2 * g); }

// Blocks are dealt round-robin over the 8 XCDs.  This bijection of a grid of
// nb = 8 q + r blocks hands XCD x the contiguous logical range starting at
// x q + min(x, r), so that blocks whose work shares data (neighbouring strips
// of a stencil, the sample tiles of one basis panel) read it through the
// same L2.
__device__ __forceinline__ int64_t xcd_contiguous(int64_t bid, int64_t nb)
{
    const int64_t q = nb / 8, r = nb % 8, x = bid % 8;
    return x * q + (x < r ? x : r) + bid / 8;
}

// Tile (mt, nt) of work index L in an nbm x nbn tiling of a product whose
// row tiles share the right operand's column panels: groups of `per` row
// tiles (the last one smaller), each group taking every column tile in turn
// with its row tiles innermost.  With L from xcd_contiguous, an XCD cycles
// through one group's row panels (which then stay in its L2) while the XCDs
// of other groups read the same column panel at about the same time.
__device__ __forceinline__ void grouped_tile(int64_t L, int64_t nbm, int64_t nbn, int64_t per,
                                             int64_t &mt, int64_t &nt)
{
    int64_t g = L / (per * nbn);
    const int64_t glast = (nbm - 1) / per;
    g = g < glast ? g : glast;
    const int64_t rem = L - g * per * nbn;
    const int64_t rest = nbm - g * per;
    const int64_t size = per < rest ? per : rest;
    mt = g * per + rem % size;
    nt = rem / size;
}

// Row tiles per group of grouped_tile.  When the whole right operand fits in
// the 256 MB last-level cache, one row tile per group: an XCD keeps its row
// panel in L2 and re-reads column panels from that cache (measured faster on
// 16384 samples x 87380 cells, s = 100).  Otherwise all row tiles, halved
// while their panels exceed an XCD's 4 MB L2 (two groups of the mixed
// digits at 1024 samples, s = 400, measured faster than one group or than
// uneven ones).
inline int64_t grouped_tile_per(int64_t nbm, int64_t panel_bytes, int64_t operand_bytes)
{
    if (operand_bytes <= ((int64_t)128 << 20)) return 1;
    int64_t per = nbm;
    while (per % 2 == 0 && per * panel_bytes > ((int64_t)4 << 20)) per /= 2;
    return per;
}

// Bilinear prolongation of a cell-centred coarse correction (Section 4): the
// fine cell gets (9 c + 3 x + 3 y + d) / 16 from its coarse parent c, the two
// coarse neighbours x, y on its side and the diagonal one d.  The rounding
// order is fixed by explicit fma, so every kernel that prolongates (LDS,
// tile and row-streaming passes) produces the same bits and a sample's result
// does not depend on which of them its batch size selects.
template <typename T>
__device__ __forceinline__ T prolong_9331(T c, T x, T y, T d)
{
    return (fma(T(3), y, fma(T(3), x, T(9) * c)) + d) * T(0.0625);
}

// Views of one chunk's multigrid hierarchy in the workspace pools.  Level g
// holds Bc samples back to back: sample b, cell p at base_g + b*n_g^2 + p.
struct Hier {
    int G = 0;            // finest multigrid level of the chunk
    int64_t Bc = 0;       // samples in the chunk
    double *a[kMaxMgLevels] = {};
    double *u[kMaxMgLevels] = {};
    double *f[kMaxMgLevels] = {};
};

// ---- kernel launchers (kernels.hip) ----
void launch_points(hipStream_t st, const uint32_t *z, const uint64_t *shifts, int s, int R,
                   int level, int shift_begin, int64_t n_begin, int64_t npts, int64_t b0,
                   int64_t Bc, uint64_t *x_out, double *y_out);
void launch_build_basis(hipStream_t st, const double *psi, const int64_t *psi_off,
                        const int32_t *mi, const int32_t *mj, const double *coef, int s,
                        int G, double *basis, int64_t ld);
// z = Y basis (first M columns) in FP64 on the matrix cores; mode 0 writes z
// to out[b*M + m]; mode 1 writes exp(z) into the level-major FP64 chunk pool
// `out` (Bc samples).
void launch_field_gemm(hipStream_t st, const double *Y, int s, const double *basis, int64_t ld,
                       int64_t M, int64_t Bc, void *out, int mode);
// a = exp(z) into the level-major pool; to_float: as float, with a double copy
// in pool64 when that is not null
void launch_exp_to_levels(hipStream_t st, const double *z, int64_t M, int64_t Bc, void *pool,
                          bool to_float, double *pool64);

// Mixed-precision field on the matrix cores: operands as kDigits bf16 digit
// arrays [rows_pad][sp] (bf16 bit patterns as uint16_t, zero padded) with a
// power-of-two scale exponent per row; exact FP32 group sums folded in FP64.
// mode 0 writes z (double) to out[b*M + m]; mode 2 writes exp(z) as float into
// the level-major pool out and as double into out64.
constexpr int kDigits = 5;
int64_t mixed_pad_rows(int64_t rows);
int64_t mixed_pad_cols(int64_t cols);
int mixed_pad_k(int s);
// rows with unit mode stride: element (r, k) at X[r*rs + k], one wavefront per row
void launch_digits_rows(hipStream_t st, const double *X, int64_t rows, int cols, int64_t rs,
                        int64_t rows_pad, int sp, uint16_t *const D[kDigits], int32_t *E);
// rows at unit stride, modes at stride ks: element (r, k) at X[r + k*ks]
void launch_digits_cols(hipStream_t st, const double *X, int64_t rows, int cols, int64_t ks,
                        int64_t rows_pad, int sp, uint16_t *const D[kDigits], int32_t *E);
void launch_field_digits(hipStream_t st, uint16_t *const Y[kDigits], const int32_t *EY,
                         uint16_t *const Bs[kDigits], const int32_t *EB, int sp, int64_t M, int64_t Bc,
                         void *out, double *out64, int mode);

void launch_coarse_solve(hipStream_t st, const double *a, const double *f, double *u, int64_t Bc,
                         const int32_t *active);
void launch_rbgs(hipStream_t st, const double *a, const double *f, double *u, int n, int64_t Bc,
                 int colour, const int32_t *active);
void launch_resid_restrict(hipStream_t st, const double *a, const double *f, const double *u,
                           int n, int64_t Bc, double *fc, double *uc, const int32_t *active);
void launch_prolong(hipStream_t st, const double *ec, double *u, int n, int64_t Bc, int add,
                    const int32_t *active);
// QoI of level l for Bc samples; grids of 128^2 cells or more need `part`,
// qoi_partials(cells of all samples) doubles of scratch
void launch_qoi(hipStream_t st, const double *u, int n, int64_t Bc, double *qoi, int nlev,
                int l, uint32_t mask, double *part);
int64_t qoi_partials(int64_t pool_cells);
void launch_fill(hipStream_t st, double *p, int64_t count, double v);
void launch_fill_f32(hipStream_t st, float *p, int64_t count, float v);
void launch_fill_i32(hipStream_t st, int32_t *p, int64_t count, int32_t v);
void launch_sums(hipStream_t st, const double *qoi, int nlev, int nq, int64_t b0, int64_t Bc,
                 int64_t npts, int nshift, double *state);
void launch_sums_final(hipStream_t st, const double *state, int64_t count, double *out);
// level-difference sums of nseg segments (first sample, count) of qoi
// [B][nlev][nq] into out [nseg][nq][nlev][2]; seg is a device array
void launch_seg_sums(hipStream_t st, const double *qoi, int nlev, int nq, const int64_t *seg,
                     int64_t nseg, double *out);

// ---- fused kernels (kernels_fused.hip), T = double or float ----
bool fused_supported(int mu1, int mu2);
// pass kinds of the tile grids (the MLMC_PASS_* values)
constexpr int kTile32 = MLMC_PASS_TILE32, kTile16 = MLMC_PASS_TILE16, kStream = MLMC_PASS_STREAM;
// pre pass on level n with tile shape kTile32 or kTile16: init 0 read u_in, 1
// zero guess, 2 u = P uc; writes u_out (never u_in: tiles read their
// neighbours' cells) and fc
template <typename T>
void launch_pre_tile(hipStream_t st, int shape, int mu1, const T *a, const T *f, const T *u_in,
                     T *u_out, const T *uc, int n, int64_t Bc, int init, T *fc,
                     const int32_t *active);
// post pass on level n: u = u_in + P ec, then mu2 sweeps, into u_out (!= u_in)
template <typename T>
void launch_post_tile(hipStream_t st, int shape, int mu2, const T *a, const T *f, const T *u_in,
                      T *u_out, const T *ec, int n, int64_t Bc, const int32_t *active);
// LDS-resident hierarchy (up to 32^2; 16^2 in the fixed-cycle schedule), one
// workgroup per sample:
// FP64 FMG stages 0..G with fixed cycles and QoI, final u of level G to the pool
void launch_lds_fmg_fixed(hipStream_t st, const double *a_pool, double *u_pool, int64_t Bc, int G,
                          int mu0, int mu1, int mu2, int g0, double *qoi, int nlev, uint32_t mask);
// one V-cycle at level G, zero guess, f from the f pool -> correction in the u pool
template <typename T>
void launch_lds_vcycle(hipStream_t st, const T *a_pool, const T *f_pool, T *u_pool, int64_t Bc,
                       int G, int mu1, int mu2, const int32_t *active);
// FMG stages 0..G, each stage g >= 1 solved to rtol by flexible CG in FP64
// with one T V-cycle as the preconditioner; x of level G to u64_pool;
// per-sample statistics
// (a64_pool: FP64 coefficients of the CG operator, the a pool itself when T = double)
template <typename T>
void launch_lds_fmg_refine(hipStream_t st, const T *a_pool, const double *a64_pool,
                           double *u64_pool, int64_t Bc, int G, int mu1, int mu2, double rtol,
                           int max_iters, int g0, double *qoi, int nlev, uint32_t mask,
                           int32_t *st_iters, double *st_rho, int32_t *st_bad);
// flexible CG of one stage on a large grid (Bc samples of n x n, n >= 64).
// Iterate x in FP64 in two buffers (x0 = the stage solution pool), residual
// only as T(r) in two buffers (r_k in f for even k, fo for odd k: the
// preconditioner of step k takes the other one), the search direction in T
// (two buffers); FP64 coefficients for the residual, T coefficients for
// (p, A p).  Partial-sum scratch: fcg_partials doubles; fs: 4 doubles per
// sample.
int64_t fcg_partials(int n, int64_t Bc);
template <typename T>
struct FcgBufs {
    const T *a;             // V-cycle coefficients (level n)
    const double *a64;      // FP64 coefficients (level n)
    const T *z;             // preconditioner output
    T *f, *fo;              // r_k for even and for odd k
    T *p0, *p1;             // search directions
    double *x0, *x1;        // iterates
    double *part, *fs, *rho;
    double *hist;           // stagnation state, 4 doubles per sample
    int32_t *active, *iters;
};
// r_0 = 1 - A x0 (every sample), f = T(r_0), partial ||r_0||^2
template <typename T>
void launch_fcg_resid(hipStream_t st, const double *a, const double *x, int n, int64_t Bc, T *f,
                      double *part);
// rho = ||r||/||1||; active = rho > rtol && iters < max_iters and rho came
// 10% below its best value within the last four steps; iters counts steps
void launch_fcg_fin_rho(hipStream_t st, const double *part, int n, int64_t Bc, double *rho,
                        double *hist, int32_t *active, int32_t *iters, double rtol, int max_iters,
                        int first);
// step k after z = B r_{k-1}: beta, p, alpha, x, r_k, convergence flags
template <typename T>
void launch_fcg_step(hipStream_t st, const FcgBufs<T> &v, int n, int64_t Bc, double rtol,
                     int max_iters);
// after the last step: x1 -> x0 for samples whose step count is odd
void launch_fcg_copyback(hipStream_t st, double *x0, const double *x1, int n, int64_t Bc,
                         const int32_t *iters);
void launch_refine_stats(hipStream_t st, const int32_t *iters, const double *rho, int64_t Bc,
                         double rtol, int32_t *st_iters, double *st_rho, int32_t *st_bad);

// ---- Matern field by the Nystrom method (matern.hip) ----
// KL basis sigma sqrt(theta_m) psi_m of the isotropic Matern covariance on
// the cell centres of MG levels 0..G: basis [s][ld] (device), theta [s]
// (host, descending).  Q x Q midpoint quadrature nodes.  Null stream,
// synchronous.  Returns "" on success, else the error.
std::string matern_basis(int Q, double nu, double lam, double sigma, int s, int G, double *basis,
                         int64_t ld, std::vector<double> &theta);

// ---- row-streaming passes (kernels_stream.hip), SPB samples per workgroup;
// T = double or float (instantiated for both) ----
bool stream_supported(int n);
template <typename T>
void launch_pre_stream(hipStream_t st, int mu1, const T *a, const T *f, const T *u_in, T *u_out,
                       const T *uc, int n, int64_t Bc, int init, T *fc, const int32_t *active);
template <typename T>
void launch_post_stream(hipStream_t st, int mu2, const T *a, const T *f, const T *u_in, T *u_out,
                        const T *ec, int n, int64_t Bc, const int32_t *active);

}  // namespace mlmc
