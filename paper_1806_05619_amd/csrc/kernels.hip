// Device kernels of the MG-MLQMC sample path for gfx950.
//
// Sampler (Section 3.2), KL field (Section 5, eq. truncatedKL), the multigrid
// components of the correction scheme and full multigrid (Section 4), QoI
// read-off of every FMG stage and the level-difference sums that feed the
// recycling estimator (Section 3.2, eq. Upsilon-reuse).
//
// Layout: a chunk of Bc samples stores multigrid level g as Bc contiguous
// n_g x n_g grids (cell (i,j) at i + n*j).  Every kernel bounds-checks its
// flat thread index against the element count it was launched for.
#include "internal.hpp"

namespace mlmc {
namespace {

inline unsigned blocks_for(int64_t n, int per_block = kBlock)
{
    int64_t b = (n + per_block - 1) / per_block;
    return (unsigned)(b < 1 ? 1 : b);
}

__device__ __forceinline__ double harmonic(double ap, double an)
{
    return 2.0 * ap * an / (ap + an);
}

// Neumaier/TwoSum helpers for deterministic compensated reductions.
struct Comp {
    double s, c;
};
__device__ __forceinline__ void comp_add(Comp &k, double v)
{
    double t = k.s + v;
    if (fabs(k.s) >= fabs(v))
        k.c += (k.s - t) + v;
    else
        k.c += (v - t) + k.s;
    k.s = t;
}
__device__ __forceinline__ Comp comp_merge(Comp x, Comp y)
{
    double s = x.s + y.s;
    double bb = s - x.s;
    double err = (x.s - (s - bb)) + (y.s - bb);
    return Comp{s, x.c + y.c + err};
}
// Butterfly over the 64 lanes of a wavefront (fixed order: deterministic).
__device__ __forceinline__ Comp wave_reduce(Comp k)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        Comp o{__shfl_xor(k.s, m, 64), __shfl_xor(k.c, m, 64)};
        k = comp_merge(k, o);
    }
    return k;
}

// ---------------------------------------------------------------------------
// Phi^-1(u): the device library's normcdfinv, then one Newton step on
// Phi(y) = u whose residual is formed without cancellation (u - 1/2 and 1 - u
// are exact for the u this path produces).
__device__ __forceinline__ double inverse_normal(double u)
{
    double y = normcdfinv(u);
    const double r2 = 0.70710678118654752440;    // 1/sqrt(2)
    double g;
    if (u < 0.25)
        g = 0.5 * erfc(-y * r2) - u;
    else if (u <= 0.75)
        g = 0.5 * erf(y * r2) - (u - 0.5);
    else
        g = (1.0 - u) - 0.5 * erfc(y * r2);
    double pdf = 0.39894228040143267794 * exp(-0.5 * y * y);   // 1/sqrt(2 pi)
    return y - g / pdf;
}

// Section 3.2: shifted lattice sequence point -> (0,1) -> inverse normal.
__global__ void k_points(const uint32_t *__restrict__ z, const uint64_t *__restrict__ shifts,
                         int s, int R, int level, int shift_begin, int64_t n_begin,
                         int64_t npts, int64_t b0, int64_t Bc, uint64_t *__restrict__ x_out,
                         double *__restrict__ y_out)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= Bc * s)
        return;
    int64_t bl = t / s;
    int j = (int)(t - bl * s);
    int64_t b = b0 + bl;
    int64_t rl = b / npts;
    int64_t n = n_begin + (b - rl * npts);
    int r = shift_begin + (int)rl;
    uint32_t rn = __brev((uint32_t)n);           // radical inverse in base 2
    uint32_t k = rn * z[j];                      // {rev(n) z_j / 2^32}
    uint64_t x = ((uint64_t)k << 32) + shifts[((int64_t)level * R + r) * s + j];
    if (x_out)
        x_out[t] = x;
    double u = (2.0 * (double)(x >> 12) + 1.0) * 0x1p-53;
    y_out[t] = inverse_normal(u);
}

// ---------------------------------------------------------------------------
// KL basis: basis[m][col] = coef_m psi_{i_m}(x1) psi_{j_m}(x2) at the cell
// centres of every level; psi tabulated per level: psi[psi_off[g] + k*n_g + c].
__global__ void k_build_basis(const double *__restrict__ psi, const int64_t *__restrict__ psi_off,
                              const int32_t *__restrict__ mi, const int32_t *__restrict__ mj,
                              const double *__restrict__ coef, int s, int G, int64_t M,
                              double *__restrict__ basis, int64_t ld)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= M * s)
        return;
    int m = (int)(t / M);
    int64_t col = t - (int64_t)m * M;
    int g = 0;
    while (g < G && level_offset(g + 1) <= col)
        ++g;
    int n = 2 << g;
    int64_t p = col - level_offset(g);
    int i = (int)(p % n), j = (int)(p / n);
    const double *pg = psi + psi_off[g];
    basis[(int64_t)m * ld + col] =
        coef[m] * pg[(int64_t)(mi[m] - 1) * n + i] * pg[(int64_t)(mj[m] - 1) * n + j];
}

// ---------------------------------------------------------------------------
// Section 5: the level-major position of field column m of sample b.
__device__ __forceinline__ int64_t level_major_index(int64_t m, int64_t b, int64_t Bc)
{
    int g = 0;
    while (g < kMaxMgLevels - 1 && level_offset(g + 1) <= m)
        ++g;
    int64_t lo = level_offset(g);
    return Bc * lo + b * level_cells(g) + (m - lo);
}

__global__ void k_exp_to_levels(const double *__restrict__ z, int64_t M, int64_t Bc,
                                void *__restrict__ pool, int to_float, double *__restrict__ pool64)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= M * Bc)
        return;
    int64_t b = t / M, m = t - b * M;
    const int64_t q = level_major_index(m, b, Bc);
    const double av = exp(z[t]);
    if (to_float) {
        ((float *)pool)[q] = (float)av;
        if (pool64) pool64[q] = av;
    } else {
        ((double *)pool)[q] = av;
    }
}

// ---------------------------------------------------------------------------
// Section 4: exact solve on the 2x2 coarsest grid (h^2 = 1/4), one sample per
// thread, dense 4x4 Cholesky.  Cells 0:(0,0) 1:(1,0) 2:(0,1) 3:(1,1).
__global__ void k_coarse_solve(const double *__restrict__ a, const double *__restrict__ f,
                               double *__restrict__ u, int64_t Bc,
                               const int32_t *__restrict__ active)
{
    int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= Bc)
        return;
    if (active && !active[b])
        return;
    const double *ab = a + 4 * b;
    double w01 = harmonic(ab[0], ab[1]), w02 = harmonic(ab[0], ab[2]);
    double w13 = harmonic(ab[1], ab[3]), w23 = harmonic(ab[2], ab[3]);
    double A[4][4] = {{w01 + w02 + 4.0 * ab[0], -w01, -w02, 0.0},
                      {-w01, w01 + w13 + 4.0 * ab[1], 0.0, -w13},
                      {-w02, 0.0, w02 + w23 + 4.0 * ab[2], -w23},
                      {0.0, -w13, -w23, w13 + w23 + 4.0 * ab[3]}};
    double rhs[4];
    for (int p = 0; p < 4; ++p) rhs[p] = 0.25 * (f ? f[4 * b + p] : 1.0);
    double L[4][4] = {};
    for (int p = 0; p < 4; ++p)
        for (int q = 0; q <= p; ++q) {
            double sum = A[p][q];
            for (int t = 0; t < q; ++t) sum -= L[p][t] * L[q][t];
            L[p][q] = (p == q) ? sqrt(sum) : sum / L[q][q];
        }
    double v[4];
    for (int p = 0; p < 4; ++p) {
        double sum = rhs[p];
        for (int q = 0; q < p; ++q) sum -= L[p][q] * v[q];
        v[p] = sum / L[p][p];
    }
    for (int p = 3; p >= 0; --p) {
        double sum = v[p];
        for (int q = p + 1; q < 4; ++q) sum -= L[q][p] * v[q];
        v[p] = sum / L[p][p];
    }
    for (int p = 0; p < 4; ++p) u[4 * b + p] = v[p];
}

// One colour of red-black Gauss-Seidel: u_P = (h^2 f_P + sum w u_nbr) / sum w.
// f == nullptr means f = 1.  One thread per cell of the colour.
__global__ void k_rbgs(const double *__restrict__ a, const double *__restrict__ f,
                       double *__restrict__ u, int n, int64_t Bc, int colour,
                       const int32_t *__restrict__ active)
{
    const int half = n / 2;
    const int64_t per = (int64_t)n * half;
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= Bc * per)
        return;
    int64_t b = t / per;
    if (active && !active[b])
        return;
    int rem = (int)(t - b * per);
    int j = rem / half;
    int i = 2 * (rem - j * half) + ((j + colour) & 1);
    const int64_t base = b * n * n;
    const double *ab = a + base;
    double *ub = u + base;
    const int p = i + n * j;
    const double ap = ab[p];
    const double h2 = 1.0 / ((double)n * (double)n);
    double num = h2 * (f ? f[base + p] : 1.0);
    double d = 0.0, w;
    if (i + 1 < n) { w = harmonic(ap, ab[p + 1]); d += w; num += w * ub[p + 1]; } else d += 2.0 * ap;
    if (i > 0)     { w = harmonic(ap, ab[p - 1]); d += w; num += w * ub[p - 1]; } else d += 2.0 * ap;
    if (j + 1 < n) { w = harmonic(ap, ab[p + n]); d += w; num += w * ub[p + n]; } else d += 2.0 * ap;
    if (j > 0)     { w = harmonic(ap, ab[p - n]); d += w; num += w * ub[p - n]; } else d += 2.0 * ap;
    ub[p] = num / d;
}

__device__ __forceinline__ double residual_at(const double *ab, const double *fb,
                                              const double *ub, int n, int i, int j,
                                              double inv_h2)
{
    // net flux out of the cell, face by face: w (u_P - u_N), or 2 a_P u_P at a wall
    const int p = i + n * j;
    const double ap = ab[p], up = ub[p];
    double v = 0.0;
    v += (i + 1 < n) ? harmonic(ap, ab[p + 1]) * (up - ub[p + 1]) : 2.0 * ap * up;
    v += (i > 0) ? harmonic(ap, ab[p - 1]) * (up - ub[p - 1]) : 2.0 * ap * up;
    v += (j + 1 < n) ? harmonic(ap, ab[p + n]) * (up - ub[p + n]) : 2.0 * ap * up;
    v += (j > 0) ? harmonic(ap, ab[p - n]) * (up - ub[p - n]) : 2.0 * ap * up;
    return (fb ? fb[p] : 1.0) - inv_h2 * v;
}

// r = f - A u on the fine grid, restricted by the 4-cell mean to fc; the
// coarse iterate uc is cleared (zero initial guess).  One thread per coarse cell.
__global__ void k_resid_restrict(const double *__restrict__ a, const double *__restrict__ f,
                                 const double *__restrict__ u, int n, int64_t Bc,
                                 double *__restrict__ fc, double *__restrict__ uc,
                                 const int32_t *__restrict__ active)
{
    const int nc = n / 2;
    const int64_t per = (int64_t)nc * nc;
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= Bc * per)
        return;
    int64_t b = t / per;
    if (active && !active[b])
        return;
    int pc = (int)(t - b * per);
    int J = pc / nc, I = pc - J * nc;
    const int64_t base = b * n * n;
    const double *fb = f ? f + base : nullptr;
    const double inv_h2 = (double)n * (double)n;
    double r00 = residual_at(a + base, fb, u + base, n, 2 * I, 2 * J, inv_h2);
    double r10 = residual_at(a + base, fb, u + base, n, 2 * I + 1, 2 * J, inv_h2);
    double r01 = residual_at(a + base, fb, u + base, n, 2 * I, 2 * J + 1, inv_h2);
    double r11 = residual_at(a + base, fb, u + base, n, 2 * I + 1, 2 * J + 1, inv_h2);
    fc[t] = 0.25 * (r00 + r10 + r01 + r11);
    uc[t] = 0.0;
}

__device__ __forceinline__ double coarse_odd(const double *e, int nc, int I, int J)
{
    double sg = 1.0;
    if (I < 0) { I = 0; sg = -sg; }
    if (I >= nc) { I = nc - 1; sg = -sg; }
    if (J < 0) { J = 0; sg = -sg; }
    if (J >= nc) { J = nc - 1; sg = -sg; }
    return sg * e[I + nc * J];
}

// Bilinear (9,3,3,1)/16 prolongation with odd reflection at the walls:
// u = P ec (add == 0, FMG interpolation) or u += P ec (coarse-grid
// correction) on n x n grids (n a power of two, at least 4).  One thread per
// coarse cell (I, J), i.e. per 2 x 2 block of fine
// cells, which interpolate from the 3 x 3 coarse cells around it (nine
// loads for four cells); each of the block's two rows is stored as one
// 16-byte vector, so a wavefront writes 128 consecutive cells of a row per
// store.  Index arithmetic by shifts (per-sample offsets and rows are powers
// of two).
__global__ void k_prolong(const double *__restrict__ ec, double *__restrict__ u, int n,
                          int64_t Bc, int add, const int32_t *__restrict__ active)
{
    const int lg = __builtin_ctz(n);                   // n = 2^lg
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t b = t >> (2 * lg - 2);               // n^2 / 4 blocks per sample
    if (b >= Bc)
        return;
    if (active && !active[b])
        return;
    const int q = (int)(t & (((int64_t)1 << (2 * lg - 2)) - 1));
    const int nc = n / 2;
    const int J = q >> (lg - 1), I = q & (nc - 1);
    const double *eb = ec + b * nc * nc;
    double c[3][3];                                    // c[dy + 1][dx + 1] = e(I + dx, J + dy)
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) c[dy + 1][dx + 1] = coarse_odd(eb, nc, I + dx, J + dy);
    // fine cell (2I + a, 2J + r) takes the horizontal neighbour column
    // I - 1 + 2a and the vertical neighbour row J - 1 + 2r
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int vy = 2 * r;                          // row index of the vertical neighbour in c
        const double v0 = prolong_9331(c[1][1], c[1][0], c[vy][1], c[vy][0]);
        const double v1 = prolong_9331(c[1][1], c[1][2], c[vy][1], c[vy][2]);
        double2 *dst = reinterpret_cast<double2 *>(u + (b << (2 * lg)) +
                                                   ((int64_t)(2 * J + r) << lg) + 2 * I);
        double2 o;
        if (add) {
            o = *dst;
            o.x += v0;
            o.y += v1;
        } else {
            o.x = v0;
            o.y = v1;
        }
        *dst = o;
    }
}

// QoI of one level, one wavefront per sample: mean (compensated) and centre.
__global__ __launch_bounds__(256) void k_qoi(const double *__restrict__ u, int n, int64_t Bc,
                                             double *__restrict__ qoi, int nlev, int l,
                                             uint32_t mask)
{
    const int lane = threadIdx.x & 63;
    const int64_t b = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
    if (b >= Bc)
        return;
    const int64_t cells = (int64_t)n * n;
    const double *ub = u + b * cells;
    Comp k{0.0, 0.0};
    for (int64_t p = lane; p < cells; p += 64)
        comp_add(k, ub[p]);
    k = wave_reduce(k);
    if (lane == 0) {
        const int nq = (mask & 1u ? 1 : 0) + (mask & 2u ? 1 : 0);
        double *qb = qoi + (b * nlev + l) * nq;
        int q = 0;
        if (mask & 1u)
            qb[q++] = (k.s + k.c) / (double)cells;
        if (mask & 2u) {
            int c = n / 2;
            qb[q] = 0.25 * (ub[(c - 1) + n * (c - 1)] + ub[c + n * (c - 1)] +
                            ub[(c - 1) + n * c] + ub[c + n * c]);
        }
    }
}

// Grids of QCH cells or more: the mean is summed in chunks of QCH cells, one
// block per chunk (a single wavefront per sample leaves most of the chip idle
// when a batch of a fine level has few samples), then the chunk sums of a
// sample are folded in chunk order.  The order depends on n only, so a
// sample's QoI does not depend on its batch.
constexpr int QCH = 16384;

__global__ __launch_bounds__(256) void k_qoi_part(const double *__restrict__ u, int n, int64_t Bc,
                                                  double *__restrict__ part)
{
    const int64_t cells = (int64_t)n * n;
    const int P = (int)(cells / QCH);
    const int64_t blk = blockIdx.x;
    const int64_t b = blk / P;
    if (b >= Bc)
        return;
    const double *src = u + b * cells + (blk - b * P) * QCH;
    Comp k{0.0, 0.0};
    for (int q = threadIdx.x; q < QCH; q += 256)
        comp_add(k, src[q]);
    k = wave_reduce(k);
    __shared__ double ws[4][2];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        ws[w][0] = k.s;
        ws[w][1] = k.c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        Comp t{0.0, 0.0};
        for (int i = 0; i < 4; ++i) {
            comp_add(t, ws[i][0]);
            comp_add(t, ws[i][1]);
        }
        part[2 * blk] = t.s;
        part[2 * blk + 1] = t.c;
    }
}

__global__ __launch_bounds__(256) void k_qoi_fin(const double *__restrict__ u,
                                                 const double *__restrict__ part, int n,
                                                 int64_t Bc, double *__restrict__ qoi, int nlev,
                                                 int l, uint32_t mask)
{
    const int lane = threadIdx.x & 63;
    const int64_t b = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
    if (b >= Bc)
        return;
    const int64_t cells = (int64_t)n * n;
    const int P = (int)(cells / QCH);
    Comp k{0.0, 0.0};
    for (int p = lane; p < P; p += 64) {
        comp_add(k, part[2 * (b * P + p)]);
        comp_add(k, part[2 * (b * P + p) + 1]);
    }
    k = wave_reduce(k);
    if (lane == 0) {
        const double *ub = u + b * cells;
        const int nq = (mask & 1u ? 1 : 0) + (mask & 2u ? 1 : 0);
        double *qb = qoi + (b * nlev + l) * nq;
        int q = 0;
        if (mask & 1u)
            qb[q++] = (k.s + k.c) / (double)cells;
        if (mask & 2u) {
            int c = n / 2;
            qb[q] = 0.25 * (ub[(c - 1) + n * (c - 1)] + ub[c + n * (c - 1)] +
                            ub[(c - 1) + n * c] + ub[c + n * c]);
        }
    }
}

__global__ void k_fill(double *p, int64_t count, double v)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count)
        p[t] = v;
}

__global__ void k_fill_f32(float *p, int64_t count, float v)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count)
        p[t] = v;
}

__global__ void k_fill_i32(int32_t *p, int64_t count, int32_t v)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count)
        p[t] = v;
}

// Level-difference sums for the estimator: one wavefront per (shift, q, l)
// accumulates sum dF and sum dF^2 over the chunk's samples of that shift into
// the compensated state [tuple][4] = (s1, c1, s2, c2).
__global__ __launch_bounds__(256) void k_sums(const double *__restrict__ qoi, int nlev, int nq,
                                              int64_t b0, int64_t Bc, int64_t npts, int nshift,
                                              double *__restrict__ state)
{
    const int lane = threadIdx.x & 63;
    const int64_t tuple = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
    const int64_t ntup = (int64_t)nshift * nq * nlev;
    if (tuple >= ntup)
        return;
    const int l = (int)(tuple % nlev);
    const int q = (int)((tuple / nlev) % nq);
    const int rl = (int)(tuple / ((int64_t)nlev * nq));
    int64_t lo = (int64_t)rl * npts, hi = lo + npts;   // global sample range of this shift
    if (lo < b0) lo = b0;
    if (hi > b0 + Bc) hi = b0 + Bc;
    Comp k1{0.0, 0.0}, k2{0.0, 0.0};
    for (int64_t b = lo + lane; b < hi; b += 64) {
        const double *qb = qoi + (b - b0) * nlev * nq;
        double d = qb[l * nq + q] - (l > 0 ? qb[(l - 1) * nq + q] : 0.0);
        comp_add(k1, d);
        comp_add(k2, d * d);
    }
    k1 = wave_reduce(k1);
    k2 = wave_reduce(k2);
    if (lane == 0) {
        double *st = state + tuple * 4;
        Comp a1 = comp_merge(Comp{st[0], st[1]}, k1);
        Comp a2 = comp_merge(Comp{st[2], st[3]}, k2);
        st[0] = a1.s;
        st[1] = a1.c;
        st[2] = a2.s;
        st[3] = a2.c;
    }
}

// Level-difference sums of segments of a QoI table (Section 3.2, eq.
// Upsilon-reuse): segment t covers samples seg[2t] .. seg[2t] + seg[2t+1] - 1
// of qoi [B][nlev][nq]; out [nseg][nq][nlev][2] receives the compensated sums
// of F_l - F_{l-1} and of its square.  One wavefront per (segment, q, l); a
// lane sums the samples lane, lane + 64, ... of its segment, as k_sums does
// for a shift of one chunk, so a segment's sums do not depend on what else
// the table holds.
__global__ __launch_bounds__(256) void k_seg_sums(const double *__restrict__ qoi, int nlev, int nq,
                                                  const int64_t *__restrict__ seg, int64_t nseg,
                                                  double *__restrict__ out)
{
    const int lane = threadIdx.x & 63;
    const int64_t tuple = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
    if (tuple >= nseg * nq * nlev)
        return;
    const int l = (int)(tuple % nlev);
    const int q = (int)((tuple / nlev) % nq);
    const int64_t t = tuple / ((int64_t)nlev * nq);
    const int64_t lo = seg[2 * t], hi = lo + seg[2 * t + 1];
    Comp k1{0.0, 0.0}, k2{0.0, 0.0};
    for (int64_t b = lo + lane; b < hi; b += 64) {
        const double *qb = qoi + b * nlev * nq;
        double d = qb[l * nq + q] - (l > 0 ? qb[(l - 1) * nq + q] : 0.0);
        comp_add(k1, d);
        comp_add(k2, d * d);
    }
    k1 = wave_reduce(k1);
    k2 = wave_reduce(k2);
    if (lane == 0) {
        const Comp a1 = comp_merge(Comp{0.0, 0.0}, k1);
        const Comp a2 = comp_merge(Comp{0.0, 0.0}, k2);
        out[2 * tuple] = a1.s + a1.c;
        out[2 * tuple + 1] = a2.s + a2.c;
    }
}

__global__ void k_sums_final(const double *__restrict__ state, int64_t count,
                             double *__restrict__ out)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count)
        return;
    out[2 * t] = state[4 * t] + state[4 * t + 1];
    out[2 * t + 1] = state[4 * t + 2] + state[4 * t + 3];
}


}  // namespace

// ---------------------------------------------------------------------------
// launchers
void launch_points(hipStream_t st, const uint32_t *z, const uint64_t *shifts, int s, int R,
                   int level, int shift_begin, int64_t n_begin, int64_t npts, int64_t b0,
                   int64_t Bc, uint64_t *x_out, double *y_out)
{
    hipLaunchKernelGGL(k_points, dim3(blocks_for(Bc * s)), dim3(kBlock), 0, st, z, shifts, s, R,
                       level, shift_begin, n_begin, npts, b0, Bc, x_out, y_out);
}

void launch_build_basis(hipStream_t st, const double *psi, const int64_t *psi_off,
                        const int32_t *mi, const int32_t *mj, const double *coef, int s, int G,
                        double *basis, int64_t ld)
{
    int64_t M = level_offset(G + 1);
    hipLaunchKernelGGL(k_build_basis, dim3(blocks_for(M * s)), dim3(kBlock), 0, st, psi, psi_off,
                       mi, mj, coef, s, G, M, basis, ld);
}


void launch_exp_to_levels(hipStream_t st, const double *z, int64_t M, int64_t Bc, void *pool,
                          bool to_float, double *pool64)
{
    hipLaunchKernelGGL(k_exp_to_levels, dim3(blocks_for(M * Bc)), dim3(kBlock), 0, st, z, M, Bc,
                       pool, (int)to_float, pool64);
}

void launch_coarse_solve(hipStream_t st, const double *a, const double *f, double *u, int64_t Bc,
                         const int32_t *active)
{
    hipLaunchKernelGGL(k_coarse_solve, dim3(blocks_for(Bc)), dim3(kBlock), 0, st, a, f, u, Bc,
                       active);
}

void launch_rbgs(hipStream_t st, const double *a, const double *f, double *u, int n, int64_t Bc,
                 int colour, const int32_t *active)
{
    int64_t cnt = Bc * (int64_t)n * (n / 2);
    hipLaunchKernelGGL(k_rbgs, dim3(blocks_for(cnt)), dim3(kBlock), 0, st, a, f, u, n, Bc, colour,
                       active);
}

void launch_resid_restrict(hipStream_t st, const double *a, const double *f, const double *u,
                           int n, int64_t Bc, double *fc, double *uc, const int32_t *active)
{
    int64_t cnt = Bc * (int64_t)(n / 2) * (n / 2);
    hipLaunchKernelGGL(k_resid_restrict, dim3(blocks_for(cnt)), dim3(kBlock), 0, st, a, f, u, n,
                       Bc, fc, uc, active);
}

void launch_prolong(hipStream_t st, const double *ec, double *u, int n, int64_t Bc, int add,
                    const int32_t *active)
{
    int64_t cnt = Bc * (int64_t)n * n / 4;         // 2 x 2 blocks of fine cells
    hipLaunchKernelGGL(k_prolong, dim3(blocks_for(cnt)), dim3(kBlock), 0, st, ec, u, n, Bc, add,
                       active);
}

void launch_qoi(hipStream_t st, const double *u, int n, int64_t Bc, double *qoi, int nlev, int l,
                uint32_t mask, double *part)
{
    if ((int64_t)n * n >= QCH) {
        const int64_t P = (int64_t)n * n / QCH;
        hipLaunchKernelGGL(k_qoi_part, dim3((unsigned)(Bc * P)), dim3(256), 0, st, u, n, Bc, part);
        hipLaunchKernelGGL(k_qoi_fin, dim3(blocks_for(Bc, kBlock / 64)), dim3(kBlock), 0, st, u,
                           part, n, Bc, qoi, nlev, l, mask);
        return;
    }
    hipLaunchKernelGGL(k_qoi, dim3(blocks_for(Bc, kBlock / 64)), dim3(kBlock), 0, st, u, n, Bc,
                       qoi, nlev, l, mask);
}

int64_t qoi_partials(int64_t pool_cells) { return 2 * (pool_cells / QCH) + 2; }

void launch_fill(hipStream_t st, double *p, int64_t count, double v)
{
    if (count <= 0)
        return;
    hipLaunchKernelGGL(k_fill, dim3(blocks_for(count)), dim3(kBlock), 0, st, p, count, v);
}

void launch_fill_f32(hipStream_t st, float *p, int64_t count, float v)
{
    if (count <= 0)
        return;
    hipLaunchKernelGGL(k_fill_f32, dim3(blocks_for(count)), dim3(kBlock), 0, st, p, count, v);
}

void launch_fill_i32(hipStream_t st, int32_t *p, int64_t count, int32_t v)
{
    if (count <= 0)
        return;
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(count)), dim3(kBlock), 0, st, p, count, v);
}

void launch_sums(hipStream_t st, const double *qoi, int nlev, int nq, int64_t b0, int64_t Bc,
                 int64_t npts, int nshift, double *state)
{
    int64_t ntup = (int64_t)nshift * nq * nlev;
    hipLaunchKernelGGL(k_sums, dim3(blocks_for(ntup, kBlock / 64)), dim3(kBlock), 0, st, qoi, nlev,
                       nq, b0, Bc, npts, nshift, state);
}

void launch_seg_sums(hipStream_t st, const double *qoi, int nlev, int nq, const int64_t *seg,
                     int64_t nseg, double *out)
{
    const int64_t ntup = nseg * nq * nlev;
    if (ntup <= 0)
        return;
    hipLaunchKernelGGL(k_seg_sums, dim3(blocks_for(ntup, kBlock / 64)), dim3(kBlock), 0, st, qoi,
                       nlev, nq, seg, nseg, out);
}

void launch_sums_final(hipStream_t st, const double *state, int64_t count, double *out)
{
    hipLaunchKernelGGL(k_sums_final, dim3(blocks_for(count)), dim3(kBlock), 0, st, state, count,
                       out);
}


}  // namespace mlmc
