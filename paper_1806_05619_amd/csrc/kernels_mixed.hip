// KL field of the mixed-precision path on the gfx950 matrix cores (Section 5,
// eq. truncatedKL): z = Y basis as a sum of exact bf16 products.
//
// Each row of Y (one sample, over the KL modes) and each field column of the
// basis (one cell centre, over the modes) gets a power-of-two scale 2^E with
// 2^E > max |x|; x 2^(7-E) is then written as five balanced base-256 digits,
// x 2^(7-E) = d1 + d2 2^-8 + d3 2^-16 + d4 2^-24 + d5 2^-32 + rest, |d| <= 128,
// |rest| <= 2^-33.  Every digit is an integer of at most 8 bits, so it is
// exact in bf16, every digit product is an integer of magnitude at most 2^14,
// and a group of up to five products of equal weight summed over 192 modes
// stays below 2^24: the FP32 accumulation of v_mfma_f32_16x16x32_bf16 is exact
// whatever its internal rounding.  The products of weight 2^-8w, w = 0..4, are
// grouped (G_w = sum over i + j = w of d_(i+1) e_(j+1); fifteen MFMAs per
// tile), and every 192 modes the groups are folded into FP64 accumulators
// (rounding at 2^-53 of the group scale).  The result is z times 2^(14 - E_r
// - E_c) up to the dropped products (weight 2^-40 and below) and the digit
// remainders: at most 2 s 2^(E_y + E_b - 38) per cell for s modes, with 2^E_y
// and 2^E_b the row and column scales.  This is the Ozaki splitting (Ozaki,
// Ogita, Oishi, Rump, Numer. Algorithms 59, 2012) with fixed-point digits
// sized for bf16 matrix cores.
//
// Operands are stored K-contiguous ([rows_pad][sp], sp = s rounded up to 32,
// zero padded) so that each lane loads its 8 consecutive k values as one
// 16-byte vector.  MFMA lane layout (16x16x32): A row l%16 and B column l%16
// take k = 8*(l/16) .. +7; lane l holds C rows 4*(l/16) .. +3 of column l%16.
#include "internal.hpp"

namespace mlmc {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int WM = 32, WN = 32;        // tile of one wave: 2 x 2 MFMA tiles
constexpr int BM = 64, BN = 64;        // tile of a 4-wave block (2 x 2 waves)
constexpr int KFOLD = 6;               // K steps of 32 between folds into FP64
constexpr int ND = kDigits;            // digits per operand
constexpr int NP = ND * (ND + 1) / 2;  // digit products of weight 2^-8w, w < ND

// the bf16 bit pattern of an integer d with |d| <= 256 (exact)
__device__ __forceinline__ uint16_t bf16_of_int(double d)
{
    return (uint16_t)(__float_as_uint((float)d) >> 16);
}

// digits of x 2^(7-E), E the row scale
__device__ __forceinline__ void digits(double x, int E, uint16_t *d)
{
    double t = ldexp(x, 7 - E);
#pragma unroll
    for (int q = 0; q < ND; ++q) {
        const double v = rint(t);
        d[q] = bf16_of_int(v);
        t = (t - v) * 256.0;             // exact: |t - v| <= 1/2 has fewer bits than t
    }
}

// scale exponent E with 2^(E-1) <= m < 2^E (m = max |x| > 0), 0 for m = 0
__device__ __forceinline__ int scale_exp(double m)
{
    int e = 0;
    if (m > 0.0) frexp(m, &e);
    return e;
}

struct DigitPtrs {
    uint16_t *d[ND];
};

// one row per wavefront, modes along the lanes (rows with unit mode stride):
// scale exponent and ND digit arrays [rows_pad][sp]; padding is zero
__global__ __launch_bounds__(256) void k_digits_wave(const double *__restrict__ X, int64_t rows,
                                                     int cols, int64_t rs, int64_t rows_pad, int sp,
                                                     DigitPtrs D, int32_t *__restrict__ E)
{
    const int lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= rows_pad) return;
    const double *xr = X + r * rs;
    const bool in = r < rows;
    double m = 0.0;
    for (int k = lane; k < cols && in; k += 64) m = fmax(m, fabs(xr[k]));
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    const int e = scale_exp(m);
    for (int k = lane; k < sp; k += 64) {
        uint16_t d[ND] = {};
        if (in && k < cols) digits(xr[k], e, d);
        const int64_t o = r * sp + k;
#pragma unroll
        for (int q = 0; q < ND; ++q) D.d[q][o] = d[q];
    }
    if (lane == 0) E[r] = e;
}

// one row per thread (rows at unit stride, modes at stride ks: the basis
// [s][ld] read as rows m = field columns)
__global__ __launch_bounds__(256) void k_digits_thread(const double *__restrict__ X, int64_t rows,
                                                       int cols, int64_t ks, int64_t rows_pad,
                                                       int sp, DigitPtrs D, int32_t *__restrict__ E)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows_pad) return;
    const bool in = r < rows;
    double m = 0.0;
    for (int k = 0; k < cols && in; ++k) m = fmax(m, fabs(X[r + (int64_t)k * ks]));
    const int e = scale_exp(m);
    for (int k = 0; k < sp; ++k) {
        uint16_t d[ND] = {};
        if (in && k < cols) digits(X[r + (int64_t)k * ks], e, d);
        const int64_t o = r * sp + k;
#pragma unroll
        for (int q = 0; q < ND; ++q) D.d[q][o] = d[q];
    }
    E[r] = e;
}

// field column m (cells of all levels, coarsest first) in the level-major
// pool of Bc samples: sample b's value sits at base + b * stride
__device__ __forceinline__ void level_major_column(int64_t m, int64_t Bc, int64_t &base,
                                                   int64_t &stride)
{
    int g = 0;
    while (g < kMaxMgLevels - 1 && level_offset(g + 1) <= m) ++g;
    const int64_t lo = level_offset(g);
    base = Bc * lo + (m - lo);
    stride = level_cells(g);
}

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// LDS place of 16-byte chunk c (modes 8c .. 8c+7) of panel row r: slot
// 4 r + (c ^ swz(r)).  The 16 rows that the lanes of a quarter-wavefront read
// at one chunk fall into 16 distinct 4-bank groups of a 64-bank LDS, and the
// rows of each eighth of a wavefront into 8 distinct groups of a 32-bank one.
__device__ __forceinline__ int swz(int r) { return ((r >> 1) ^ (r >> 3)) & 3; }

// out mode 0: z (double) at out[b*M + m]; mode 2: exp(z) as float into the
// level-major pool `out` and as double into `out64`.
// Two workgroups per CU (registers <= 256, LDS 80 KiB each): one's loads and
// epilogue overlap the other's matrix-core work.
__global__ __launch_bounds__(256, 2) void k_field_digits(DigitPtrs Yp, const int32_t *__restrict__ EY,
                                                         DigitPtrs Bp, const int32_t *__restrict__ EB,
                                                         int sp, int64_t M, int64_t Bc, int64_t nbm,
                                                         int64_t per, void *__restrict__ out,
                                                         double *__restrict__ out64, int mode)
{
    // The block's 64 x 32 digit panels of Y and of the basis go from global
    // memory straight into LDS (global_load_lds, 16 bytes a lane), double
    // buffered: every chunk is fetched once per block, and the panels of the
    // next 32 modes are in flight while the matrix cores work on the current
    // ones.  A load instruction of a wavefront fills 64 consecutive slots
    // (16 rows of one digit of one operand); lane l takes slot l, i.e. row
    // l / 4 of the group and the chunk that the swizzle places there.
    __shared__ __attribute__((aligned(16))) uint16_t As[2][ND][BM * 32];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[2][ND][BN * 32];
    const int t = threadIdx.x, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    // groups of `per` sample tiles over every basis panel (grouped_tile), so
    // that the digits of Y an XCD cycles through stay in its L2
    int64_t mt, nt;
    grouped_tile(xcd_contiguous(blockIdx.x, gridDim.x), nbm, gridDim.x / nbm, per, mt, nt);
    const int64_t brow0 = mt * BM, bcol0 = nt * BN;
    const int64_t row0 = brow0 + (wave >> 1) * WM;    // sample rows of this wave
    const int64_t col0 = bcol0 + (wave & 1) * WN;     // field columns of this wave
    const int wr = (wave >> 1) * WM, wc = (wave & 1) * WN;
    const int lr = lane & 15, q4 = lane >> 4;
    double acc[2][2][4];
    f32x4 G[ND][2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[i][j][e] = 0.0;
#pragma unroll
            for (int g = 0; g < ND; ++g) G[g][i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
    // wave w loads row group w (rows 16 w .. 16 w + 15) of every digit of
    // both operands: 2 ND instructions per K step (rows and columns are
    // padded, all in range)
    const int ldr = 16 * wave + (lane >> 2);
    const int ldc = 8 * ((lane & 3) ^ swz(ldr));
    const uint16_t *ysrc[ND], *bsrc[ND];
#pragma unroll
    for (int q = 0; q < ND; ++q) {
        ysrc[q] = Yp.d[q] + (brow0 + ldr) * sp + ldc;
        bsrc[q] = Bp.d[q] + (bcol0 + ldr) * sp + ldc;
    }
    auto issue = [&](int k0, int buf) {
#pragma unroll
        for (int q = 0; q < ND; ++q) {
            __builtin_amdgcn_global_load_lds(ysrc[q] + k0,
                                             (__attribute__((address_space(3))) void *)&As[buf][q][512 * wave],
                                             16, 0, 0);
            __builtin_amdgcn_global_load_lds(bsrc[q] + k0,
                                             (__attribute__((address_space(3))) void *)&Bs[buf][q][512 * wave],
                                             16, 0, 0);
        }
    };
    // LDS element offsets of the operand chunks this lane reads (row, chunk q4)
    int aoff[2], boff[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int ra = wr + 16 * i + lr, rb = wc + 16 * i + lr;
        aoff[i] = 8 * (4 * ra + (q4 ^ swz(ra)));
        boff[i] = 8 * (4 * rb + (q4 ^ swz(rb)));
    }
    // the digit products (digit of Y, digit of the basis, weight group), in
    // increasing weight
    constexpr int PA[NP] = {0, 0, 1, 0, 2, 1, 0, 3, 1, 2, 0, 4, 1, 3, 2};
    constexpr int PB[NP] = {0, 1, 0, 2, 0, 1, 3, 0, 2, 1, 4, 0, 3, 1, 2};
    constexpr int PG[NP] = {0, 1, 1, 2, 2, 2, 3, 3, 3, 3, 4, 4, 4, 4, 4};
    static_assert(ND == 5, "product table written for five digits");
    const int nk = sp / 32;
    issue(0, 0);
    // scale exponents and level-major addresses of the epilogue, fetched
    // while the first panels load (the exponent arrays are padded like the
    // digit rows, so every index is in range)
    int ey[2][4], eb[2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int e = 0; e < 4; ++e) ey[i][e] = EY[row0 + 16 * i + 4 * q4 + e];
#pragma unroll
    for (int j = 0; j < 2; ++j) eb[j] = EB[col0 + 16 * j + lr];
    // the epilogue writes whole rows of the block: lane l takes column l
    const int64_t mcol = bcol0 + lane;
    int64_t base = 0, stride = 0;
    if (mode != 0 && mcol < M) level_major_column(mcol, Bc, base, stride);
    for (int ks = 0; ks < nk; ++ks) {
        const int buf = ks & 1;
        // this wave's loads of step ks have landed; after the barrier every
        // wave's have, and buffer buf ^ 1 is free (its readers of step ks - 1
        // passed the barrier)
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        bf16x8 a[2][ND], b[2][ND];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int d = 0; d < ND; ++d)
                a[i][d] = *(const bf16x8 *)(&As[buf][d][aoff[i]]);
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int d = 0; d < ND; ++d)
                b[j][d] = *(const bf16x8 *)(&Bs[buf][d][boff[j]]);
        // the next panels' loads go out after this step's reads, so that no
        // wait for them falls before the matrix-core work of this step
        if (ks + 1 < nk) issue(32 * (ks + 1), buf ^ 1);
        // each product over the four 16 x 16 tiles in turn, so that
        // consecutive MFMAs write different accumulators
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    G[PG[p]][i][j] = mfma(a[i][PA[p]], b[j][PB[p]], G[PG[p]][i][j]);
        if ((ks + 1) % KFOLD == 0 || ks + 1 == nk) {
            // the groups are integers of magnitude below 2^24
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        double v = 0x1p-32 * (double)G[4][i][j][e];
                        v += 0x1p-24 * (double)G[3][i][j][e];
                        v += 0x1p-16 * (double)G[2][i][j][e];
                        v += 0x1p-8 * (double)G[1][i][j][e];
                        acc[i][j][e] += (double)G[0][i][j][e] + v;
                    }
#pragma unroll
                    for (int g = 0; g < ND; ++g) G[g][i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
                }
        }
    }
    // The block's 64 x 64 results go through LDS (rows of ZS doubles, the
    // padding spreading the four row groups of a store over the banks), so
    // that every store instruction writes 64 consecutive cells of one sample
    // (256 bytes of float, 512 of double) instead of four rows of 16.
    constexpr int ZS = 68;
    static_assert(sizeof(As) >= sizeof(double) * BM * ZS, "staging fits the Y panels");
    double *Zs = reinterpret_cast<double *>(&As[0][0][0]);
    __syncthreads();   // every wavefront has read its last panels
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const double z = ldexp(acc[i][j][e], ey[i][e] + eb[j] - 14);
                Zs[(wr + 16 * i + 4 * q4 + e) * ZS + wc + 16 * j + lr] = mode == 0 ? z : exp(z);
            }
    __syncthreads();
    if (mcol < M) {
#pragma unroll 4
        for (int r = 0; r < 16; ++r) {
            const int R = 16 * wave + r;
            const int64_t b = brow0 + R;
            if (b >= Bc) break;
            const double v = Zs[R * ZS + lane];
            if (mode == 0) {
                ((double *)out)[b * M + mcol] = v;
            } else {
                const int64_t q = base + b * stride;
                ((float *)out)[q] = (float)v;
                out64[q] = v;
            }
        }
    }
}

}  // namespace

int64_t mixed_pad_rows(int64_t rows) { return (rows + BM - 1) / BM * BM; }
int64_t mixed_pad_cols(int64_t cols) { return (cols + BN - 1) / BN * BN; }
int mixed_pad_k(int s) { return (s + 31) / 32 * 32; }

void launch_digits_rows(hipStream_t st, const double *X, int64_t rows, int cols, int64_t rs,
                        int64_t rows_pad, int sp, uint16_t *const D[kDigits], int32_t *E)
{
    DigitPtrs P;
    for (int q = 0; q < ND; ++q) P.d[q] = D[q];
    hipLaunchKernelGGL(k_digits_wave, dim3((unsigned)((rows_pad + 3) / 4)), dim3(256), 0, st, X, rows,
                       cols, rs, rows_pad, sp, P, E);
}

void launch_digits_cols(hipStream_t st, const double *X, int64_t rows, int cols, int64_t ks,
                        int64_t rows_pad, int sp, uint16_t *const D[kDigits], int32_t *E)
{
    DigitPtrs P;
    for (int q = 0; q < ND; ++q) P.d[q] = D[q];
    hipLaunchKernelGGL(k_digits_thread, dim3((unsigned)((rows_pad + 255) / 256)), dim3(256), 0, st, X,
                       rows, cols, ks, rows_pad, sp, P, E);
}

void launch_field_digits(hipStream_t st, uint16_t *const Y[kDigits], const int32_t *EY,
                         uint16_t *const Bs[kDigits], const int32_t *EB, int sp, int64_t M, int64_t Bc,
                         void *out, double *out64, int mode)
{
    DigitPtrs PY, PB;
    for (int q = 0; q < ND; ++q) {
        PY.d[q] = Y[q];
        PB.d[q] = Bs[q];
    }
    const int64_t nbm = (Bc + BM - 1) / BM, nbn = (M + BN - 1) / BN;
    const int64_t per = grouped_tile_per(nbm, (int64_t)BM * sp * 2 * ND, nbn * BN * sp * 2 * ND);
    hipLaunchKernelGGL(k_field_digits, dim3((unsigned)(nbm * nbn)), dim3(256), 0, st, PY, EY, PB, EB,
                       sp, M, Bc, nbm, per, out, out64, mode);
}

}  // namespace mlmc
