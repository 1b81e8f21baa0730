// KL field of the mixed-precision path on the gfx950 matrix cores (Section 5,
// eq. truncatedKL): z = Y basis with both operands split into three bf16
// terms, x = x1 + x2 + x3 (x1 = bf16(x), x2 = bf16(x - x1), x3 = bf16(x - x1 -
// x2)), and the six products x1 y1, x1 y2, x2 y1, x1 y3, x3 y1, x2 y2 issued as
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation over each 32-wide K chunk;
// chunk sums are added in FP64 registers, a = exp(z) is formed in FP64 and
// stored as FP32.
//
// Operands are stored K-contiguous (Y splits [rows][sp], basis splits
// transposed [M][sp], sp = s rounded up to 32, zero padded) so that each lane
// loads its 8 consecutive k values as one 16-byte vector.  MFMA lane layout
// (16x16x32): A row l%16 and B column l%16 take k = 8*(l/16) .. +7; lane l
// holds C rows 4*(l/16) .. +3 of column l%16.
#include "internal.hpp"

namespace mlmc {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int WM = 32, WN = 64;        // tile of one wave: 2 x 4 MFMA tiles
constexpr int BM = 64, BN = 128;       // tile of a 4-wave block (2 x 2 waves)

// bf16 nearest to x (ties to even) via the FP32 value, as a bit pattern;
// finite inputs only.  Written out so the split does not depend on the
// rounding mode of a conversion instruction: a directed rounding would bias
// every term the same way.
__device__ __forceinline__ uint16_t bf16_rne(double x, double *value)
{
    uint32_t u = __float_as_uint((float)x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    const uint16_t h = (uint16_t)(u >> 16);
    *value = (double)__uint_as_float((uint32_t)h << 16);
    return h;
}

// split X (rows x cols, element (r, k) at X[r*rs + k*ks]) into three bf16
// arrays [rows_pad][sp]; padding rows and columns are zero.  Each residual is
// exact in FP64.
__global__ void k_split3(const double *__restrict__ X, int64_t rows, int cols, int64_t rs,
                         int64_t ks, int64_t rows_pad, int sp, uint16_t *__restrict__ X1,
                         uint16_t *__restrict__ X2, uint16_t *__restrict__ X3)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= rows_pad * sp) return;
    const int64_t r = t / sp;
    const int k = (int)(t - r * sp);
    const double x = (r < rows && k < cols) ? X[r * rs + (int64_t)k * ks] : 0.0;
    double v1, v2, v3;
    X1[t] = bf16_rne(x, &v1);
    const double r1 = x - v1;
    X2[t] = bf16_rne(r1, &v2);
    X3[t] = bf16_rne(r1 - v2, &v3);
}

__device__ __forceinline__ int64_t level_major_index_m(int64_t m, int64_t b, int64_t Bc)
{
    int g = 0;
    while (g < kMaxMgLevels - 1 && level_offset(g + 1) <= m) ++g;
    const int64_t lo = level_offset(g);
    return Bc * lo + b * level_cells(g) + (m - lo);
}

// out mode 0: z (double) at out[b*M + m]; mode 2: exp(z) as float into the
// level-major chunk pool.
__global__ __launch_bounds__(256) void k_field_bf16x3(
    const __bf16 *__restrict__ Y1, const __bf16 *__restrict__ Y2, const __bf16 *__restrict__ Y3,
    const __bf16 *__restrict__ B1, const __bf16 *__restrict__ B2, const __bf16 *__restrict__ B3,
    int sp, int64_t M, int64_t Bc, void *__restrict__ out, int mode)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t row0 = (int64_t)blockIdx.y * BM + (wave >> 1) * WM;    // sample rows
    const int64_t col0 = (int64_t)blockIdx.x * BN + (wave & 1) * WN;     // field columns
    const int lr = lane & 15, kg = 8 * (lane >> 4);
    double acc[2][4][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[i][j][e] = 0.0;

    for (int k0 = 0; k0 < sp; k0 += 32) {
        bf16x8 a[2][3], bb[4][3];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int64_t o = (row0 + 16 * i + lr) * sp + k0 + kg;
            a[i][0] = *(const bf16x8 *)(Y1 + o);
            a[i][1] = *(const bf16x8 *)(Y2 + o);
            a[i][2] = *(const bf16x8 *)(Y3 + o);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t o = (col0 + 16 * j + lr) * sp + k0 + kg;
            bb[j][0] = *(const bf16x8 *)(B1 + o);
            bb[j][1] = *(const bf16x8 *)(B2 + o);
            bb[j][2] = *(const bf16x8 *)(B3 + o);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                f32x4 c = {0.f, 0.f, 0.f, 0.f};
                // smallest terms first
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][1], bb[j][1], c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][2], bb[j][0], c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][0], bb[j][2], c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][1], bb[j][0], c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][0], bb[j][1], c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][0], bb[j][0], c, 0, 0, 0);
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[i][j][e] += (double)c[e];
            }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t m = col0 + 16 * j + lr;
        if (m >= M) continue;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t b = row0 + 16 * i + 4 * (lane >> 4) + e;
                if (b >= Bc) continue;
                if (mode == 0)
                    ((double *)out)[b * M + m] = acc[i][j][e];
                else
                    ((float *)out)[level_major_index_m(m, b, Bc)] = (float)exp(acc[i][j][e]);
            }
    }
}

}  // namespace

int64_t mixed_pad_rows(int64_t rows) { return (rows + BM - 1) / BM * BM; }
int64_t mixed_pad_cols(int64_t cols) { return (cols + BN - 1) / BN * BN; }
int mixed_pad_k(int s) { return (s + 31) / 32 * 32; }

void launch_split3(hipStream_t st, const double *X, int64_t rows, int cols, int64_t rs, int64_t ks,
                   int64_t rows_pad, int sp, uint16_t *const X3[3])
{
    const int64_t n = rows_pad * sp;
    hipLaunchKernelGGL(k_split3, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, X, rows, cols,
                       rs, ks, rows_pad, sp, X3[0], X3[1], X3[2]);
}

void launch_field_bf16x3(hipStream_t st, uint16_t *const Y[3], uint16_t *const Bs[3], int sp,
                         int64_t M, int64_t Bc, void *out, int mode)
{
    dim3 grid((unsigned)((M + BN - 1) / BN), (unsigned)((Bc + BM - 1) / BM));
    hipLaunchKernelGGL(k_field_bf16x3, grid, dim3(256), 0, st, (const __bf16 *)Y[0],
                       (const __bf16 *)Y[1], (const __bf16 *)Y[2], (const __bf16 *)Bs[0],
                       (const __bf16 *)Bs[1], (const __bf16 *)Bs[2], sp, M, Bc, out, mode);
}

}  // namespace mlmc
