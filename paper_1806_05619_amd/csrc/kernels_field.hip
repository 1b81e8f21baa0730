// KL field of the FP64 path on the gfx950 matrix cores (Section 5, eq.
// truncatedKL): z = Y basis with v_mfma_f64_16x16x4f64, a = exp(z) in the
// epilogue.
//
// Block tile 128 samples x 128 field columns, 8 wavefronts of 32 x 64 (2 x 4
// MFMA tiles, 32 FP64 accumulators per lane), K staged through LDS 16 modes at
// a time.  MFMA lane layout (16x16x4 f64, checked on the device): A row l%16 and
// B column l%16 take mode l/16; lane l holds D rows l/16 + 4 i (i = 0..3) of
// column l%16.
#include "internal.hpp"

namespace mlmc {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int FBM = 128, FBN = 128, FKB = 16, FNT = 512;


// mode 0: z to out[b*M + m]; mode 1: exp(z) into the level-major FP64 pool
__global__ __launch_bounds__(FNT) void k_field_mfma64(const double *__restrict__ Y, int s,
                                                      const double *__restrict__ basis, int64_t ld,
                                                      int64_t M, int64_t Bc, int64_t nbm,
                                                      int64_t per, double *__restrict__ out,
                                                      int mode)
{
    __shared__ double As[FKB][FBM];      // Y tile, mode-major
    __shared__ double Bs[FKB][FBN];      // basis tile
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    // groups of `per` sample tiles over every basis panel (grouped_tile), so
    // that the rows of Y an XCD cycles through stay in its L2
    int64_t mt, nt;
    grouped_tile(xcd_contiguous(blockIdx.x, gridDim.x), nbm, gridDim.x / nbm, per, mt, nt);
    const int64_t row0 = mt * FBM, col0 = nt * FBN;
    const int wr = wave >> 1, wc = wave & 1;      // 4 x 2 waves
    d4 acc[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

    // global loads of the next 16 modes are in flight while the matrix cores
    // work on the current ones (register prefetch)
    const int yr = t >> 2, yk = (t & 3) * 4;          // Y: sample row0 + yr, modes yk..yk+3
    const int bk = t >> 5, bc = (t & 31) * 4;         // basis: mode bk, columns bc..bc+3
    double yv[4], bv[4];
    auto fetch = [&](int k0) {
        const int64_t gr = row0 + yr;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int gk = k0 + yk + q;
            yv[q] = (gr < Bc && gk < s) ? Y[gr * s + gk] : 0.0;
        }
        const int gk = k0 + bk;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t gc = col0 + bc + q;
            bv[q] = (gk < s && gc < M) ? basis[(int64_t)gk * ld + gc] : 0.0;
        }
    };
    fetch(0);
    for (int k0 = 0; k0 < s; k0 += FKB) {
#pragma unroll
        for (int q = 0; q < 4; ++q) As[yk + q][yr] = yv[q];
#pragma unroll
        for (int q = 0; q < 4; ++q) Bs[bk][bc + q] = bv[q];
        __syncthreads();
        if (k0 + FKB < s) fetch(k0 + FKB);
        // one group of 4 modes on the matrix cores
        auto mma = [&](int ks) __attribute__((always_inline)) {
            const int kr = 4 * ks + (lane >> 4);
            double a[2], b[4];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = As[kr][32 * wr + 16 * i + (lane & 15)];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[kr][64 * wc + 16 * j + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] =
                        __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        };
        // in the last, partial stage only the groups that hold a mode below
        // s (the rest is zero padding; a uniform branch)
        const int ksn = s - k0 >= FKB ? FKB / 4 : (s - k0 + 3) / 4;
        mma(0);
#pragma unroll
        for (int ks = 1; ks < FKB / 4; ++ks)
            if (ks < ksn) mma(ks);
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t m = col0 + 64 * wc + 16 * j + (lane & 15);
        if (m >= M) continue;
        // column m of sample b: out[b*M + m], or level g of the level-major pool
        int64_t base = m, stride = M;
        if (mode != 0) {
            int g = 0;
            while (g < kMaxMgLevels - 1 && level_offset(g + 1) <= m) ++g;
            const int64_t lo = level_offset(g);
            base = Bc * lo + (m - lo);
            stride = level_cells(g);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t b = row0 + 32 * wr + 16 * i + (lane >> 4) + 4 * e;
                if (b >= Bc) continue;
                out[base + b * stride] = mode == 0 ? acc[i][j][e] : exp(acc[i][j][e]);
            }
    }
}

}  // namespace

void launch_field_gemm(hipStream_t st, const double *Y, int s, const double *basis, int64_t ld,
                       int64_t M, int64_t Bc, void *out, int mode)
{
    const int64_t nbm = (Bc + FBM - 1) / FBM, nbn = (M + FBN - 1) / FBN;
    const int64_t per = grouped_tile_per(nbm, (int64_t)FBM * s * 8, M * s * 8);
    hipLaunchKernelGGL(k_field_mfma64, dim3((unsigned)(nbm * nbn)), dim3(FNT), 0, st, Y, s, basis,
                       ld, M, Bc, nbm, per, (double *)out, mode);
}

}  // namespace mlmc
