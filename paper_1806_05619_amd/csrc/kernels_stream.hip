// Row-streaming multigrid passes for gfx950 (Section 4), FP64.
//
// One workgroup solves one sample's grid of n x n cells (64 <= n <= 512).
// Lane L owns the two columns 2L and 2L+1, so every row gives each lane one
// red and one black cell, and the workgroup spans the full width: no halo is
// recomputed.  Rows stream bottom to top through a ring of 8 rows of u and 2
// rows of a in LDS; the 2*mu red-black half-sweeps run as a pipeline one row
// apart (half-sweep t works on row s - t while row s + 1 is being fetched),
// which reproduces the global sweep order exactly:
//   pre  pass: half-sweeps red, black, ... then the residual of row s-2mu-1
//              and, for every odd row, the 4-cell restriction -> coarse f;
//   post pass: rows arrive as u + P e_c (bilinear, odd reflection), half-sweeps
//              black, red, ...; row s-2mu is final.
// Face weights, diagonal and right-hand side of a row are computed once when
// the row above has arrived and then travel down a register window.
#include <type_traits>

#include "internal.hpp"

namespace mlmc {
namespace {

__device__ __forceinline__ double frcp_s(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}

__device__ __forceinline__ double hmean(double ap, double an) { return 2.0 * ap * an * frcp_s(ap + an); }

__device__ __forceinline__ double codd_s(const double *__restrict__ e, int nc, int I, int J)
{
    double sg = 1.0;
    if (I < 0) { I = 0; sg = -sg; }
    if (I >= nc) { I = nc - 1; sg = -sg; }
    if (J < 0) { J = 0; sg = -sg; }
    if (J >= nc) { J = nc - 1; sg = -sg; }
    return sg * e[I + nc * J];
}

// compile-time loop: f(integral_constant<int, I>) for I = B .. E-1, so that
// register-window slots are always addressed with constant indices
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// Stencil of the lane's two cells of one row, stored by colour (red cell
// first): sweeps of a known colour then read fixed fields, so the window stays
// in registers.  wS of a cell is wN of the cell below, which has the other
// colour in the row below.
struct RowW {
    double wE_r, wW_r, wN_r, dw_r, inv_r, rhs_r;   // dw: wall term, 2 a_P per wall face
    double wE_b, wW_b, wN_b, dw_b, inv_b, rhs_b;
};

// field-wise copy (a struct copy becomes a memcpy that keeps the window in
// scratch memory)
__device__ __forceinline__ void copy_row(RowW &d, const RowW &s)
{
    d.wE_r = s.wE_r; d.wW_r = s.wW_r; d.wN_r = s.wN_r; d.dw_r = s.dw_r; d.inv_r = s.inv_r; d.rhs_r = s.rhs_r;
    d.wE_b = s.wE_b; d.wW_b = s.wW_b; d.wN_b = s.wN_b; d.dw_b = s.dw_b; d.inv_b = s.inv_b; d.rhs_b = s.rhs_b;
}

__device__ __forceinline__ void zero_row(RowW &d)
{
    d.wE_r = d.wW_r = d.wN_r = d.dw_r = d.inv_r = d.rhs_r = 0.0;
    d.wE_b = d.wW_b = d.wN_b = d.dw_b = d.inv_b = d.rhs_b = 0.0;
}

// coarse values of row R's prolongation for lane L: columns L-1, L, L+1 of
// coarse rows J = R/2 and J + sy
struct Coarse6 {
    double m0, c0, p0, m1, c1, p1;
};

__device__ __forceinline__ void load_coarse(Coarse6 &k, const double *__restrict__ e, int nc, int L,
                                            int R)
{
    const int J = R >> 1, J2 = J + ((R & 1) ? 1 : -1);
    k.m0 = codd_s(e, nc, L - 1, J);
    k.c0 = codd_s(e, nc, L, J);
    k.p0 = codd_s(e, nc, L + 1, J);
    k.m1 = codd_s(e, nc, L - 1, J2);
    k.c1 = codd_s(e, nc, L, J2);
    k.p1 = codd_s(e, nc, L + 1, J2);
}

// (9 e_IJ + 3 e_{I+sx,J} + 3 e_{I,J+sy} + e_{I+sx,J+sy}) / 16 for columns 2L (sx=-1), 2L+1 (sx=+1)
__device__ __forceinline__ void prolong2(const Coarse6 &k, double &v0, double &v1)
{
    v0 = prolong_9331(k.c0, k.m0, k.c1, k.m1);
    v1 = prolong_9331(k.c0, k.p0, k.c1, k.p1);
}

// PRE: init 0 = read u_in, 1 = zero, 2 = u = P uc.  POST: u = u_in + P ec.
// The result goes to u_out (may equal u_in: rows are read before written).
// F1: f = 1 (the top level of a stage), so every rhs is h^2 and no row of
// the register window carries one.
template <int MU, bool PRE, bool F1>
__global__ __launch_bounds__(256) void k_stream(const double *__restrict__ a,
                                                 const double *__restrict__ f,
                                                 const double *u_in, double *u_out,
                                                 const double *__restrict__ ec, int n, int64_t Bc,
                                                 int init, double *__restrict__ fc,
                                                 const int32_t *__restrict__ active)
{
    constexpr int D = 2 * MU;                  // half-sweeps in the pass
    constexpr int NS = PRE ? D + 2 : D + 1;    // rows s-1 .. s-NS in the register window
    extern __shared__ double smem[];
    double *u_ring = smem;                     // [8][n]
    double *a_ring = smem + 8 * n;             // [2][n]

    const int64_t b = blockIdx.x;
    if (b >= Bc) return;
    if (active && !active[b]) return;
    const int L = threadIdx.x;
    const bool lane = L < n / 2;
    const int c0 = 2 * L, c1 = 2 * L + 1;
    const int nc = n / 2;
    const int64_t cells = (int64_t)n * n;
    const double *ab = a + b * cells;
    const double *fb = f ? f + b * cells : nullptr;
    const double *ub = u_in ? u_in + b * cells : nullptr;
    double *ob = u_out + b * cells;
    const double *eb = ec ? ec + b * (int64_t)nc * nc : nullptr;
    double *fcb = PRE ? fc + b * (int64_t)nc * nc : nullptr;
    const double h2 = 1.0 / ((double)n * (double)n);
    const double inv_h2 = (double)n * (double)n;
    const bool need_coarse = PRE ? (init == 2) : true;

    for (int q = threadIdx.x; q < 10 * n; q += blockDim.x) smem[q] = 0.0;

    // prefetch registers for the next row
    double pa0 = 0, pa1 = 0, pu0 = 0, pu1 = 0, pf0 = 1.0, pf1 = 1.0;
    Coarse6 pk{};
    auto fetch = [&](int R) __attribute__((always_inline)) {
        if (!lane || R >= n) return;
        const int64_t o = (int64_t)R * n;
        pa0 = ab[o + c0];
        pa1 = ab[o + c1];
        if (fb) {
            pf0 = fb[o + c0];
            pf1 = fb[o + c1];
        }
        if (need_coarse) load_coarse(pk, eb, nc, L, R);
        if (!PRE || init == 0) {
            pu0 = ub[o + c0];
            pu1 = ub[o + c1];
        }
    };
    fetch(0);
    __syncthreads();

    RowW w[NS];
    static_for<0, NS>([&](auto K) __attribute__((always_inline)) { zero_row(w[K.value]); });
    double rhs_cur0 = 0, rhs_cur1 = 0, rkeep0 = 0, rkeep1 = 0;
    const int s_end = PRE ? n + D : n + D - 1;

    for (int s = 0; s <= s_end; ++s) {
        // (A) row s enters the rings; fetch row s + 1
        double rhs_prev0 = rhs_cur0, rhs_prev1 = rhs_cur1;
        if (s < n && lane) {
            double u0 = pu0, u1 = pu1;
            if (need_coarse) {
                double v0, v1;
                prolong2(pk, v0, v1);
                if (PRE) { u0 = v0; u1 = v1; }
                else { u0 += v0; u1 += v1; }
            } else if (PRE && init == 1) {
                u0 = u1 = 0.0;
            }
            u_ring[(s & 7) * n + c0] = u0;
            u_ring[(s & 7) * n + c1] = u1;
            a_ring[(s & 1) * n + c0] = pa0;
            a_ring[(s & 1) * n + c1] = pa1;
            rhs_cur0 = h2 * pf0;
            rhs_cur1 = h2 * pf1;
            fetch(s + 1);
        }
        __syncthreads();

        // (B) stencil of row q = s - 1 (its upper neighbour row s is now present)
        static_for<0, NS - 1>([&](auto K) __attribute__((always_inline)) {
            copy_row(w[NS - 1 - K.value], w[NS - 2 - K.value]);
        });
        const int q = s - 1;
        if (q >= 0 && q < n && lane) {
            // no contraction: weights and diagonal round as in the tile passes
#pragma clang fp contract(off)
            const double *aq = a_ring + (q & 1) * n, *aq1 = a_ring + ((q + 1) & 1) * n;
            const double ap0 = aq[c0], ap1 = aq[c1];
            // faces of the two cells (zero weight at a wall, whose 2a_P goes to d)
            const double wE0 = hmean(ap0, ap1);                       // c0|c1
            const double wE1 = (c1 + 1 < n) ? hmean(ap1, aq[c1 + 1]) : 0.0;
            const double wW0 = (c0 > 0) ? hmean(ap0, aq[c0 - 1]) : 0.0;
            const double wN0 = (q + 1 < n) ? hmean(ap0, aq1[c0]) : 0.0;
            const double wN1 = (q + 1 < n) ? hmean(ap1, aq1[c1]) : 0.0;
            // south faces: wN of the cell below, stored by that row's colours
            // (row q-1 has the opposite parity: c0 there is black if c0 here is red)
            const bool odd = q & 1;                // c0 is red iff q is even
            const double wS0 = (q > 0) ? (odd ? w[1].wN_r : w[1].wN_b) : 0.0;
            const double wS1 = (q > 0) ? (odd ? w[1].wN_b : w[1].wN_r) : 0.0;
            double d0 = 0.0, d1 = 0.0;             // E, W, N, S in this order
            d0 += wE0;
            d0 += (c0 > 0) ? wW0 : 2.0 * ap0;
            d0 += (q + 1 < n) ? wN0 : 2.0 * ap0;
            d0 += (q > 0) ? wS0 : 2.0 * ap0;
            d1 += (c1 + 1 < n) ? wE1 : 2.0 * ap1;
            d1 += wE0;
            d1 += (q + 1 < n) ? wN1 : 2.0 * ap1;
            d1 += (q > 0) ? wS1 : 2.0 * ap1;
            const double dw0 = ((c0 > 0) ? 0.0 : 2.0 * ap0) + ((q + 1 < n) ? 0.0 : 2.0 * ap0) +
                               ((q > 0) ? 0.0 : 2.0 * ap0);
            const double dw1 = ((c1 + 1 < n) ? 0.0 : 2.0 * ap1) + ((q + 1 < n) ? 0.0 : 2.0 * ap1) +
                               ((q > 0) ? 0.0 : 2.0 * ap1);
            const double i0 = frcp_s(d0), i1 = frcp_s(d1);
            RowW &r = w[0];
            r.wE_r = odd ? wE1 : wE0;   r.wE_b = odd ? wE0 : wE1;
            r.wW_r = odd ? wE0 : wW0;   r.wW_b = odd ? wW0 : wE0;
            r.wN_r = odd ? wN1 : wN0;   r.wN_b = odd ? wN0 : wN1;
            r.dw_r = odd ? dw1 : dw0;   r.dw_b = odd ? dw0 : dw1;
            r.inv_r = odd ? i1 : i0;    r.inv_b = odd ? i0 : i1;
            r.rhs_r = odd ? rhs_prev1 : rhs_prev0;
            r.rhs_b = odd ? rhs_prev0 : rhs_prev1;
        }

        // (C) half-sweep t on row s - t (register slot t - 1)
        static_for<1, D + 1>([&](auto T) __attribute__((always_inline)) {
            constexpr int t = T.value;
            const int rr = s - t;
            if (rr >= 0 && rr < n && lane) {
                constexpr bool red = PRE ? (t & 1) : !(t & 1);
                const RowW &r = w[t - 1];
                const RowW &rs = w[t];
                double *row = u_ring + (rr & 7) * n;
                const double *up = u_ring + ((rr + 1) & 7) * n;
                const double *dn = u_ring + ((rr - 1) & 7) * n;
                // the red cell of row rr is column c0 when rr is even
                const int c = red ? c0 + (rr & 1) : c1 - (rr & 1);
                // explicit fma in the face order E, W, N, S of the tile passes,
                // so that both kinds of pass give the same bits
                double num = F1 ? h2 : (red ? r.rhs_r : r.rhs_b);
                if (c + 1 < n) num = fma(red ? r.wE_r : r.wE_b, row[c + 1], num);
                if (c > 0) num = fma(red ? r.wW_r : r.wW_b, row[c - 1], num);
                if (rr + 1 < n) num = fma(red ? r.wN_r : r.wN_b, up[c], num);
                if (rr > 0) num = fma(red ? rs.wN_b : rs.wN_r, dn[c], num);
                row[c] = num * (red ? r.inv_r : r.inv_b);
            }
            __syncthreads();
        });

        // (D) leave the pipeline
        if (PRE) {
            const int rr = s - D - 1;
            if (rr >= 0 && rr < n && lane) {
                const RowW &r = w[D];
                const RowW &rs = w[D + 1];
                const double *row = u_ring + (rr & 7) * n;
                const double *up = u_ring + ((rr + 1) & 7) * n, *dn = u_ring + ((rr - 1) & 7) * n;
                const int cr = c0 + (rr & 1), cb = c1 - (rr & 1);
                const double ur = row[cr], ubk = row[cb];
                // net flux face by face, w (u_P - u_nbr) in the order E, W, N,
                // S with explicit fma, a wall face as 2 a_P (u_P - 0): the
                // rounding of the tile passes.  2 a_P is the wall term, halved
                // (exactly) at a corner, whose two wall faces it sums.
                auto flux = [&](double u, int c, double wE, double wW, double wN, double wS,
                                double dw) {
                    const int walls = (c == 0) + (c + 1 == n) + (rr == 0) + (rr + 1 == n);
                    const double ww = walls == 2 ? 0.5 * dw : dw;
                    double v = (c + 1 < n ? wE : ww) * (u - (c + 1 < n ? row[c + 1] : 0.0));
                    v = fma(c > 0 ? wW : ww, u - (c > 0 ? row[c - 1] : 0.0), v);
                    v = fma(rr + 1 < n ? wN : ww, u - (rr + 1 < n ? up[c] : 0.0), v);
                    v = fma(rr > 0 ? wS : ww, u - (rr > 0 ? dn[c] : 0.0), v);
                    return v;
                };
                const double fr = flux(ur, cr, r.wE_r, r.wW_r, r.wN_r, rs.wN_b, r.dw_r);
                const double fbk = flux(ubk, cb, r.wE_b, r.wW_b, r.wN_b, rs.wN_r, r.dw_b);
                const double resr = inv_h2 * ((F1 ? h2 : r.rhs_r) - fr);
                const double resb = inv_h2 * ((F1 ? h2 : r.rhs_b) - fbk);
                const bool odd = rr & 1;
                const double u0 = odd ? ubk : ur, u1 = odd ? ur : ubk;
                const double res0 = odd ? resb : resr, res1 = odd ? resr : resb;
                const int64_t o = (int64_t)rr * n;
                ob[o + c0] = u0;
                ob[o + c1] = u1;
                if (rr & 1) fcb[L + (int64_t)nc * (rr >> 1)] = 0.25 * (rkeep0 + rkeep1 + res0 + res1);
                else { rkeep0 = res0; rkeep1 = res1; }
            }
        } else {
            const int rr = s - D;
            if (rr >= 0 && rr < n && lane) {
                const double *row = u_ring + (rr & 7) * n;
                const int64_t o = (int64_t)rr * n;
                ob[o + c0] = row[c0];
                ob[o + c1] = row[c1];
            }
        }
    }
}

template <int MU, bool PRE, bool F1>
void launch_one(hipStream_t st, const double *a, const double *f, const double *u_in,
                double *u_out, const double *ec, int n, int64_t Bc, int init, double *fc,
                const int32_t *active)
{
    // once per instantiation; the static's initialisation is thread-safe
    static const bool attr_set = [] {
        (void)hipFuncSetAttribute((const void *)k_stream<MU, PRE, F1>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        return true;
    }();
    (void)attr_set;
    const size_t lds = sizeof(double) * 10 * (size_t)n;
    const int threads = n / 2 < 64 ? 64 : n / 2;
    hipLaunchKernelGGL((k_stream<MU, PRE, F1>), dim3((unsigned)Bc), dim3(threads), lds, st, a, f, u_in,
                       u_out, ec, n, Bc, init, fc, active);
}

}  // namespace

bool stream_supported(int n) { return n >= 64 && n <= 512; }

void launch_pre_stream(hipStream_t st, int mu1, const double *a, const double *f,
                       const double *u_in, double *u_out, const double *uc, int n, int64_t Bc,
                       int init, double *fc, const int32_t *active)
{
    if (mu1 == 2)
        f ? launch_one<2, true, false>(st, a, f, u_in, u_out, uc, n, Bc, init, fc, active)
          : launch_one<2, true, true>(st, a, f, u_in, u_out, uc, n, Bc, init, fc, active);
    else
        f ? launch_one<1, true, false>(st, a, f, u_in, u_out, uc, n, Bc, init, fc, active)
          : launch_one<1, true, true>(st, a, f, u_in, u_out, uc, n, Bc, init, fc, active);
}

void launch_post_stream(hipStream_t st, int mu2, const double *a, const double *f,
                        const double *u_in, double *u_out, const double *ec, int n, int64_t Bc,
                        const int32_t *active)
{
    if (mu2 == 2)
        f ? launch_one<2, false, false>(st, a, f, u_in, u_out, ec, n, Bc, 0, nullptr, active)
          : launch_one<2, false, true>(st, a, f, u_in, u_out, ec, n, Bc, 0, nullptr, active);
    else
        f ? launch_one<1, false, false>(st, a, f, u_in, u_out, ec, n, Bc, 0, nullptr, active)
          : launch_one<1, false, true>(st, a, f, u_in, u_out, ec, n, Bc, 0, nullptr, active);
}

}  // namespace mlmc
