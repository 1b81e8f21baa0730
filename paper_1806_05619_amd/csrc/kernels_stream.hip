// Row-streaming multigrid passes for gfx950 (Section 4), FP64 and FP32 (the
// mixed path's V-cycles), each with the arithmetic of the tile passes of its type.
//
// One workgroup solves the grids of SPB samples of n x n cells (32 <= n <=
// 2048; SPB = 64 / (n/2) samples on grids narrower than a wavefront, so that no
// lane idles, else 1, with n/2 threads: up to 1024 on 2048^2, the largest
// workgroup).  Lane L of a sample owns the two columns 2L and 2L+1,
// so every row gives each lane one red and one black cell, and the lanes of a
// sample span the full width: no halo is recomputed.  Rows stream bottom to
// top through a ring of 8 rows of u and 2 rows of a in LDS, each row stored
// as its even columns followed by its odd columns, so that the lanes of a
// wavefront touch consecutive words in every access (a cell's E and W
// neighbours sit in the other plane, at the lane's own or the next or
// previous lane's slot): no bank conflicts.  Lanes load and store their two
// cells of a row as one 8- or 16-byte vector.  The 2*mu
// red-black half-sweeps run as a pipeline one row apart (half-sweep t works
// on row s - t while row s + 1 is being fetched), which reproduces the global
// sweep order exactly:
//   pre  pass: half-sweeps red, black, ... then the residual of row s-2mu-1
//              and, for every odd row, the 4-cell restriction -> coarse f;
//   post pass: rows arrive as u + P e_c (bilinear, odd reflection), half-sweeps
//              black, red, ...; row s-2mu is final.
// Face weights, diagonal and right-hand side of a row are computed once when
// the row above has arrived and then stay in a register window.  A row step
// needs one workgroup barrier (lanes exchange only values of earlier steps),
// and the row loop is unrolled by 8 so that window slots and ring rows are
// compile-time indices.
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

// FP32 (the mixed path's V-cycles): one Newton step, as the tile passes
__device__ __forceinline__ float frcp_s(float x)
{
    float y = __builtin_amdgcn_rcpf(x);
    float e = fmaf(-x, y, 1.0f);
    return fmaf(y, e, y);
}

template <typename T>
__device__ __forceinline__ T hmean(T ap, T an) { return T(2) * ap * an * frcp_s(ap + an); }


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

// Face weights of the lane's two cells (columns c0 = 2L, c1 = 2L+1) of one
// row, by column: the face between them is stored once, a wall face holds
// 2 a_P as in the tile passes, and the south faces of a row are the north
// faces of the row below (row -1 holds the south wall of row 0).  The
// diagonal and its reciprocal are formed again at each use from the same
// rounded weights in the same order, so they carry the same bits as a
// stored copy would, and the window needs 5 doubles a row (7 with f).
template <bool F1, typename T>
struct RowW {
    T wW0, wC, wE1, wN0, wN1;   // W face of c0, c0|c1, E face of c1, N faces
    T rhs0, rhs1;               // h^2 f (unused when f = 1)
};

template <bool F1, typename T>
__device__ __forceinline__ void zero_row(RowW<F1, T> &d)
{
    d.wW0 = d.wC = d.wE1 = d.wN0 = d.wN1 = T(0);
    d.rhs0 = d.rhs1 = T(0);
}

// coarse values of row R's prolongation for lane L: columns L-1, L, L+1 of
// coarse rows J = R/2 and J + sy.  Outside the coarse grid the correction is
// continued oddly (reflected, sign flipped).  The loads take the clamped
// indices only and the signs are applied when the row is used, so that the
// loads of the next row stay in flight through a whole row step.
template <typename T>
struct Coarse6 {
    T m0, c0, p0, m1, c1, p1;
};

template <typename T>
__device__ __forceinline__ void load_coarse_raw(Coarse6<T> &k, const T *__restrict__ e, int nc,
                                                int L, int R)
{
    const int J = R >> 1;
    int J2 = J + ((R & 1) ? 1 : -1);
    J2 = J2 < 0 ? 0 : (J2 >= nc ? nc - 1 : J2);
    const int Im = L > 0 ? L - 1 : 0, Ip = L + 1 < nc ? L + 1 : nc - 1;
    const T *r0 = e + (int64_t)nc * J, *r1 = e + (int64_t)nc * J2;
    k.m0 = r0[Im];
    k.c0 = r0[L];
    k.p0 = r0[Ip];
    k.m1 = r1[Im];
    k.c1 = r1[L];
    k.p1 = r1[Ip];
}

// the reflection signs of load_coarse_raw's values (products of exact -1
// factors: the bits of the reflected values themselves)
template <typename T>
__device__ __forceinline__ void sign_coarse(Coarse6<T> &k, int nc, int L, int R, int n)
{
    if (L == 0) { k.m0 = -k.m0; k.m1 = -k.m1; }
    if (L == nc - 1) { k.p0 = -k.p0; k.p1 = -k.p1; }
    if (R == 0 || R == n - 1) { k.m1 = -k.m1; k.c1 = -k.c1; k.p1 = -k.p1; }
}

// (9 e_IJ + 3 e_{I+sx,J} + 3 e_{I,J+sy} + e_{I+sx,J+sy}) / 16 for columns 2L (sx=-1), 2L+1 (sx=+1)
template <typename T>
__device__ __forceinline__ void prolong2(const Coarse6<T> &k, T &v0, T &v1)
{
    v0 = prolong_9331(k.c0, k.m0, k.c1, k.m1);
    v1 = prolong_9331(k.c0, k.p0, k.c1, k.p1);
}

// Faces of the lane's cell in column K (0: c0, 1: c1) of a row: r the row,
// rs the row below.
template <int K, bool F1, typename T>
struct Faces {
    T e, w, nn, s;
    __device__ __forceinline__ Faces(const RowW<F1, T> &r, const RowW<F1, T> &rs)
    {
        e = K == 0 ? r.wC : r.wE1;
        w = K == 0 ? r.wW0 : r.wC;
        nn = K == 0 ? r.wN0 : r.wN1;
        s = K == 0 ? rs.wN0 : rs.wN1;
    }
    // the diagonal as the tile passes form it: E + W + N + S, no contraction
    __device__ __forceinline__ T diag() const
    {
#pragma clang fp contract(off)
        T d = e;
        d += w;
        d += nn;
        d += s;
        return d;
    }
};

// PRE: INIT 0 = read u_in, 1 = zero, 2 = u = P uc (a template parameter, so
// that a launch holds registers only for the loads it makes).  POST (INIT 0):
// u = u_in + P ec.
// The result goes to u_out (may equal u_in: rows are read before written).
// F1: f = 1 (the top level of a stage), so every rhs is h^2 and no row of
// the register window carries one.
// T: double (FP64 path) or float (the mixed path's V-cycles), with the
// arithmetic of the tile passes of the same type.
// Register budget: 128 (4 waves per SIMD) with f = 1, whose window carries
// no right-hand side, or in FP32, else 168 (3 waves); measured against each
// other in FP64.  The grid side N is a template parameter, so that every
// LDS address of a ring row is one lane offset plus an immediate.
// SPB: samples per workgroup; NT: the launch bound (256, or N/2 above 512^2;
// a 1024-thread workgroup holds 4 waves per SIMD, so 128 registers).
template <int N>
struct StreamShape {
    static constexpr int SPB = N >= 128 ? 1 : 64 / (N / 2);
    static constexpr int NT = N <= 512 ? 256 : N / 2;
    static constexpr int THREADS = SPB * (N / 2);
};

template <int MU, bool PRE, bool F1, int N, int INIT, typename T>
__global__ __launch_bounds__(StreamShape<N>::NT)
__attribute__((amdgpu_waves_per_eu(F1 || sizeof(T) == 4 || N > 1024 ? 4 : 3)))
void k_stream(const T *__restrict__ a, const T *__restrict__ f, const T *u_in, T *u_out,
              const T *__restrict__ ec, int64_t Bc, T *__restrict__ fc,
              const int32_t *__restrict__ active)
{
    constexpr int n = N;
    constexpr int SPB = StreamShape<N>::SPB;
    constexpr int D = 2 * MU;                  // half-sweeps in the pass
    constexpr int NS = PRE ? D + 2 : D + 1;    // rows s-1 .. s-NS in the register window
    // rows fetched ahead: two in FP32; one in FP64, whose second row of
    // registers measured no faster (or spills)
    constexpr int PD = sizeof(T) == 4 ? 2 : 1;
    static_assert(8 % PD == 0, "prefetch sets are indexed by row mod 8");
    extern __shared__ double smem_words[];
    T *smem = reinterpret_cast<T *>(smem_words);
    constexpr int nc = n / 2;
    // sample `sub` of the block: lanes sub * n/2 .. (sub+1) * n/2 - 1; a
    // sample past the batch or inactive keeps its lanes idle but passes every
    // barrier with the others
    const int sub = SPB == 1 ? 0 : threadIdx.x / nc;
    const int L = threadIdx.x - sub * nc;
    const int64_t bs = (int64_t)blockIdx.x * SPB + sub;
    if constexpr (SPB == 1) {           // the whole workgroup is one sample
        if (bs >= Bc) return;
        if (active && !active[bs]) return;
    }
    const bool lane = SPB == 1 ? L < nc : (sub < SPB && bs < Bc && (!active || active[bs]));
    const int64_t b = (SPB == 1 || lane) ? bs : 0;
    T *u_ring = smem + (SPB == 1 || !lane ? 0 : sub) * 10 * n;   // [8][n]
    T *a_ring = u_ring + 8 * n;                                  // [2][n]
    const int c0 = 2 * L, c1 = 2 * L + 1;
    // LDS slots of a row (even columns, then odd ones): the lane's cells c0
    // and c1, and their outer neighbours c0 - 1 (odd plane, lane L-1) and
    // c1 + 1 (even plane, lane L+1)
    const int l0 = L, l1 = nc + L, lw = nc + L - 1, le = L + 1;
    using V2 = typename std::conditional<sizeof(T) == 4, float2, double2>::type;
    auto ld2 = [](const T *p, T &x, T &y) __attribute__((always_inline)) {
        const V2 v = *reinterpret_cast<const V2 *>(p);
        x = v.x;
        y = v.y;
    };
    auto st2 = [](T *p, T x, T y) __attribute__((always_inline)) {
        V2 v;
        v.x = x;
        v.y = y;
        *reinterpret_cast<V2 *>(p) = v;
    };
    const int64_t cells = (int64_t)n * n;
    const T *ab = a + b * cells;
    const T *fb = f ? f + b * cells : nullptr;
    const T *ub = u_in ? u_in + b * cells : nullptr;
    T *ob = u_out + b * cells;
    const T *eb = ec ? ec + b * (int64_t)nc * nc : nullptr;
    T *fcb = PRE ? fc + b * (int64_t)nc * nc : nullptr;
    const T h2 = T(1) / (T(n) * T(n));
    const T inv_h2 = T(n) * T(n);
    constexpr bool need_coarse = PRE ? INIT == 2 : true;

    for (int q = threadIdx.x; q < SPB * 10 * n; q += blockDim.x) smem[q] = T(0);

    // prefetch registers: row R is fetched PD row steps before it enters,
    // into set R % PD
    struct Prefetch {
        T a0 = 0, a1 = 0, u0 = 0, u1 = 0, f0 = 1, f1 = 1;
        Coarse6<T> k{};
    };
    Prefetch pre[PD];
    // In the post pass unconditional, so that no register keeps an older
    // value beside the new one: past the last row the last row is fetched
    // again, and an idle lane (b = 0) fetches sample 0; neither is used.
    // (Measured the other way round in the pre pass, whose register budget
    // it overflows.)
    auto fetch = [&](int R, Prefetch &pp) __attribute__((always_inline)) {
        if constexpr (PRE) {
            if (!lane || R >= n) return;
        } else {
            R = R < n ? R : n - 1;
        }
        const int64_t o = (int64_t)R * n + c0;
        ld2(ab + o, pp.a0, pp.a1);
        if (!F1) ld2(fb + o, pp.f0, pp.f1);
        if constexpr (need_coarse) load_coarse_raw(pp.k, eb, nc, L, R);
        if constexpr (!PRE || INIT == 0) ld2(ub + o, pp.u0, pp.u1);
    };
    static_for<0, PD>([&](auto K) __attribute__((always_inline)) { fetch(K.value, pre[K.value]); });

    // The register window and the u ring are indexed by row mod 8, and the
    // row loop is unrolled by 8, so that every slot is a compile-time index:
    // the window needs no moves and the ring rows sit at fixed offsets.  At
    // most NS <= 8 window slots are live.
    static_assert(NS <= 8 && D + 2 <= 8, "window and ring hold 8 rows");
    RowW<F1, T> w[8];
    static_for<0, 8>([&](auto K) __attribute__((always_inline)) { zero_row(w[K.value]); });
    T rhs_cur0 = 0, rhs_cur1 = 0, rkeep0 = 0, rkeep1 = 0;
    // With mu = 2, half-sweeps t and t + 2 update the same cell of a row, two
    // steps apart: the reciprocal of its diagonal is formed at the first and
    // kept for the second (the same bits), by row mod 4, for the colour of
    // half-sweeps 1 and 3 (rdA) and of 2 and 4 (rdB).
    T rdA[4] = {}, rdB[4] = {};
    const int s_end = PRE ? n + D : n + D - 1;

    // One pipeline step for row s entering; J = s & 8 - 1 and P = s & 1 are
    // compile-time constants.
    auto step = [&](int s_in, auto Jc) __attribute__((always_inline)) {
        constexpr int J = decltype(Jc)::value;
        constexpr int P = J & 1;
        // the row index as an opaque scalar: without this the unrolled steps'
        // row addresses become separate pointer induction variables, more
        // than the registers hold (an empty asm: no instruction is emitted)
        int s = s_in;
        asm volatile("" : "+s"(s));
        // The one barrier of a row step.  A lane shares nothing with another
        // lane inside a step: every value it reads from another lane's columns
        // (the E/W neighbours of a half-sweep or of the residual, the a of
        // row s-1 beside its own) was written in an earlier step, and every
        // ring slot it writes was last read by another lane in an earlier
        // step (the u slot of row s-8, the a slot of row s-2, cells of the
        // colour that the previous step's next half-sweep read as E/W
        // neighbours).  What a lane reads of its own columns it wrote itself.
        __syncthreads();
        // (A) row s enters the rings; fetch row s + 1
        const T rhs_prev0 = rhs_cur0, rhs_prev1 = rhs_cur1;
        Prefetch &pp = pre[J % PD];      // row s's set (row mod PD)
        if (s < n && lane) {
            T u0 = pp.u0, u1 = pp.u1;
            if constexpr (need_coarse) {
                Coarse6<T> k = pp.k;
                sign_coarse(k, nc, L, s, n);
                T v0, v1;
                prolong2(k, v0, v1);
                if (PRE) { u0 = v0; u1 = v1; }
                else { u0 += v0; u1 += v1; }
            } else if (PRE && INIT == 1) {
                u0 = u1 = T(0);
            }
            u_ring[J * n + l0] = u0;
            u_ring[J * n + l1] = u1;
            a_ring[P * n + l0] = pp.a0;
            a_ring[P * n + l1] = pp.a1;
        }
        if (!F1) {
            rhs_cur0 = h2 * pp.f0;
            rhs_cur1 = h2 * pp.f1;
        }
        if (!PRE || (s < n && lane)) fetch(s + PD, pp);

        // window slot of row s - k
        auto slot = [](int k) constexpr { return (J - k) & 7; };
        // (B) faces of row q = s - 1 (its upper neighbour row s is now
        // present).  Formed whether or not q is a row of the grid, so that a
        // slot's previous row is dead once the step begins: a slot filled
        // outside the grid is never read, and every LDS read stays inside
        // the workgroup's rings.
        const int q = s - 1;
        {
            const T *aq = a_ring + (1 - P) * n, *aq1 = a_ring + P * n;
            const T ap0 = aq[l0], ap1 = aq[l1];
            RowW<F1, T> &r = w[slot(1)];
            r.wC = hmean(ap0, ap1);
            r.wW0 = c0 > 0 ? hmean(ap0, aq[lw]) : T(2) * ap0;
            r.wE1 = c1 + 1 < n ? hmean(ap1, aq[le]) : T(2) * ap1;
            r.wN0 = q + 1 < n ? hmean(ap0, aq1[l0]) : T(2) * ap0;
            r.wN1 = q + 1 < n ? hmean(ap1, aq1[l1]) : T(2) * ap1;
            if constexpr (!F1) {
                r.rhs0 = rhs_prev0;
                r.rhs1 = rhs_prev1;
            }
            if (q == 0) {          // south wall of row 0, in the slot of row -1
                w[slot(2)].wN0 = T(2) * ap0;
                w[slot(2)].wN1 = T(2) * ap1;
            }
        }

        // (C) half-sweep t on row s - t
        static_for<1, D + 1>([&](auto Tc) __attribute__((always_inline)) {
            constexpr int t = Tc.value;
            const int rr = s - t;
            constexpr bool red = PRE ? (t & 1) : !(t & 1);
            // the red cell of row rr is column c0 when rr is even
            constexpr int K = red ? ((P - t) & 1) : 1 - ((P - t) & 1);
            const Faces<K, F1, T> fw(w[slot(t)], w[slot(t + 1)]);
            // formed whether or not rr is a row of the grid, so that no cache
            // slot keeps an older value beside the new one
            T rdiag;
            if constexpr (MU == 2) {
                T &rd = (t & 1) ? rdA[(J - t) & 3] : rdB[(J - t) & 3];
                if constexpr (t <= 2) rd = frcp_s(fw.diag());
                rdiag = rd;
            } else {
                rdiag = frcp_s(fw.diag());
            }
            if (rr >= 0 && rr < n && lane) {
                T *row = u_ring + slot(t) * n;
                const T *up = u_ring + slot(t - 1) * n;
                const T *dn = u_ring + slot(t + 1) * n;
                const int c = K == 0 ? c0 : c1;
                // slots of the cell and of its E and W neighbours
                const int lc = K == 0 ? l0 : l1, lE = K == 0 ? l1 : le, lW = K == 0 ? lw : l0;
                // explicit fma in the face order E, W, N, S of the tile passes
                // (a wall face meets a neighbour of value 0 there: skipped)
                T num = F1 ? h2 : (K == 0 ? w[slot(t)].rhs0 : w[slot(t)].rhs1);
                if (c + 1 < n) num = fma(fw.e, row[lE], num);
                if (c > 0) num = fma(fw.w, row[lW], num);
                if (rr + 1 < n) num = fma(fw.nn, up[lc], num);
                if (rr > 0) num = fma(fw.s, dn[lc], num);
                row[lc] = num * rdiag;
            }
        });

        // (D) leave the pipeline
        if constexpr (PRE) {
            const int rr = s - D - 1;
            if (rr >= 0 && rr < n && lane) {
                const T *row = u_ring + slot(D + 1) * n;
                const T *up = u_ring + slot(D) * n, *dn = u_ring + slot(D + 2) * n;
                // net flux face by face, w (u_P - u_nbr) in the order E, W, N,
                // S with explicit fma, a wall face as 2 a_P (u_P - 0): the
                // rounding of the tile passes
                auto flux = [&](auto Kc) __attribute__((always_inline)) {
                    constexpr int K = decltype(Kc)::value;
                    const Faces<K, F1, T> fw(w[slot(D + 1)], w[slot(D + 2)]);
                    const int c = K == 0 ? c0 : c1;
                    const int lc = K == 0 ? l0 : l1, lE = K == 0 ? l1 : le, lW = K == 0 ? lw : l0;
                    const T u = row[lc];
                    T v = fw.e * (u - (c + 1 < n ? row[lE] : T(0)));
                    v = fma(fw.w, u - (c > 0 ? row[lW] : T(0)), v);
                    v = fma(fw.nn, u - (rr + 1 < n ? up[lc] : T(0)), v);
                    v = fma(fw.s, u - (rr > 0 ? dn[lc] : T(0)), v);
                    return v;
                };
                const T res0 =
                    inv_h2 * ((F1 ? h2 : w[slot(D + 1)].rhs0) - flux(std::integral_constant<int, 0>{}));
                const T res1 =
                    inv_h2 * ((F1 ? h2 : w[slot(D + 1)].rhs1) - flux(std::integral_constant<int, 1>{}));
                st2(ob + (int64_t)rr * n + c0, row[l0], row[l1]);
                constexpr bool odd = ((P - D - 1) & 1) != 0;
                if constexpr (odd) fcb[L + (int64_t)nc * (rr >> 1)] = T(0.25) * (rkeep0 + rkeep1 + res0 + res1);
                else { rkeep0 = res0; rkeep1 = res1; }
            }
        } else {
            const int rr = s - D;
            if (rr >= 0 && rr < n && lane) {
                const T *row = u_ring + slot(D) * n;
                st2(ob + (int64_t)rr * n + c0, row[l0], row[l1]);
            }
        }
    };
    // steps past s_end (at most 7) find no row in range and only pass the
    // barrier, which every lane of the workgroup reaches alike
    for (int s0 = 0; s0 <= s_end; s0 += 8)
        static_for<0, 8>([&](auto Jc) __attribute__((always_inline)) { step(s0 + Jc.value, Jc); });
}

template <int MU, bool PRE, bool F1, int N, int INIT, typename T>
void launch_n(hipStream_t st, const T *a, const T *f, const T *u_in, T *u_out, const T *ec,
              int64_t Bc, T *fc, const int32_t *active)
{
    using S = StreamShape<N>;
    // once per instantiation; the static's initialisation is thread-safe
    static const bool attr_set = [] {
        (void)hipFuncSetAttribute((const void *)k_stream<MU, PRE, F1, N, INIT, T>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        return true;
    }();
    (void)attr_set;
    const size_t lds = sizeof(T) * 10 * (size_t)N * S::SPB;
    const unsigned blocks = (unsigned)((Bc + S::SPB - 1) / S::SPB);
    hipLaunchKernelGGL((k_stream<MU, PRE, F1, N, INIT, T>), dim3(blocks), dim3(S::THREADS), lds, st,
                       a, f, u_in, u_out, ec, Bc, fc, active);
}

template <int MU, bool PRE, bool F1, int N, typename T>
void launch_init(hipStream_t st, const T *a, const T *f, const T *u_in, T *u_out, const T *ec,
                 int64_t Bc, int init, T *fc, const int32_t *active)
{
    if constexpr (PRE) {
        if (init == 1) {
            launch_n<MU, PRE, F1, N, 1>(st, a, f, u_in, u_out, ec, Bc, fc, active);
            return;
        }
        if (init == 2) {
            launch_n<MU, PRE, F1, N, 2>(st, a, f, u_in, u_out, ec, Bc, fc, active);
            return;
        }
    }
    launch_n<MU, PRE, F1, N, 0>(st, a, f, u_in, u_out, ec, Bc, fc, active);
}

template <int MU, bool PRE, bool F1, typename T>
void launch_one(hipStream_t st, const T *a, const T *f, const T *u_in, T *u_out, const T *ec,
                int n, int64_t Bc, int init, T *fc, const int32_t *active)
{
    switch (n) {
    case 32: launch_init<MU, PRE, F1, 32>(st, a, f, u_in, u_out, ec, Bc, init, fc, active); break;
    case 64: launch_init<MU, PRE, F1, 64>(st, a, f, u_in, u_out, ec, Bc, init, fc, active); break;
    case 128: launch_init<MU, PRE, F1, 128>(st, a, f, u_in, u_out, ec, Bc, init, fc, active); break;
    case 256: launch_init<MU, PRE, F1, 256>(st, a, f, u_in, u_out, ec, Bc, init, fc, active); break;
    case 512: launch_init<MU, PRE, F1, 512>(st, a, f, u_in, u_out, ec, Bc, init, fc, active); break;
    case 1024: launch_init<MU, PRE, F1, 1024>(st, a, f, u_in, u_out, ec, Bc, init, fc, active); break;
    case 2048: launch_init<MU, PRE, F1, 2048>(st, a, f, u_in, u_out, ec, Bc, init, fc, active); break;
    default: break;   // stream_supported() admits only these sides
    }
}

}  // namespace

// the rings of a 2048^2 FP64 grid take 160 KiB, all of a CU's LDS
bool stream_supported(int n) { return n >= 32 && n <= 2048 && (n & (n - 1)) == 0; }

template <typename T>
void launch_pre_stream(hipStream_t st, int mu1, const T *a, const T *f, const T *u_in, T *u_out,
                       const T *uc, int n, int64_t Bc, int init, T *fc, const int32_t *active)
{
    if (mu1 == 2)
        f ? launch_one<2, true, false>(st, a, f, u_in, u_out, uc, n, Bc, init, fc, active)
          : launch_one<2, true, true>(st, a, f, u_in, u_out, uc, n, Bc, init, fc, active);
    else
        f ? launch_one<1, true, false>(st, a, f, u_in, u_out, uc, n, Bc, init, fc, active)
          : launch_one<1, true, true>(st, a, f, u_in, u_out, uc, n, Bc, init, fc, active);
}

template <typename T>
void launch_post_stream(hipStream_t st, int mu2, const T *a, const T *f, const T *u_in, T *u_out,
                        const T *ec, int n, int64_t Bc, const int32_t *active)
{
    if (mu2 == 2)
        f ? launch_one<2, false, false>(st, a, f, u_in, u_out, ec, n, Bc, 0, (T *)nullptr, active)
          : launch_one<2, false, true>(st, a, f, u_in, u_out, ec, n, Bc, 0, (T *)nullptr, active);
    else
        f ? launch_one<1, false, false>(st, a, f, u_in, u_out, ec, n, Bc, 0, (T *)nullptr, active)
          : launch_one<1, false, true>(st, a, f, u_in, u_out, ec, n, Bc, 0, (T *)nullptr, active);
}

template void launch_pre_stream<double>(hipStream_t, int, const double *, const double *,
                                        const double *, double *, const double *, int, int64_t,
                                        int, double *, const int32_t *);
template void launch_pre_stream<float>(hipStream_t, int, const float *, const float *,
                                       const float *, float *, const float *, int, int64_t, int,
                                       float *, const int32_t *);
template void launch_post_stream<double>(hipStream_t, int, const double *, const double *,
                                         const double *, double *, const double *, int, int64_t,
                                         const int32_t *);
template void launch_post_stream<float>(hipStream_t, int, const float *, const float *,
                                        const float *, float *, const float *, int, int64_t,
                                        const int32_t *);

}  // namespace mlmc
