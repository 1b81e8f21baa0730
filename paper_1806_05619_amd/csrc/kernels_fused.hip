// Fused multigrid kernels for gfx950 (Section 4: correction scheme, V-cycle,
// full multigrid), templated on the value type T of the V-cycle (double for
// the FP64 path, float for the FP32 V-cycles of the mixed-precision path).
//
// Large grids (n >= 64): temporally blocked tile passes.  One workgroup owns a
// 32 x 32 tile of one sample (256 threads; or a 16 x 16 tile with 128 threads,
// four times the workgroups for small batches) and stages the tile plus a halo
// of u and a in LDS:
//   pre pass  : mu1 red-black sweeps (red first), residual, 4-cell restriction
//               -> writes u (tile) and the coarse right-hand side;
//   post pass : bilinear prolongation of the coarse correction, mu2 sweeps
//               (black first) -> writes u (tile).
// Each half-sweep t updates the cells of its colour within a ring that shrinks
// by one cell per half-sweep, so the tile's result equals the global sweep
// order exactly.  Face weights and the inverse diagonal of every cell a thread
// updates are computed once and kept in registers for all half-sweeps.
//
// Small grids (up to 32^2; the fixed-cycle schedule uses them up to 16^2):
// one workgroup per sample keeps the whole hierarchy 2^2 .. n^2 in LDS and
// runs the FMG stages (fixed cycles, or refinement to a residual tolerance by
// flexible CG with an FP64 residual), or one V-cycle.
//
// Flexible-CG passes for larger grids: FP64 residual of the top grid from the
// FP64 coefficients and the FP64 iterate, search directions in the V-cycle
// type, per-sample reproducible two-stage reductions and the convergence flags
// of the host-driven loop.
//
// Block ids of tile passes are remapped so that consecutive tiles of a sample
// run on the same XCD (blocks are dealt round-robin over the 8 XCDs), which
// keeps the overlapping halos in that XCD's L2.
#include "internal.hpp"

namespace mlmc {
namespace {


// 1/x for the well-scaled positive values of this path (coefficients within
// e^+-15 and sums of them): hardware reciprocal estimate refined by Newton
// steps, about one ulp, without the special-case handling of IEEE division.
__device__ __forceinline__ double frcp(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}
__device__ __forceinline__ float frcp(float x)
{
    float y = __builtin_amdgcn_rcpf(x);
    float e = fmaf(-x, y, 1.0f);
    return fmaf(y, e, y);
}

// harmonic face weight 2 a_P a_N / (a_P + a_N)
template <typename T>
__device__ __forceinline__ T hm(T ap, T an) { return T(2) * ap * an * frcp(ap + an); }

__device__ __forceinline__ int xcd_remap(int bid, int nb)
{
    const int per = nb / 8;
    return bid < per * 8 ? (bid % 8) * per + bid / 8 : bid;
}

// value of the coarse grid e (nc x nc) at coarse index (I, J), odd reflection
template <typename T>
__device__ __forceinline__ T codd(const T *__restrict__ e, int nc, int I, int J)
{
    T sg = T(1);
    if (I < 0) { I = 0; sg = -sg; }
    if (I >= nc) { I = nc - 1; sg = -sg; }
    if (J < 0) { J = 0; sg = -sg; }
    if (J >= nc) { J = nc - 1; sg = -sg; }
    return sg * e[I + nc * J];
}

// Coarse values needed to prolongate onto a fine region [fi0, fi0+S)^2, staged
// in LDS with the odd wall reflection already applied (indices -1 and nc).
template <int S, int NT, typename T>
struct CoarseStage {
    static constexpr int CS = S / 2 + 3;
    __device__ static void load(T *cs, const T *__restrict__ e, int nc, int cI0, int cJ0)
    {
        for (int q = threadIdx.x; q < CS * CS; q += NT) {
            const int cj = q / CS, ci = q - cj * CS;
            const int I = cI0 + ci, J = cJ0 + cj;
            cs[q] = (I >= -1 && I <= nc && J >= -1 && J <= nc) ? codd(e, nc, I, J) : T(0);
        }
    }
    // P e at in-domain fine cell (gi, gj): (9, 3, 3, 1) / 16
    __device__ static T at(const T *cs, int cI0, int cJ0, int gi, int gj)
    {
        const int I = (gi >> 1) - cI0, J = (gj >> 1) - cJ0;
        const int sx = (gi & 1) ? 1 : -1, sy = (gj & 1) ? CS : -CS;
        const int q = I + CS * J;
        return prolong_9331(cs[q], cs[q + sx], cs[q + sy], cs[q + sx + sy]);
    }
};

// Per-cell stencil kept in registers.
template <typename T>
struct Cell {
    // LDS index l = li + S*lj in the low 16 bits, distance to the region edge
    // min(li, lj, S-1-li, S-1-lj) above; -1 if not owned / outside the grid
    int lr;
    __device__ int l() const { return lr & 0xFFFF; }
    __device__ int ring() const { return lr >> 16; }
    T wE, wW, wN, wS, inv, rhs;  // face weights (2 a_P at a wall, whose
                                 // neighbour slot holds 0), 1 / diagonal, h^2 f
};

template <int S, typename T>
__device__ __forceinline__ void make_cell(Cell<T> &c, const T *a_s, int li, int lj, int gi, int gj,
                                          int n, T rhs)
{
    // no contraction: the diagonal is the plain sum of the rounded face
    // weights, as in the row-streaming pass, whatever the compiler fuses
#pragma clang fp contract(off)
    const int l = li + S * lj;
    const T ap = a_s[l];
    const T wall = T(2) * ap;
    c.wE = gi + 1 < n ? hm(ap, a_s[l + 1]) : wall;
    c.wW = gi > 0 ? hm(ap, a_s[l - 1]) : wall;
    c.wN = gj + 1 < n ? hm(ap, a_s[l + S]) : wall;
    c.wS = gj > 0 ? hm(ap, a_s[l - S]) : wall;
    T d = c.wE;
    d += c.wW;
    d += c.wN;
    d += c.wS;
    c.inv = frcp(d);
    c.rhs = rhs;
    c.lr = l | (min(min(li, lj), min(S - 1 - li, S - 1 - lj)) << 16);
}

template <int S, typename T>
__device__ __forceinline__ void relax(const Cell<T> &c, T *u_s)
{
    const int l = c.l();
    // explicit fma, faces in the order E, W, N, S: the row-streaming pass
    // rounds identically (a wall face multiplies a neighbour slot holding 0)
    T num = fma(c.wE, u_s[l + 1], c.rhs);
    num = fma(c.wW, u_s[l - 1], num);
    num = fma(c.wN, u_s[l + S], num);
    num = fma(c.wS, u_s[l - S], num);
    u_s[l] = num * c.inv;
}

// Owned cells of one colour inside the square ring [lo, S-lo)^2 of the region.
// q-th cell: row r = q / half, column 2*(q % half) + parity.
template <int S, int NT, int LO, int COLOUR>
struct OwnSet {
    static constexpr int SIDE = S - 2 * LO;
    static constexpr int COUNT = SIDE * SIDE / 2;
    static constexpr int PER = (COUNT + NT - 1) / NT;
    __device__ static void coords(int q, int &li, int &lj)
    {
        const int half = SIDE / 2;
        const int r = q / half;
        const int cc = q - r * half;
        // colour of region cell (li, lj) = (li + lj) & 1 (tile origins are even)
        lj = LO + r;
        li = LO + 2 * cc + ((lj + LO + COLOUR) & 1);
    }
};

// Region loads: all global loads first (memory-level parallelism), then LDS.
// mode 0: u = u; 1: u = 0; 2: u = P(coarse); 3: u = u + P(coarse)
template <int S, int NT, int H, typename T>
__device__ __forceinline__ void load_region(T *a_s, T *u_s, const T *c_s, const T *ab, const T *ub,
                                            int n, int i0, int j0, int cI0, int cJ0, int mode)
{
    using CSt = CoarseStage<S, NT, T>;
    constexpr int PERT = (S * S + NT - 1) / NT;
    T av[PERT], uv[PERT];
#pragma unroll
    for (int k = 0; k < PERT; ++k) {
        const int e = threadIdx.x + NT * k;
        const int lj = e / S, li = e - lj * S;
        const int gi = i0 - H + li, gj = j0 - H + lj;
        av[k] = T(0);
        uv[k] = T(0);
        if (e < S * S && gi >= 0 && gi < n && gj >= 0 && gj < n) {
            const int64_t p = gi + (int64_t)n * gj;
            av[k] = ab[p];
            if (mode == 0) uv[k] = ub[p];
            else if (mode == 2) uv[k] = CSt::at(c_s, cI0, cJ0, gi, gj);
            else if (mode == 3) uv[k] = ub[p] + CSt::at(c_s, cI0, cJ0, gi, gj);
        }
    }
    if (mode >= 2) __syncthreads();      // c_s may share storage with a_s
#pragma unroll
    for (int k = 0; k < PERT; ++k) {
        const int e = threadIdx.x + NT * k;
        if (e < S * S) {
            a_s[e] = av[k];
            u_s[e] = uv[k];
        }
    }
    __syncthreads();
}

template <int S, int NT, int LO, int COLOUR, typename T>
__device__ __forceinline__ void make_cells(Cell<T> *cs, const T *a_s, const T *fb, int n, int i0,
                                           int j0, int H, T h2)
{
    using Own = OwnSet<S, NT, LO, COLOUR>;
#pragma unroll
    for (int k = 0; k < Own::PER; ++k) {
        const int q = threadIdx.x + NT * k;
        cs[k].lr = -1;
        if (q < Own::COUNT) {
            int li, lj;
            Own::coords(q, li, lj);
            const int gi = i0 - H + li, gj = j0 - H + lj;
            if (gi >= 0 && gi < n && gj >= 0 && gj < n)
                make_cell<S>(cs[k], a_s, li, lj, gi, gj, n, h2 * (fb ? fb[gi + (int64_t)n * gj] : T(1)));
        }
    }
}

template <int S, int PER, typename T>
__device__ __forceinline__ void sweep_ring(const Cell<T> *cs, T *u_s, int lo)
{
    // cells in the square ring [lo, S - lo)^2 of the region
#pragma unroll
    for (int k = 0; k < PER; ++k)
        if (cs[k].ring() >= lo) relax<S>(cs[k], u_s);
}

// ---------------------------------------------------------------------------
// Pre pass: mu1 red-black sweeps + residual + restriction on one tile.
// init: 0 = read u_in, 1 = zero initial guess, 2 = FMG interpolation from uc.
// The result goes to u_out, which no block of the launch reads: a tile reads
// its neighbours' cells as halo, so an in-place write would race with them.
template <int TILE, int NT, int MU, typename T>
__global__ __launch_bounds__(NT) void k_pre_tile(const T *__restrict__ a, const T *__restrict__ f,
                                                 const T *__restrict__ u_in, T *__restrict__ u_out,
                                                 const T *__restrict__ uc, int n,
                                                 int64_t Bc, int init, T *__restrict__ fc,
                                                 const int32_t *__restrict__ active)
{
    constexpr int H = 2 * MU + 1;
    constexpr int S = TILE + 2 * H;
    using Red = OwnSet<S, NT, 1, 0>;          // red cells are updated within ring H-1
    using Blk = OwnSet<S, NT, 2, 1>;          // black cells within ring H-2
    using CSt = CoarseStage<S, NT, T>;
    __shared__ T u_s[S * S];
    __shared__ T a_s[S * S];
    // the coarse values for the interpolation are read before a_s is written
    static_assert(CSt::CS * CSt::CS <= S * S, "coarse stage fits in a_s");
    T *const c_s = a_s;

    const int tiles_side = n / TILE;
    const int tps = tiles_side * tiles_side;
    const int L = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t b = L / tps;
    if (b >= Bc) return;
    if (active && !active[b]) return;
    const int tile = L - (int)(b * tps);
    const int i0 = (tile % tiles_side) * TILE, j0 = (tile / tiles_side) * TILE;
    const int64_t cells = (int64_t)n * n;
    const T *ab = a + b * cells;
    const T *ub = init == 0 ? u_in + b * cells : nullptr;
    T *ob = u_out + b * cells;
    const T *fb = f ? f + b * cells : nullptr;
    const int nc = n / 2;
    const T h2 = T(1) / (T(n) * T(n));
    const int cI0 = i0 / 2 - (H + 1) / 2 - 1, cJ0 = j0 / 2 - (H + 1) / 2 - 1;
    if (init == 2) {
        CSt::load(c_s, uc + b * (int64_t)nc * nc, nc, cI0, cJ0);
        __syncthreads();
    }
    load_region<S, NT, H>(a_s, u_s, c_s, ab, ub, n, i0, j0, cI0, cJ0, init);

    Cell<T> red[Red::PER], blk[Blk::PER];
    make_cells<S, NT, 1, 0>(red, a_s, fb, n, i0, j0, H, h2);
    make_cells<S, NT, 2, 1>(blk, a_s, fb, n, i0, j0, H, h2);
    // half-sweep t (1-based) covers ring H - t around the tile
#pragma unroll
    for (int t = 1; t <= 2 * MU; ++t) {
        if (t & 1) sweep_ring<S, Red::PER>(red, u_s, t);
        else sweep_ring<S, Blk::PER>(blk, u_s, t);
        __syncthreads();
    }
    // residual r = f - A u on the tile, into a_s (a is no longer read)
    const T inv_h2 = T(n) * T(n);
    auto resid = [&](const Cell<T> &c) {
        if (c.ring() < H) return;               // tile cells only (ring H of the region)
        const int l = c.l();
        // h^-2 (h^2 f - net flux); the flux is summed face by face as
        // w (u_P - u_nbr), a wall face giving 2 a_P u_P (its neighbour slot
        // holds 0); h^2, h^-2 are powers of two
        // explicit fma in the face order E, W, N, S: the row-streaming pre
        // pass rounds identically
        const T up = u_s[l];
        T v = c.wE * (up - u_s[l + 1]);
        v = fma(c.wW, up - u_s[l - 1], v);
        v = fma(c.wN, up - u_s[l + S], v);
        v = fma(c.wS, up - u_s[l - S], v);
        a_s[l] = inv_h2 * (c.rhs - v);
    };
#pragma unroll
    for (int k = 0; k < Red::PER; ++k)
        resid(red[k]);
#pragma unroll
    for (int k = 0; k < Blk::PER; ++k)
        resid(blk[k]);
    __syncthreads();
    // restriction (mean of the 4 children) and write-back of the tile
    constexpr int CT = TILE / 2;
    for (int e = threadIdx.x; e < CT * CT; e += NT) {
        const int J = e / CT, I = e - J * CT;
        const int l = (H + 2 * I) + S * (H + 2 * J);
        const T v = T(0.25) * (a_s[l] + a_s[l + 1] + a_s[l + S] + a_s[l + S + 1]);
        fc[b * (int64_t)nc * nc + (i0 / 2 + I) + (int64_t)nc * (j0 / 2 + J)] = v;
    }
    for (int e = threadIdx.x; e < TILE * TILE; e += NT) {
        const int lj = e / TILE, li = e - lj * TILE;
        ob[(i0 + li) + (int64_t)n * (j0 + lj)] = u_s[(H + li) + S * (H + lj)];
    }
}

// Post pass: u = u_in + P ec on the tile and its halo, then mu2 sweeps black
// first; the result goes to u_out (not read by the launch).
template <int TILE, int NT, int MU, typename T>
__global__ __launch_bounds__(NT) void k_post_tile(const T *__restrict__ a, const T *__restrict__ f,
                                                  const T *__restrict__ u_in, T *__restrict__ u_out,
                                                  const T *__restrict__ ec, int n,
                                                  int64_t Bc, const int32_t *__restrict__ active)
{
    constexpr int H = 2 * MU;
    constexpr int S = TILE + 2 * H;
    using Blk = OwnSet<S, NT, 1, 1>;          // first half-sweep (black): ring H-1
    using Red = OwnSet<S, NT, 2, 0>;          // second (red): ring H-2
    using CSt = CoarseStage<S, NT, T>;
    __shared__ T u_s[S * S];
    __shared__ T a_s[S * S];
    // the coarse correction is read before a_s is written
    static_assert(CSt::CS * CSt::CS <= S * S, "coarse stage fits in a_s");
    T *const c_s = a_s;

    const int tiles_side = n / TILE;
    const int tps = tiles_side * tiles_side;
    const int L = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t b = L / tps;
    if (b >= Bc) return;
    if (active && !active[b]) return;
    const int tile = L - (int)(b * tps);
    const int i0 = (tile % tiles_side) * TILE, j0 = (tile / tiles_side) * TILE;
    const int64_t cells = (int64_t)n * n;
    const T *ab = a + b * cells;
    const T *ub = u_in + b * cells;
    T *ob = u_out + b * cells;
    const T *fb = f ? f + b * cells : nullptr;
    const int nc = n / 2;
    const T h2 = T(1) / (T(n) * T(n));
    const int cI0 = i0 / 2 - (H + 1) / 2 - 1, cJ0 = j0 / 2 - (H + 1) / 2 - 1;
    CSt::load(c_s, ec + b * (int64_t)nc * nc, nc, cI0, cJ0);
    __syncthreads();
    load_region<S, NT, H>(a_s, u_s, c_s, ab, ub, n, i0, j0, cI0, cJ0, 3);

    Cell<T> blk[Blk::PER], red[Red::PER];
    make_cells<S, NT, 1, 1>(blk, a_s, fb, n, i0, j0, H, h2);
    make_cells<S, NT, 2, 0>(red, a_s, fb, n, i0, j0, H, h2);
#pragma unroll
    for (int t = 1; t <= 2 * MU; ++t) {
        if (t & 1) sweep_ring<S, Blk::PER>(blk, u_s, t);
        else sweep_ring<S, Red::PER>(red, u_s, t);
        __syncthreads();
    }
    for (int e = threadIdx.x; e < TILE * TILE; e += NT) {
        const int lj = e / TILE, li = e - lj * TILE;
        ob[(i0 + li) + (int64_t)n * (j0 + lj)] = u_s[(H + li) + S * (H + lj)];
    }
}

// ---------------------------------------------------------------------------
// LDS-resident hierarchy 2^2 .. 2^(GS+1) for one sample per workgroup of LT
// threads (LT is a template parameter of every routine below: one wavefront
// for grids <= 8^2, up to 256 threads for 32^2).

template <int GS>
struct LdsHier {
    static constexpr int TOTAL = (int)(4 * ((1LL << (2 * (GS + 1))) - 1) / 3);
    static __device__ constexpr int off(int g) { return (int)(4 * ((1LL << (2 * g)) - 1) / 3); }
};

// Stencil of cell (i, j) from coefficients of type TA, weights in type TW,
// rounded as in the tile passes (make_cell): a wall face carries 2 a_P (its
// neighbour reads as 0), the diagonal is the plain sum E + W + N + S.  The
// LDS-resident and the tile kernels then give the same bits on a grid that
// either may run, whichever the batch size selects.
template <typename TW, typename TA>
__device__ __forceinline__ void lds_stencil(const TA *a, int n, int i, int j, TW &wE, TW &wW,
                                            TW &wN, TW &wS, TW &d)
{
#pragma clang fp contract(off)
    const int p = i + n * j;
    const TW ap = TW(a[p]);
    const TW wall = TW(2) * ap;
    wE = i + 1 < n ? hm(ap, TW(a[p + 1])) : wall;
    wW = i > 0 ? hm(ap, TW(a[p - 1])) : wall;
    wN = j + 1 < n ? hm(ap, TW(a[p + n])) : wall;
    wS = j > 0 ? hm(ap, TW(a[p - n])) : wall;
    d = wE;
    d += wW;
    d += wN;
    d += wS;
}

template <typename T>
__device__ __forceinline__ T lds_nb(const T *u, int n, int i, int j)
{
    return (i < 0 || j < 0 || i >= n || j >= n) ? T(0) : u[i + n * j];
}

// one colour; f == nullptr means f = 1.  Explicit fma in the face order E, W,
// N, S, as in the tile passes.
template <int LT, typename T>
__device__ void lds_sweep(const T *a, const T *f, T *u, int n, int colour)
{
    const int half = n / 2;
    const T h2 = T(1) / (T(n) * T(n));
    for (int q = threadIdx.x; q < n * half; q += LT) {
        const int j = q >> (__builtin_ctz(n) - 1);          // n / 2 cells per row
        const int i = 2 * (q - j * half) + ((j + colour) & 1);
        T wE, wW, wN, wS, d;
        lds_stencil<T>(a, n, i, j, wE, wW, wN, wS, d);
        T num = h2 * (f ? f[i + n * j] : T(1));
        num = fma(wE, lds_nb(u, n, i + 1, j), num);
        num = fma(wW, lds_nb(u, n, i - 1, j), num);
        num = fma(wN, lds_nb(u, n, i, j + 1), num);
        num = fma(wS, lds_nb(u, n, i, j - 1), num);
        u[i + n * j] = num * frcp(d);
    }
    __syncthreads();
}

// r = f - A u at one cell, in the arithmetic of TU (coefficients TA promoted)
// net flux out of cell (i, j) times h^2, face by face w (u_P - u_nbr) in the
// order E, W, N, S with explicit fma, a wall face as 2 a_P (u_P - 0): the
// rounding of the tile passes.  (Their residual h^-2 (h^2 f - flux) equals
// f - h^-2 flux bit for bit: both scalings are by powers of two.)
template <typename TU, typename TA, typename TV>
__device__ __forceinline__ TU lds_flux(const TA *a, const TV *u, int n, int i, int j)
{
    // each face weight as in lds_stencil, formed where it is used; a wall
    // face's 2 a_P (u_P - 0) written as 2 a_P u_P
    const int p = i + n * j;
    const TU ap = TU(a[p]), up = TU(u[p]), wall = TU(2) * ap;
    TU v = (i + 1 < n) ? hm(ap, TU(a[p + 1])) * (up - TU(u[p + 1])) : wall * up;
    v = (i > 0) ? fma(hm(ap, TU(a[p - 1])), up - TU(u[p - 1]), v) : fma(wall, up, v);
    v = (j + 1 < n) ? fma(hm(ap, TU(a[p + n])), up - TU(u[p + n]), v) : fma(wall, up, v);
    v = (j > 0) ? fma(hm(ap, TU(a[p - n])), up - TU(u[p - n]), v) : fma(wall, up, v);
    return v;
}

template <typename TU, typename TA>
__device__ __forceinline__ TU lds_resid(const TA *a, const TU *f, const TU *u, int n, int i, int j)
{
    return (f ? f[i + n * j] : TU(1)) - TU(n) * TU(n) * lds_flux<TU>(a, u, n, i, j);
}

// Cholesky factor of h^2 A on the 2x2 grid (h^2 = 1/4), in the arithmetic of
// TU, computed by thread 0 into L[10] (row-packed lower triangle).  The
// coefficients do not change during a sample's solve, so it is factored once.
// Cells 0:(0,0) 1:(1,0) 2:(0,1) 3:(1,1).
template <typename TU, typename TA>
__device__ void lds_chol4(const TA *a, TU *L)
{
    if (threadIdx.x == 0) {
        const TU a0 = TU(a[0]), a1 = TU(a[1]), a2 = TU(a[2]), a3 = TU(a[3]);
        const TU w01 = hm(a0, a1), w02 = hm(a0, a2), w13 = hm(a1, a3), w23 = hm(a2, a3);
        const TU A[4][4] = {{w01 + w02 + TU(4) * a0, -w01, -w02, TU(0)},
                            {-w01, w01 + w13 + TU(4) * a1, TU(0), -w13},
                            {-w02, TU(0), w02 + w23 + TU(4) * a2, -w23},
                            {TU(0), -w13, -w23, w13 + w23 + TU(4) * a3}};
        TU l[4][4] = {};
        for (int p = 0; p < 4; ++p)
            for (int q = 0; q <= p; ++q) {
                TU s = A[p][q];
                for (int k = 0; k < q; ++k) s -= l[p][k] * l[q][k];
                l[p][q] = (p == q) ? sqrt(s) : s / l[q][q];
            }
        int k = 0;
        for (int p = 0; p < 4; ++p)
            for (int q = 0; q <= p; ++q) L[k++] = l[p][q];
    }
}

// exact 2x2 solve A u = f (f nullptr: f = 1) with the factor of lds_chol4
template <typename TU>
__device__ void lds_coarse_solve(const TU *L, const TU *f, TU *u)
{
    if (threadIdx.x == 0) {
        // row p of the packed factor starts at p (p + 1) / 2
        TU v[4];
        for (int p = 0; p < 4; ++p) {
            const TU *lp = L + p * (p + 1) / 2;
            TU s = TU(0.25) * (f ? f[p] : TU(1));
            for (int q = 0; q < p; ++q) s -= lp[q] * v[q];
            v[p] = s / lp[p];
        }
        for (int p = 3; p >= 0; --p) {
            TU s = v[p];
            for (int q = p + 1; q < 4; ++q) s -= L[q * (q + 1) / 2 + p] * v[q];
            v[p] = s / L[p * (p + 1) / 2 + p];
        }
        for (int p = 0; p < 4; ++p) u[p] = v[p];
    }
    __syncthreads();
}

// u = P e (add = false) or u += P e on the n x n grid
template <int LT, typename T>
__device__ void lds_prolong(const T *e, T *u, int n, bool add)
{
    const int nc = n / 2;
    for (int p = threadIdx.x; p < n * n; p += LT) {
        const int j = p >> __builtin_ctz(n), i = p & (n - 1);   // n is a power of two
        const int I = i >> 1, J = j >> 1, sx = (i & 1) ? 1 : -1, sy = (j & 1) ? 1 : -1;
        const T v = prolong_9331(codd(e, nc, I, J), codd(e, nc, I + sx, J), codd(e, nc, I, J + sy),
                                 codd(e, nc, I + sx, J + sy));
        u[p] = add ? u[p] + v : v;
    }
    __syncthreads();
}

template <int GS, typename T, int LT>
struct LdsVcycle {
    T *a, *u, *f;   // LDS bases, level g at LdsHier<GS>::off(g)
    const T *chol;  // Cholesky factor of the 2x2 grid (lds_chol4), in LDS
    int mu1, mu2;
    // V(mu1,mu2) at level g (one coarse-grid correction per level, so the
    // recursion unrolls into a descent and an ascent).  The top right-hand
    // side may be nullptr (f = 1); the coarser ones live in LDS.
    __device__ void run(int g, const T *ftop)
    {
        for (int l = g; l >= 1; --l) {
            const int n = 2 << l, nc = n / 2;
            T *al = a + LdsHier<GS>::off(l), *ul = u + LdsHier<GS>::off(l);
            const T *fl = (l == g) ? ftop : f + LdsHier<GS>::off(l);
            for (int it = 0; it < mu1; ++it) {
                lds_sweep<LT>(al, fl, ul, n, 0);
                lds_sweep<LT>(al, fl, ul, n, 1);
            }
            T *fcl = f + LdsHier<GS>::off(l - 1), *ucl = u + LdsHier<GS>::off(l - 1);
            for (int q = threadIdx.x; q < nc * nc; q += LT) {
                const int J = q >> __builtin_ctz(nc), I = q & (nc - 1);
                const T r00 = lds_resid<T>(al, fl, ul, n, 2 * I, 2 * J);
                const T r10 = lds_resid<T>(al, fl, ul, n, 2 * I + 1, 2 * J);
                const T r01 = lds_resid<T>(al, fl, ul, n, 2 * I, 2 * J + 1);
                const T r11 = lds_resid<T>(al, fl, ul, n, 2 * I + 1, 2 * J + 1);
                fcl[q] = T(0.25) * (r00 + r10 + r01 + r11);
                ucl[q] = T(0);
            }
            __syncthreads();
        }
        lds_coarse_solve<T>(chol, g == 0 ? ftop : f, u);
        for (int l = 1; l <= g; ++l) {
            const int n = 2 << l;
            T *al = a + LdsHier<GS>::off(l), *ul = u + LdsHier<GS>::off(l);
            const T *fl = (l == g) ? ftop : f + LdsHier<GS>::off(l);
            lds_prolong<LT>(u + LdsHier<GS>::off(l - 1), ul, n, true);
            for (int it = 0; it < mu2; ++it) {
                lds_sweep<LT>(al, fl, ul, n, 1);
                lds_sweep<LT>(al, fl, ul, n, 0);
            }
        }
    }
};

__device__ __forceinline__ void neumaier(double &s, double &c, double x)
{
    const double t = s + x;
    if (fabs(s) >= fabs(x)) c += (s - t) + x; else c += (x - t) + s;
    s = t;
}

// (s, c) += (s2, c2) for compensated pairs (TwoSum of the leading parts)
__device__ __forceinline__ void two_sum_fold(double &s, double &c, double s2, double c2)
{
    const double t = s + s2, bb = t - s;
    c = c + c2 + ((s - (t - bb)) + (s2 - bb));
    s = t;
}

// Deterministic block reduction of NV per-thread compensated partial sums:
// a butterfly inside each wavefront, then every thread folds the wavefront
// totals in wavefront order (scratch: 2 NV doubles per wavefront).  Returns
// the totals in every thread.
template <int LT, int NV>
__device__ __forceinline__ void lds_reduce_n(double *s, double *c, double *scratch, double *v)
{
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1)
            two_sum_fold(s[k], c[k], __shfl_xor(s[k], m, 64), __shfl_xor(c[k], m, 64));
    if constexpr (LT == 64) {
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] = s[k] + c[k];
        return;
    }
    constexpr int NW = LT / 64;
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            scratch[(wave * NV + k) * 2] = s[k];
            scratch[(wave * NV + k) * 2 + 1] = c[k];
        }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double S = scratch[k * 2], C = scratch[k * 2 + 1];
#pragma unroll
        for (int w = 1; w < NW; ++w) two_sum_fold(S, C, scratch[(w * NV + k) * 2], scratch[(w * NV + k) * 2 + 1]);
        v[k] = S + C;
    }
    __syncthreads();
}

template <int LT>
__device__ __forceinline__ double lds_reduce(double s, double c, double *scratch)
{
    double v;
    lds_reduce_n<LT, 1>(&s, &c, scratch, &v);
    return v;
}

// QoI of one sample's grid ug in LDS, summed in the order of the QoI kernel
// of the larger grids (k_qoi: lane k of one wavefront adds cells k, k + 64,
// ... compensated, then a butterfly), so a grid gives the same bits in either
// kernel.  Ends with a barrier: the grid may be overwritten next.
template <int LT>
__device__ void lds_write_qoi(const double *ug, int n, double *qoi, int64_t b, int nlev, int l,
                              uint32_t mask)
{
    if (threadIdx.x < 64) {
        const int nq = (mask & 1u ? 1 : 0) + (mask & 2u ? 1 : 0);
        double qm = 0.0;
        if (mask & 1u) {
            double s = 0.0, c = 0.0;
            for (int p = threadIdx.x; p < n * n; p += 64) neumaier(s, c, ug[p]);
#pragma unroll
            for (int m = 32; m >= 1; m >>= 1)
                two_sum_fold(s, c, __shfl_xor(s, m, 64), __shfl_xor(c, m, 64));
            qm = (s + c) / ((double)n * n);
        }
        if (threadIdx.x == 0) {
            double *qb = qoi + (b * nlev + l) * nq;
            int q = 0;
            if (mask & 1u) qb[q++] = qm;
            if (mask & 2u) {
                const int c = n / 2;
                qb[q] = 0.25 * (ug[(c - 1) + n * (c - 1)] + ug[c + n * (c - 1)] +
                                ug[(c - 1) + n * c] + ug[c + n * c]);
            }
        }
    }
    __syncthreads();
}

// FMG stages 0..G (G <= GS) with fixed mu0 cycles, FP64; QoI of stages g >= g0;
// final u of level G to the u pool.
template <int GS, int LT>
__global__ __launch_bounds__(LT) void k_lds_fmg_fixed(const double *__restrict__ a_pool,
                                                      double *__restrict__ u_pool, int64_t Bc,
                                                      int G, int mu0, int mu1, int mu2, int g0,
                                                      double *__restrict__ qoi, int nlev,
                                                      uint32_t mask)
{
    constexpr int TOT = LdsHier<GS>::TOTAL;
    __shared__ double a_s[TOT], u_s[TOT], f_s[TOT];
    __shared__ double chol_s[10];
    const int64_t b = blockIdx.x;
    if (b >= Bc) return;
    for (int g = 0; g <= G; ++g) {
        const int cnt = 4 << (2 * g);
        const double *src = a_pool + Bc * level_offset(g) + b * (int64_t)cnt;
        for (int p = threadIdx.x; p < cnt; p += LT) a_s[LdsHier<GS>::off(g) + p] = src[p];
    }
    __syncthreads();
    lds_chol4<double>(a_s, chol_s);
    __syncthreads();
    LdsVcycle<GS, double, LT> V{a_s, u_s, f_s, chol_s, mu1, mu2};
    for (int g = 0; g <= G; ++g) {
        const int n = 2 << g;
        double *ug = u_s + LdsHier<GS>::off(g);
        if (g == 0) {
            V.run(0, nullptr);
        } else {
            lds_prolong<LT>(u_s + LdsHier<GS>::off(g - 1), ug, n, false);
            for (int c = 0; c < mu0; ++c) V.run(g, nullptr);
        }
        if (g >= g0) lds_write_qoi<LT>(ug, n, qoi, b, nlev, g - g0, mask);
    }
    const int cntG = 4 << (2 * G);
    double *dst = u_pool + Bc * level_offset(G) + b * (int64_t)cntG;
    for (int p = threadIdx.x; p < cntG; p += LT) dst[p] = u_s[LdsHier<GS>::off(G) + p];
}

// One V-cycle at level G (<= GS) with zero initial guess, f from the f pool,
// correction to the u pool.
template <int GS, typename T, int LT>
__global__ __launch_bounds__(LT) void k_lds_vcycle(const T *__restrict__ a_pool,
                                                   const T *__restrict__ f_pool, T *__restrict__ u_pool,
                                                   int64_t Bc, int G, int mu1, int mu2,
                                                   const int32_t *__restrict__ active)
{
    constexpr int TOT = LdsHier<GS>::TOTAL;
    __shared__ T a_s[TOT], u_s[TOT], f_s[TOT], chol_s[10];
    const int64_t b = blockIdx.x;
    if (b >= Bc) return;
    if (active && !active[b]) return;
    for (int g = 0; g <= G; ++g) {
        const int cnt = 4 << (2 * g);
        const T *src = a_pool + Bc * level_offset(g) + b * (int64_t)cnt;
        for (int p = threadIdx.x; p < cnt; p += LT) a_s[LdsHier<GS>::off(g) + p] = src[p];
    }
    const int cntG = 4 << (2 * G);
    const T *fsrc = f_pool + Bc * level_offset(G) + b * (int64_t)cntG;
    for (int p = threadIdx.x; p < cntG; p += LT) {
        f_s[LdsHier<GS>::off(G) + p] = fsrc[p];
        u_s[LdsHier<GS>::off(G) + p] = T(0);
    }
    __syncthreads();
    lds_chol4<T>(a_s, chol_s);
    __syncthreads();
    LdsVcycle<GS, T, LT> V{a_s, u_s, f_s, chol_s, mu1, mu2};
    V.run(G, f_s + LdsHier<GS>::off(G));
    T *dst = u_pool + Bc * level_offset(G) + b * (int64_t)cntG;
    for (int p = threadIdx.x; p < cntG; p += LT) dst[p] = u_s[LdsHier<GS>::off(G) + p];
}

// Two compensated partial sums reduced together.
template <int LT>
__device__ __forceinline__ void lds_reduce2(double s0, double c0, double s1, double c1,
                                            double *scratch, double &v0, double &v1)
{
    double s[2] = {s0, s1}, c[2] = {c0, c1}, v[2];
    lds_reduce_n<LT, 2>(s, c, scratch, v);
    v0 = v[0];
    v1 = v[1];
}

// (A u)_P in FP64 at cell (i, j) of the n x n grid, coefficients TA promoted
template <typename TA, typename TV>
__device__ __forceinline__ double lds_apply(const TA *a, const TV *u, int n, int i, int j)
{
    return double(n) * double(n) * lds_flux<double>(a, u, n, i, j);
}

// FMG stages 0..G (G <= GS) with every stage g >= 1 solved to
// ||1 - A x||_2 / ||1||_2 <= rtol by flexible preconditioned CG in FP64 from
// the interpolated x = P x_prev, the preconditioner z = B r being one
// V(mu1, mu2) cycle in T from a zero guess:
//   z = B r;  beta = (z, r - r_old) / (z_old, r_old)  (0 at the first step);
//   p = z + beta p;  alpha = (z, r) / (p, A p);  x += alpha p;  r = 1 - A x.
// QoI of stages g >= g0 from x; x of level G to u64_pool; per sample the
// largest step count, the largest final relative residual and whether a stage
// stopped at max_iters.
template <int GS, typename T, int LT>
__global__ __launch_bounds__(LT, LT == 64 ? 4 : 1) void k_lds_fmg_refine(
    const T *__restrict__ a_pool, const double *__restrict__ a64_pool,
    double *__restrict__ u64_pool, int64_t Bc, int G, int mu1, int mu2, double rtol, int max_iters,
    int g0, double *__restrict__ qoi, int nlev, uint32_t mask, int32_t *__restrict__ st_iters,
    double *__restrict__ st_rho, int32_t *__restrict__ st_bad)
{
    constexpr int TOT = LdsHier<GS>::TOTAL;
    constexpr int TOP = 4 << (2 * GS);   // cells of the finest LDS level
    constexpr bool F64 = sizeof(T) == sizeof(double);
    constexpr int RPT = (TOP + LT - 1) / LT;   // top-level cells per thread
    __shared__ T a_s[TOT], u_s[TOT], f_s[TOT], chol_s[10];
    // FP64 coefficients of the current stage's CG operator (the FP64 context
    // uses a_s itself)
    __shared__ double a64_s[F64 ? 1 : TOP];
    __shared__ double w_s[TOT];          // FP64 stage solutions x
    __shared__ T p_s[TOP];               // search direction, in the V-cycle type
    __shared__ double red_s[4 * (LT / 64)], chol64_s[10];
    double r_v[RPT], ro_v[RPT];          // r and r_old of this thread's cells p = tid + LT q
    const int64_t b = blockIdx.x;
    if (b >= Bc) return;
    for (int g = 0; g <= G; ++g) {
        const int cnt = 4 << (2 * g);
        const int64_t o = Bc * level_offset(g) + b * (int64_t)cnt;
        for (int p = threadIdx.x; p < cnt; p += LT) a_s[LdsHier<GS>::off(g) + p] = a_pool[o + p];
    }
    if (!F64 && threadIdx.x < 4) a64_s[threadIdx.x] = a64_pool[b * 4 + threadIdx.x];
    __syncthreads();
    lds_chol4<T>(a_s, chol_s);
    lds_chol4<double>(F64 ? (const double *)a_s : a64_s, chol64_s);
    __syncthreads();
    LdsVcycle<GS, T, LT> V{a_s, u_s, f_s, chol_s, mu1, mu2};
    int it_max = 0, bad = 0;
    double rho_max = 0.0;
    for (int g = 0; g <= G; ++g) {
        const int n = 2 << g, cells = n * n;
        double *xg = w_s + LdsHier<GS>::off(g);
        T *zg = u_s + LdsHier<GS>::off(g), *fg = f_s + LdsHier<GS>::off(g);
        if (!F64 && g > 0) {
            const int64_t o = Bc * level_offset(g) + b * (int64_t)cells;
            __syncthreads();             // the previous stage's operator is no longer read
            for (int p = threadIdx.x; p < cells; p += LT) a64_s[p] = a64_pool[o + p];
        }
        const double *ag = F64 ? (const double *)a_s + LdsHier<GS>::off(g) : a64_s;
        if (g == 0) lds_coarse_solve<double>(chol64_s, (const double *)nullptr, xg);
        else lds_prolong<LT>(w_s + LdsHier<GS>::off(g - 1), xg, n, false);
        int it = 0;
        double rho, rz_old = 1.0;
        double best = 0.0;                        // smallest rho of a 10% improvement
        int since = 0;                            // steps since then
        for (;;) {
            // r = 1 - A x, staged as the T right-hand side of the preconditioner
            double s = 0.0, c = 0.0;
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int p = threadIdx.x + LT * q;
                if (p < cells) {
                    const int j = p >> __builtin_ctz(n), i = p & (n - 1);
                    const double r = 1.0 - lds_apply(ag, xg, n, i, j);
                    r_v[q] = r;
                    fg[p] = T(r);
                    zg[p] = T(0);
                    neumaier(s, c, r * r);
                }
            }
            rho = sqrt(lds_reduce<LT>(s, c, red_s)) / (double)n;   // ||1||_2 = n
            // attainable accuracy: stop once four steps in a row have not
            // brought rho 10% below the best value so far
            if (it == 0 || rho < 0.9 * best) {
                best = rho;
                since = 0;
            } else {
                ++since;
            }
            const bool stalled = since >= 4;
            if (rho <= rtol || it >= max_iters || g == 0 || stalled) break;
            V.run(g, fg);                                       // z = B r
            double s0 = 0.0, c0 = 0.0, s1 = 0.0, c1 = 0.0;
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int p = threadIdx.x + LT * q;
                if (p < cells) {
                    const double z = double(zg[p]);
                    neumaier(s0, c0, r_v[q] * z);
                    neumaier(s1, c1, it == 0 ? 0.0 : ro_v[q] * z);
                    ro_v[q] = r_v[q];
                }
            }
            double rz, rzo;
            lds_reduce2<LT>(s0, c0, s1, c1, red_s, rz, rzo);
            const double beta = it == 0 ? 0.0 : (rz - rzo) / rz_old;
            for (int p = threadIdx.x; p < cells; p += LT)
                p_s[p] = T(it == 0 ? double(zg[p]) : double(zg[p]) + beta * double(p_s[p]));
            __syncthreads();
            s = 0.0;
            c = 0.0;
            for (int p = threadIdx.x; p < cells; p += LT) {
                const int j = p >> __builtin_ctz(n), i = p & (n - 1);
                neumaier(s, c, double(p_s[p]) * lds_apply(ag, p_s, n, i, j));
            }
            const double alpha = rz / lds_reduce<LT>(s, c, red_s);
            for (int p = threadIdx.x; p < cells; p += LT) xg[p] += alpha * double(p_s[p]);
            __syncthreads();
            rz_old = rz;
            ++it;
        }
        if (g > 0 && rho > rtol) bad = 1;
        it_max = it > it_max ? it : it_max;
        rho_max = rho > rho_max ? rho : rho_max;
        if (g >= g0) lds_write_qoi<LT>(xg, n, qoi, b, nlev, g - g0, mask);
    }
    const int cntG = 4 << (2 * G);
    double *dst = u64_pool + Bc * level_offset(G) + b * (int64_t)cntG;
    for (int p = threadIdx.x; p < cntG; p += LT) dst[p] = w_s[LdsHier<GS>::off(G) + p];
    if (threadIdx.x == 0) {
        st_iters[b] = it_max;
        st_rho[b] = rho_max;
        st_bad[b] = bad;
    }
}

// ---------------------------------------------------------------------------
// Flexible CG of one FMG stage on a large grid (the same iteration as the
// LDS-resident kernel above), one pass per vector operation over all active
// samples.  Geometry (grids n >= 64): a thread owns CW consecutive cells of a
// row, CW = 16 bytes over the widest element type the pass moves (2 for
// FP64 arrays, 4 for FP32), so that each lane of a wavefront loads and stores
// 16 contiguous bytes per array and row; it marches along the QH = 4 q / CW
// rows of its strip (q = 4 on 64^2, 8 above; upwards, or downwards for odd
// strips, see strip_march).  The 256 threads of a block
// take 256 consecutive cell groups of the sample's strip space (group g:
// strip g / (n/CW), columns CW (g mod n/CW) .. +CW-1), so every pass covers
// 1024 q cells per block and n^2 / (1024 q) blocks per sample.  A stencil
// pass keeps the rows above and below in registers as it marches (the row
// two ahead in flight), takes the horizontal neighbours from the adjacent
// lanes (a global load only at the two ends of a wavefront), and forms each
// harmonic face weight once (an E face is the next cell's W face, an N face
// the next row's S face: the same bits, hm being symmetric).  Every block
// leaves one compensated partial sum (or two); a wavefront per sample folds
// the partials in block order, so every sum is reproducible and a sample's
// result does not depend on its batch.
__host__ __device__ inline int fcg_q(int n) { return n >= 128 ? 8 : 4; }
__host__ __device__ inline int fcg_nch(int n) { return (int)((int64_t)n * n / (1024 * fcg_q(n))); }

struct FcgMap {
    int64_t b;       // sample
    int blk;         // block of the sample (partial-sum index)
    int nch;         // blocks per sample
    int i0, j0;      // first column and first row of the thread's strip
};
// Blocks go through xcd_contiguous, so that the strips above and below a
// block's rows (the stencil's neighbours) are read by blocks of the same XCD.

template <int CW, int QH>
__device__ __forceinline__ bool fcg_map(int n, int64_t Bc, const int32_t *active, FcgMap &m)
{
    m.nch = fcg_nch(n);
    const int64_t L = xcd_contiguous(blockIdx.x, gridDim.x);
    m.b = L / m.nch;
    m.blk = (int)(L - m.b * m.nch);
    if (m.b >= Bc) return false;
    const int W = n / CW;                                  // cell groups per row
    const int64_t g = (int64_t)m.blk * 256 + threadIdx.x;  // group of the strip space
    m.j0 = (int)(g / W) * QH;
    m.i0 = (int)(g % W) * CW;
    return !active || active[m.b];
}

// CW consecutive elements as 16 bytes (or 8 for two floats)
template <int CW, typename T>
__device__ __forceinline__ void ldv(const T *__restrict__ p, T (&v)[CW])
{
    if constexpr (sizeof(T) == 4 && CW == 4) {
        const float4 t = *(const float4 *)p;
        v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
    } else if constexpr (sizeof(T) == 4 && CW == 2) {
        const float2 t = *(const float2 *)p;
        v[0] = t.x; v[1] = t.y;
    } else {
        static_assert(sizeof(T) == 8 && CW == 2, "FP64 cell groups are pairs");
        const double2 t = *(const double2 *)p;
        v[0] = t.x; v[1] = t.y;
    }
}
template <int CW, typename T>
__device__ __forceinline__ void stv(T *__restrict__ p, const T (&v)[CW])
{
    if constexpr (sizeof(T) == 4 && CW == 4) {
        *(float4 *)p = make_float4(v[0], v[1], v[2], v[3]);
    } else if constexpr (sizeof(T) == 4 && CW == 2) {
        *(float2 *)p = make_float2(v[0], v[1]);
    } else {
        static_assert(sizeof(T) == 8 && CW == 2, "FP64 cell groups are pairs");
        *(double2 *)p = make_double2(v[0], v[1]);
    }
}

// One row of a thread's cell group in a stencil pass: the coefficient (TA)
// and the vector the operator is applied to (TV), formed from the stored
// arrays (the iterate x + alpha p, or z + beta p).
template <typename TA, typename TV, int CW>
struct GroupRow {
    TA a[CW];
    TV v[CW];
};

// left/right neighbours (cells i0-1 and i0+CW) of the group row held by the
// lanes of a wavefront; lanes at the wavefront's ends load them
template <int CW, typename TA, typename TV, typename Get>
__device__ __forceinline__ void row_ends(const GroupRow<TA, TV, CW> &q, const TA *__restrict__ arow,
                                         int64_t rowoff, int i0, int n, Get get, TA &al, TV &vl,
                                         TA &ar, TV &vr)
{
    const int lane = threadIdx.x & 63;
    al = __shfl_up(q.a[CW - 1], 1, 64);
    vl = __shfl_up(q.v[CW - 1], 1, 64);
    ar = __shfl_down(q.a[0], 1, 64);
    vr = __shfl_down(q.v[0], 1, 64);
    if (lane == 0 && i0 > 0) {
        al = arow[i0 - 1];
        vl = get(rowoff + i0 - 1);
    }
    if (lane == 63 && i0 + CW < n) {
        ar = arow[i0 + CW];
        vr = get(rowoff + i0 + CW);
    }
}

// Net flux h^2 (A v)_P of the cells of a group row, faces summed in the
// order E, W, N, S (walls: 2 a_P v_P), as TS.  A strip marched upwards
// carries the S face weights from the row below and forms the N ones, which
// it returns in `fresh` (the next row's S faces); a strip marched downwards
// (down) carries the N faces and forms the S ones.  Either way each cell sees
// the same face weights (hm is symmetric) and the same sum.
// (the rows above and below are passed by reference with flags, never as
// pointers that may be null: a select between the addresses of two register
// arrays would force them into scratch memory)
template <typename TS, int CW, typename TA, typename TV>
__device__ __forceinline__ void row_flux(const GroupRow<TA, TV, CW> &c, TA al, TV vl, TA ar, TV vr,
                                         const GroupRow<TA, TV, CW> &up, bool has_up,
                                         const GroupRow<TA, TV, CW> &dn, bool has_dn, bool down,
                                         const TS (&carried)[CW], TS (&fresh)[CW], int i0, int n,
                                         TS (&flux)[CW])
{
    TS hx[CW + 1];   // faces between columns i0-1 | i0 | .. | i0+CW
    hx[0] = i0 > 0 ? hm(TS(al), TS(c.a[0])) : TS(0);
#pragma unroll
    for (int k = 1; k < CW; ++k) hx[k] = hm(TS(c.a[k - 1]), TS(c.a[k]));
    hx[CW] = i0 + CW < n ? hm(TS(c.a[CW - 1]), TS(ar)) : TS(0);
    const bool has_nb = down ? has_dn : has_up;
#pragma unroll
    for (int k = 0; k < CW; ++k) {
        const TS ap = TS(c.a[k]), xp = TS(c.v[k]);
        const TS xe = k < CW - 1 ? TS(c.v[k + 1]) : TS(vr);
        const TS xw = k > 0 ? TS(c.v[k - 1]) : TS(vl);
        const TS anb = TS(down ? dn.a[k] : up.a[k]);
        fresh[k] = has_nb ? hm(ap, anb) : TS(0);
        const TS fN = down ? carried[k] : fresh[k], fS = down ? fresh[k] : carried[k];
        TS v = TS(0);
        v += (i0 + k + 1 < n) ? hx[k + 1] * (xp - xe) : TS(2) * ap * xp;
        v += (i0 + k > 0) ? hx[k] * (xp - xw) : TS(2) * ap * xp;
        v += has_up ? fN * (xp - TS(up.v[k])) : TS(2) * ap * xp;
        v += has_dn ? fS * (xp - TS(dn.v[k])) : TS(2) * ap * xp;
        flux[k] = v;
    }
}

// the rows of a pass, moved as values (a select between two register arrays'
// addresses would put them in scratch memory)
template <typename TA, typename TV, int CW>
__device__ __forceinline__ void row_pick(GroupRow<TA, TV, CW> &dst, bool take,
                                         const GroupRow<TA, TV, CW> &src)
{
#pragma unroll
    for (int k = 0; k < CW; ++k) {
        dst.a[k] = take ? src.a[k] : dst.a[k];
        dst.v[k] = take ? src.v[k] : dst.v[k];
    }
}

// The rows of a thread's strip in marching order: strips whose index is odd
// march downwards when a wavefront's lanes share one strip, so that the two
// rows on either side of a strip boundary are read by both strips at the same
// end of their marches, close together in time (the second read hits the
// L2; with every strip marching upwards, a boundary row is read at the start
// of one march and at the end of the other, after the XCD has streamed far
// more than its L2 holds).  `load(j, row)` fills row j; `body(j, cur, up, dn,
// carried, fresh)` handles row j with the rows above and below it.  The row
// two ahead is in flight while a row is handled.
template <int QH, typename TS, int CW, typename Row, typename Load, typename Body>
__device__ __forceinline__ void strip_march(bool down, int j0, int n, Load load, Body body)
{
    const int d = down ? -1 : 1;
    const int js = down ? j0 + QH - 1 : j0;
    Row up, cur, dn, nn;              // rows j+1, j, j-1 and the one two ahead
    TS carried[CW], fresh[CW];
    load(js, cur);
    if (js + 1 < n) load(js + 1, up);
    if (js > 0) load(js - 1, dn);
    // the face to the row behind in marching order
    const bool has_bhd = down ? js + 1 < n : js > 0;
#pragma unroll
    for (int q = 0; q < CW; ++q)
        carried[q] = has_bhd ? hm(TS(cur.a[q]), TS(down ? up.a[q] : dn.a[q])) : TS(0);
#pragma unroll 1
    for (int t = 0; t < QH; ++t) {
        const int j = js + d * t;
        if (t + 1 < QH && j + 2 * d >= 0 && j + 2 * d < n) load(j + 2 * d, nn);
        body(j, cur, up, dn, carried, fresh);
#pragma unroll
        for (int q = 0; q < CW; ++q) carried[q] = fresh[q];
        // upwards: dn <- cur, cur <- up, up <- nn; downwards: up <- cur,
        // cur <- dn, dn <- nn
        Row nc = up;
        row_pick(nc, down, dn);
        row_pick(dn, !down, cur);
        row_pick(up, down, cur);
        row_pick(dn, down, nn);
        row_pick(up, !down, nn);
        cur = nc;
    }
}

__device__ __forceinline__ bool strip_down(int n, int CW, int j0, int QH)
{
    return n / CW >= 64 && ((j0 / QH) & 1);
}

// block (256 threads) compensated sums of NV values -> out[2 NV] (sum, comp)
template <int NV>
__device__ __forceinline__ void block_partials(double *s, double *c, double *out)
{
    __shared__ double red[4][2 * NV];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1)
            two_sum_fold(s[v], c[v], __shfl_xor(s[v], m, 64), __shfl_xor(c[v], m, 64));
    if (lane == 0)
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            red[wave][2 * v] = s[v];
            red[wave][2 * v + 1] = c[v];
        }
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            double S = red[0][2 * v], Cc = red[0][2 * v + 1];
            for (int w = 1; w < 4; ++w) two_sum_fold(S, Cc, red[w][2 * v], red[w][2 * v + 1]);
            out[2 * v] = S;
            out[2 * v + 1] = Cc;
        }
}

// fold the per-block partials of sample b (one wavefront): value v of NV
template <int NV>
__device__ __forceinline__ double fold_partials(const double *__restrict__ part, int64_t b, int nch,
                                                int v)
{
    const int lane = threadIdx.x & 63;
    double s = 0.0, c = 0.0;
    for (int k = lane; k < nch; k += 64) {
        const double *q = part + ((b * nch + k) * NV + v) * 2;
        two_sum_fold(s, c, q[0], q[1]);
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) two_sum_fold(s, c, __shfl_xor(s, m, 64), __shfl_xor(c, m, 64));
    return s + c;
}

// Step k >= 1 of a stage (iters[b] = k while it runs; every active sample of
// a chunk is at the same step).  The residual lives only as T(r), in two
// buffers: r_k in F[k & 1] (F[0] = f, the stage's right-hand-side pool, holds
// r_0), so the preconditioner of step k reads F[(k-1) & 1] and r_{k-2} is
// still in F[k & 1] when the inner products of step k need it.  The search
// direction p is T in two buffers (p_k written from p_{k-1}), the iterate x
// FP64 in two buffers (x_k in X[k & 1], X[0] being the stage solution pool).
// Inner products and step lengths see T-rounded r and p; the residual that
// decides convergence is recomputed from x in FP64 with the FP64
// coefficients.

// x_k = x_{k-1} + alpha p_k into X[k & 1] and r = 1 - A x_k in FP64 (UPDATE),
// or r = 1 - A x_0 (the stage's first residual, from X[0]); F[k & 1] = T(r),
// partial ||r||^2.  FP64 arrays: cell pairs.
template <typename T, int QH, bool UPDATE>
__global__ __launch_bounds__(256, 4) void k_fcg_x(const double *__restrict__ a64, double *__restrict__ X0,
                                                  double *__restrict__ X1, const T *__restrict__ P0,
                                                  const T *__restrict__ P1, T *__restrict__ F0,
                                                  T *__restrict__ F1, int n, int64_t Bc,
                                                  const double *__restrict__ fs,
                                                  double *__restrict__ part,
                                                  const int32_t *__restrict__ active,
                                                  const int32_t *__restrict__ iters)
{
    constexpr int CW = 2;
    FcgMap m;
    if (!fcg_map<CW, QH>(n, Bc, UPDATE ? active : nullptr, m)) return;
    const int64_t cells = (int64_t)n * n, base = m.b * cells;
    const int k = UPDATE ? iters[m.b] : 0;
    const double alpha = UPDATE ? fs[4 * m.b + 2] : 0.0;
    const double *ab = a64 + base;
    const double *xold = (UPDATE && ((k - 1) & 1) ? X1 : X0) + base;
    double *xnew = (k & 1 ? X1 : X0) + base;
    const T *pb = UPDATE ? (k & 1 ? P1 : P0) + base : nullptr;
    T *fb = (k & 1 ? F1 : F0) + base;
    auto xk = [&](int64_t q) { return UPDATE ? xold[q] + alpha * double(pb[q]) : xold[q]; };
    using Row = GroupRow<double, double, CW>;
    auto load = [&](int j, Row &r) {
        const int64_t o = (int64_t)j * n + m.i0;
        ldv<CW>(ab + o, r.a);
        ldv<CW>(xold + o, r.v);
        if (UPDATE) {
            T pp[CW];
            ldv<CW>(pb + o, pp);
#pragma unroll
            for (int c = 0; c < CW; ++c) r.v[c] = r.v[c] + alpha * double(pp[c]);
        }
    };
    const double n2 = double(n) * double(n);
    const bool down = strip_down(n, CW, m.j0, QH);
    double s[1] = {0.0}, c[1] = {0.0};
    auto body = [&](int j, const Row &cur, const Row &up, const Row &dn,
                    const double (&carried)[CW], double (&fresh)[CW]) {
        double al, vl, ar, vr;
        row_ends<CW>(cur, ab + (int64_t)j * n, (int64_t)j * n, m.i0, n, xk, al, vl, ar, vr);
        double flux[CW];
        row_flux<double, CW>(cur, al, vl, ar, vr, up, j + 1 < n, dn, j > 0, down, carried, fresh,
                             m.i0, n, flux);
        T fv[CW];
#pragma unroll
        for (int q = 0; q < CW; ++q) {
            const double r = 1.0 - n2 * flux[q];
            fv[q] = T(r);
            neumaier(s[0], c[0], r * r);
        }
        const int64_t o = (int64_t)j * n + m.i0;
        if (UPDATE) stv<CW>(xnew + o, cur.v);
        stv<CW>(fb + o, fv);
    };
    strip_march<QH, double, CW, Row>(down, m.j0, n, load, body);
    block_partials<1>(s, c, part + (m.b * m.nch + m.blk) * 2);
}

// rho_b = ||r|| / ||1||.  first: every sample starts with iters = 0.  Then,
// for the samples still iterating: active = rho > rtol && iters < max_iters,
// and iters becomes the number of the step about to be taken.
__global__ __launch_bounds__(256) void k_fcg_fin_rho(const double *__restrict__ part, int n,
                                                     int64_t Bc, double *__restrict__ rho,
                                                     double *__restrict__ hist,
                                                     int32_t *__restrict__ active,
                                                     int32_t *__restrict__ iters, double rtol,
                                                     int max_iters, int first)
{
    const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= Bc) return;
    if (!first && !active[b]) return;
    const double v = sqrt(fold_partials<1>(part, b, fcg_nch(n), 0)) / (double)n;
    if ((threadIdx.x & 63) == 0) {
        const int it = first ? 0 : iters[b];
        // attainable accuracy: stop once four steps in a row have not brought
        // rho 10% below the best value so far (hist[4b]: that value,
        // hist[4b + 1]: steps since it was reached)
        double best = hist[4 * b], since = hist[4 * b + 1];
        if (it == 0 || v < 0.9 * best) {
            best = v;
            since = 0.0;
        } else {
            since += 1.0;
        }
        hist[4 * b] = best;
        hist[4 * b + 1] = since;
        const int go = v > rtol && it < max_iters && since < 4.0;
        rho[b] = v;
        active[b] = go;
        iters[b] = it + go;
    }
}

// partials of (r_{k-1}, z) and (r_{k-2}, z) (the second 0 at the first step)
template <typename T, int QH>
__global__ __launch_bounds__(256) void k_fcg_dots(const T *__restrict__ z, const T *__restrict__ F0,
                                                  const T *__restrict__ F1, int n, int64_t Bc,
                                                  double *__restrict__ part,
                                                  const int32_t *__restrict__ active,
                                                  const int32_t *__restrict__ iters)
{
    constexpr int CW = 16 / sizeof(T);
    FcgMap m;
    if (!fcg_map<CW, QH>(n, Bc, active, m)) return;
    const int64_t cells = (int64_t)n * n, base = m.b * cells;
    const int k = iters[m.b];
    const T *rb = ((k - 1) & 1 ? F1 : F0) + base;
    const T *rob = (k & 1 ? F1 : F0) + base;
    double s[2] = {0.0, 0.0}, c[2] = {0.0, 0.0};
#pragma unroll 2
    for (int t = 0; t < QH; ++t) {
        const int64_t o = (int64_t)(m.j0 + t) * n + m.i0;
        T zv[CW], rv[CW], ro[CW];
        ldv<CW>(z + base + o, zv);
        ldv<CW>(rb + o, rv);
        if (k > 1) ldv<CW>(rob + o, ro);
#pragma unroll
        for (int q = 0; q < CW; ++q) {
            neumaier(s[0], c[0], double(rv[q]) * double(zv[q]));
            neumaier(s[1], c[1], k > 1 ? double(ro[q]) * double(zv[q]) : 0.0);
        }
    }
    block_partials<2>(s, c, part + (m.b * m.nch + m.blk) * 4);
}

// fs[b] = {rz, rz_old, alpha, beta}: rz = (r, z), beta = (rz - (r_old, z)) / rz_old
__global__ __launch_bounds__(256) void k_fcg_fin_beta(const double *__restrict__ part, int n,
                                                      int64_t Bc, double *__restrict__ fs,
                                                      const int32_t *__restrict__ active,
                                                      const int32_t *__restrict__ iters)
{
    const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= Bc || !active[b]) return;
    const int nch = fcg_nch(n);
    const double rz = fold_partials<2>(part, b, nch, 0);
    const double rzo = fold_partials<2>(part, b, nch, 1);
    if ((threadIdx.x & 63) == 0) {
        fs[4 * b] = rz;
        fs[4 * b + 3] = iters[b] == 1 ? 0.0 : (rz - rzo) / fs[4 * b + 1];
    }
}

// p_k = z + beta p_{k-1} (p_1 = z), written to P[k & 1]; partial (p_k, A p_k)
// with A p_k in the V-cycle type T (p is stored in T; the step length only
// scales the update of the FP64 iterate, whose residual is recomputed in
// FP64), the products summed in FP64
template <typename T, int QH>
__global__ __launch_bounds__(256, 4) void k_fcg_p(const T *__restrict__ a, const T *__restrict__ z,
                                                  T *__restrict__ P0, T *__restrict__ P1, int n,
                                                  int64_t Bc, const double *__restrict__ fs,
                                                  double *__restrict__ part,
                                                  const int32_t *__restrict__ active,
                                                  const int32_t *__restrict__ iters)
{
    constexpr int CW = 16 / sizeof(T);
    FcgMap m;
    if (!fcg_map<CW, QH>(n, Bc, active, m)) return;
    const int64_t cells = (int64_t)n * n, base = m.b * cells;
    const int k = iters[m.b];
    const T bt = T(k == 1 ? 0.0 : fs[4 * m.b + 3]);
    const T *ab = a + base, *zb = z + base;
    const T *pold = ((k - 1) & 1 ? P1 : P0) + base;
    T *pnew = (k & 1 ? P1 : P0) + base;
    auto pk = [&](int64_t q) { return k == 1 ? zb[q] : T(zb[q] + bt * pold[q]); };
    using Row = GroupRow<T, T, CW>;
    auto load = [&](int j, Row &r) {
        const int64_t o = (int64_t)j * n + m.i0;
        ldv<CW>(ab + o, r.a);
        ldv<CW>(zb + o, r.v);
        if (k > 1) {
            T po[CW];
            ldv<CW>(pold + o, po);
#pragma unroll
            for (int c = 0; c < CW; ++c) r.v[c] = T(r.v[c] + bt * po[c]);
        }
    };
    const double n2 = double(n) * double(n);
    const bool down = strip_down(n, CW, m.j0, QH);
    double s[1] = {0.0}, c[1] = {0.0};
    auto body = [&](int j, const Row &cur, const Row &up, const Row &dn,
                    const T (&carried)[CW], T (&fresh)[CW]) {
        T al, vl, ar, vr;
        row_ends<CW>(cur, ab + (int64_t)j * n, (int64_t)j * n, m.i0, n, pk, al, vl, ar, vr);
        T flux[CW];
        row_flux<T, CW>(cur, al, vl, ar, vr, up, j + 1 < n, dn, j > 0, down, carried, fresh, m.i0,
                        n, flux);
#pragma unroll
        for (int q = 0; q < CW; ++q) neumaier(s[0], c[0], double(cur.v[q]) * n2 * double(flux[q]));
        stv<CW>(pnew + (int64_t)j * n + m.i0, cur.v);
    };
    strip_march<QH, T, CW, Row>(down, m.j0, n, load, body);
    block_partials<1>(s, c, part + (m.b * m.nch + m.blk) * 2);
}

// alpha = rz / (p, A p); rz_old = rz
__global__ __launch_bounds__(256) void k_fcg_fin_alpha(const double *__restrict__ part, int n,
                                                       int64_t Bc, double *__restrict__ fs,
                                                       const int32_t *__restrict__ active)
{
    const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= Bc || !active[b]) return;
    const double pq = fold_partials<1>(part, b, fcg_nch(n), 0);
    if ((threadIdx.x & 63) == 0) {
        fs[4 * b + 2] = fs[4 * b] / pq;
        fs[4 * b + 1] = fs[4 * b];
    }
}

// samples whose last step wrote X[1]: copy it to the stage solution X[0]
template <int QH>
__global__ __launch_bounds__(256) void k_fcg_copyback(double *__restrict__ X0,
                                                      const double *__restrict__ X1, int n,
                                                      int64_t Bc, const int32_t *__restrict__ iters)
{
    constexpr int CW = 2;
    FcgMap m;
    if (!fcg_map<CW, QH>(n, Bc, nullptr, m)) return;
    if (!(iters[m.b] & 1)) return;
    const int64_t base = m.b * (int64_t)n * n;
#pragma unroll 2
    for (int t = 0; t < QH; ++t) {
        const int64_t o = base + (int64_t)(m.j0 + t) * n + m.i0;
        double v[CW];
        ldv<CW>(X1 + o, v);
        stv<CW>(X0 + o, v);
    }
}

// fold one stage's final per-sample state into the per-sample statistics
__global__ void k_refine_stats(const int32_t *__restrict__ iters, const double *__restrict__ rho,
                               int64_t Bc, double rtol, int32_t *__restrict__ st_iters,
                               double *__restrict__ st_rho, int32_t *__restrict__ st_bad)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= Bc) return;
    if (iters[b] > st_iters[b]) st_iters[b] = iters[b];
    if (rho[b] > st_rho[b]) st_rho[b] = rho[b];
    if (rho[b] > rtol) st_bad[b] = 1;
}

inline unsigned nblocks(int64_t n) { return (unsigned)(n < 1 ? 1 : n); }
inline unsigned blocks_of(int64_t n, int per) { return nblocks((n + per - 1) / per); }

}  // namespace

// ---------------------------------------------------------------------------
bool fused_supported(int mu1, int mu2) { return mu1 >= 1 && mu1 <= 2 && mu2 >= 1 && mu2 <= 2; }

// Tile shapes: 32 x 32 cells per 256-thread workgroup, or 16 x 16 per 128
// threads; every shape gives the bits of the global sweep order.
int tile_side(int shape) { return shape == kTile16 ? 16 : 32; }

template <typename T>
void launch_pre_tile(hipStream_t st, int shape, int mu1, const T *a, const T *f, const T *u_in,
                     T *u_out, const T *uc, int n, int64_t Bc, int init, T *fc,
                     const int32_t *active)
{
    const int ts = tile_side(shape);
    const unsigned blocks = nblocks(Bc * (int64_t)(n / ts) * (n / ts));
#define L(TL, NTH, MU)                                                                             \
    hipLaunchKernelGGL((k_pre_tile<TL, NTH, MU, T>), dim3(blocks), dim3(NTH), 0, st, a, f, u_in,  \
                       u_out, uc, n, Bc, init, fc, active)
    if (ts == 16) {
        if (mu1 == 2) L(16, 128, 2); else L(16, 128, 1);
    } else {
        if (mu1 == 2) L(32, 256, 2); else L(32, 256, 1);
    }
#undef L
}

template <typename T>
void launch_post_tile(hipStream_t st, int shape, int mu2, const T *a, const T *f, const T *u_in,
                      T *u_out, const T *ec, int n, int64_t Bc, const int32_t *active)
{
    const int ts = tile_side(shape);
    const unsigned blocks = nblocks(Bc * (int64_t)(n / ts) * (n / ts));
#define L(TL, NTH, MU)                                                                             \
    hipLaunchKernelGGL((k_post_tile<TL, NTH, MU, T>), dim3(blocks), dim3(NTH), 0, st, a, f, u_in, \
                       u_out, ec, n, Bc, active)
    if (ts == 16) {
        if (mu2 == 2) L(16, 128, 2); else L(16, 128, 1);
    } else {
        if (mu2 == 2) L(32, 256, 2); else L(32, 256, 1);
    }
#undef L
}

// Workgroups sized to the top LDS grid: LDS for exactly levels 0..G, one
// wavefront for grids <= 8^2, 128 threads for 16^2, 256 for 32^2.
#define MLMC_LDS_DISPATCH(G, LAUNCH)                                                               \
    switch (G) {                                                                                   \
    case 0:                                                                                        \
    case 1: LAUNCH(1, 64); break;                                                                  \
    case 2: LAUNCH(2, 64); break;                                                                  \
    case 3: LAUNCH(3, 128); break;                                                                 \
    default: LAUNCH(4, 256); break;                                                                \
    }

void launch_lds_fmg_fixed(hipStream_t st, const double *a_pool, double *u_pool, int64_t Bc, int G,
                          int mu0, int mu1, int mu2, int g0, double *qoi, int nlev, uint32_t mask)
{
#define L(GS, NTH)                                                                                 \
    hipLaunchKernelGGL((k_lds_fmg_fixed<GS, NTH>), dim3(nblocks(Bc)), dim3(NTH), 0, st, a_pool,   \
                       u_pool, Bc, G, mu0, mu1, mu2, g0, qoi, nlev, mask)
    MLMC_LDS_DISPATCH(G, L)
#undef L
}

template <typename T>
void launch_lds_vcycle(hipStream_t st, const T *a_pool, const T *f_pool, T *u_pool, int64_t Bc,
                       int G, int mu1, int mu2, const int32_t *active)
{
#define L(GS, NTH)                                                                                 \
    hipLaunchKernelGGL((k_lds_vcycle<GS, T, NTH>), dim3(nblocks(Bc)), dim3(NTH), 0, st, a_pool,   \
                       f_pool, u_pool, Bc, G, mu1, mu2, active)
    MLMC_LDS_DISPATCH(G, L)
#undef L
}

template <typename T>
void launch_lds_fmg_refine(hipStream_t st, const T *a_pool, const double *a64_pool,
                           double *u64_pool, int64_t Bc, int G, int mu1, int mu2, double rtol,
                           int max_iters, int g0, double *qoi, int nlev, uint32_t mask,
                           int32_t *st_iters, double *st_rho, int32_t *st_bad)
{
#define L(GS, NTH)                                                                                 \
    hipLaunchKernelGGL((k_lds_fmg_refine<GS, T, NTH>), dim3(nblocks(Bc)), dim3(NTH), 0, st,       \
                       a_pool, a64_pool, u64_pool, Bc, G, mu1, mu2, rtol, max_iters, g0, qoi,     \
                       nlev, mask, st_iters, st_rho, st_bad)
    MLMC_LDS_DISPATCH(G, L)
#undef L
}
#undef MLMC_LDS_DISPATCH

int64_t fcg_partials(int n, int64_t Bc) { return Bc * fcg_nch(n) * 4; }

// the CG passes' strip height: QH = 4 q / CW rows (q = 4 on 64^2, 8 above)
#define MLMC_FCG_QH(n, CW, LAUNCH)          \
    do {                                    \
        if (fcg_q(n) == 4) {                \
            constexpr int QH = 16 / (CW);   \
            LAUNCH;                         \
        } else {                            \
            constexpr int QH = 32 / (CW);   \
            LAUNCH;                         \
        }                                   \
    } while (0)

template <typename T>
void launch_fcg_resid(hipStream_t st, const double *a, const double *x, int n, int64_t Bc, T *f,
                      double *part)
{
    const unsigned nb = nblocks(Bc * fcg_nch(n));
    MLMC_FCG_QH(n, 2, hipLaunchKernelGGL((k_fcg_x<T, QH, false>), dim3(nb), dim3(256), 0, st, a,
                                         const_cast<double *>(x), nullptr, nullptr, nullptr, f,
                                         nullptr, n, Bc, nullptr, part, nullptr, nullptr));
}

void launch_fcg_fin_rho(hipStream_t st, const double *part, int n, int64_t Bc, double *rho,
                        double *hist, int32_t *active, int32_t *iters, double rtol, int max_iters,
                        int first)
{
    hipLaunchKernelGGL(k_fcg_fin_rho, dim3(blocks_of(Bc, 4)), dim3(256), 0, st, part, n, Bc, rho,
                       hist, active, iters, rtol, max_iters, first);
}

template <typename T>
void launch_fcg_step(hipStream_t st, const FcgBufs<T> &v, int n, int64_t Bc, double rtol,
                     int max_iters)
{
    constexpr int CWT = 16 / sizeof(T);
    const unsigned nb = nblocks(Bc * fcg_nch(n));
    const unsigned ns = blocks_of(Bc, 4);
    MLMC_FCG_QH(n, CWT, hipLaunchKernelGGL((k_fcg_dots<T, QH>), dim3(nb), dim3(256), 0, st, v.z,
                                           v.f, v.fo, n, Bc, v.part, v.active, v.iters));
    hipLaunchKernelGGL(k_fcg_fin_beta, dim3(ns), dim3(256), 0, st, v.part, n, Bc, v.fs, v.active,
                       v.iters);
    MLMC_FCG_QH(n, CWT, hipLaunchKernelGGL((k_fcg_p<T, QH>), dim3(nb), dim3(256), 0, st, v.a, v.z,
                                           v.p0, v.p1, n, Bc, v.fs, v.part, v.active, v.iters));
    hipLaunchKernelGGL(k_fcg_fin_alpha, dim3(ns), dim3(256), 0, st, v.part, n, Bc, v.fs, v.active);
    MLMC_FCG_QH(n, 2, hipLaunchKernelGGL((k_fcg_x<T, QH, true>), dim3(nb), dim3(256), 0, st, v.a64,
                                         v.x0, v.x1, v.p0, v.p1, v.f, v.fo, n, Bc, v.fs, v.part,
                                         v.active, v.iters));
    hipLaunchKernelGGL(k_fcg_fin_rho, dim3(ns), dim3(256), 0, st, v.part, n, Bc, v.rho, v.hist, v.active,
                       v.iters, rtol, max_iters, 0);
}

void launch_fcg_copyback(hipStream_t st, double *x0, const double *x1, int n, int64_t Bc,
                         const int32_t *iters)
{
    const unsigned nb = nblocks(Bc * fcg_nch(n));
    MLMC_FCG_QH(n, 2, hipLaunchKernelGGL((k_fcg_copyback<QH>), dim3(nb), dim3(256), 0, st, x0, x1,
                                         n, Bc, iters));
}
#undef MLMC_FCG_QH

void launch_refine_stats(hipStream_t st, const int32_t *iters, const double *rho, int64_t Bc,
                         double rtol, int32_t *st_iters, double *st_rho, int32_t *st_bad)
{
    hipLaunchKernelGGL(k_refine_stats, dim3(blocks_of(Bc, 256)), dim3(256), 0, st, iters, rho, Bc,
                       rtol, st_iters, st_rho, st_bad);
}

#define MLMC_INSTANTIATE(T)                                                                        \
    template void launch_pre_tile<T>(hipStream_t, int, int, const T *, const T *, const T *, T *, \
                                     const T *, int, int64_t, int, T *, const int32_t *);          \
    template void launch_post_tile<T>(hipStream_t, int, int, const T *, const T *, const T *, T *,\
                                      const T *, int, int64_t, const int32_t *);                   \
    template void launch_lds_vcycle<T>(hipStream_t, const T *, const T *, T *, int64_t, int, int, \
                                       int, const int32_t *);                                      \
    template void launch_lds_fmg_refine<T>(hipStream_t, const T *, const double *, double *,      \
                                           int64_t, int, int, int, double, int, int, double *,     \
                                           int, uint32_t, int32_t *, double *, int32_t *);         \
    template void launch_fcg_resid<T>(hipStream_t, const double *, const double *, int, int64_t,\
                                      T *, double *);                                             \
    template void launch_fcg_step<T>(hipStream_t, const FcgBufs<T> &, int, int64_t, double, int);
MLMC_INSTANTIATE(double)
MLMC_INSTANTIATE(float)
#undef MLMC_INSTANTIATE

}  // namespace mlmc
