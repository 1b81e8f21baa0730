// Fused multigrid kernels for gfx950 (Section 4: correction scheme, V-cycle,
// full multigrid), FP64.
//
// Large grids (n >= 64): temporally blocked tile passes.  One workgroup owns a
// T x T tile of one sample and stages the tile plus a halo of u and a in LDS:
//   pre pass  : mu1 red-black sweeps (red first), residual, 4-cell restriction
//               -> writes u (tile) and the coarse right-hand side;
//   post pass : bilinear prolongation of the coarse correction, mu2 sweeps
//               (black first) -> writes u (tile).
// Each half-sweep t updates the cells of its colour within a ring that shrinks
// by one cell per half-sweep, so the tile's result equals the global sweep
// order exactly.  Face weights and the inverse diagonal of every cell a thread
// updates are computed once and kept in registers for all half-sweeps.
//
// Small grids (n <= 32): one workgroup per sample keeps the whole hierarchy
// 2^2 .. n^2 in LDS and runs the FMG stages (or one V-cycle) without leaving
// the CU.
//
// Block ids are remapped so that consecutive tiles of a sample run on the
// same XCD (the dispatcher deals blocks round-robin over the 8 XCDs), which
// keeps the overlapping halos in that XCD's L2.
#include "internal.hpp"

namespace mlmc {
namespace {

constexpr int TILE = 32;
constexpr int NT = 256;                 // threads per tile workgroup

// 1/x for the well-scaled positive values of this path (coefficients within
// e^+-15, diagonals of their sums): hardware reciprocal estimate refined by two
// Newton steps, accurate to about one ulp without the special-case handling of
// IEEE division.
__device__ __forceinline__ double frcp(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}

// harmonic face weight 2 a_P a_N / (a_P + a_N)
__device__ __forceinline__ double hm(double ap, double an) { return 2.0 * ap * an * frcp(ap + an); }

__device__ __forceinline__ int xcd_remap(int bid, int nb)
{
    const int per = nb / 8;
    return bid < per * 8 ? (bid % 8) * per + bid / 8 : bid;
}

// value of the coarse grid e (nc x nc) at coarse index (I, J), odd reflection
__device__ __forceinline__ double codd(const double *__restrict__ e, int nc, int I, int J)
{
    double sg = 1.0;
    if (I < 0) { I = 0; sg = -sg; }
    if (I >= nc) { I = nc - 1; sg = -sg; }
    if (J < 0) { J = 0; sg = -sg; }
    if (J >= nc) { J = nc - 1; sg = -sg; }
    return sg * e[I + nc * J];
}

// bilinear (9,3,3,1)/16 value of P e at fine cell (i, j)
__device__ __forceinline__ double prolong_at(const double *__restrict__ e, int nc, int i, int j)
{
    const int I = i >> 1, J = j >> 1;
    const int sx = (i & 1) ? 1 : -1, sy = (j & 1) ? 1 : -1;
    return (9.0 * codd(e, nc, I, J) + 3.0 * codd(e, nc, I + sx, J) + 3.0 * codd(e, nc, I, J + sy) +
            codd(e, nc, I + sx, J + sy)) / 16.0;
}

// Coarse values needed to prolongate onto a fine region [fi0, fi0+S)^2, staged
// in LDS with the odd wall reflection already applied (indices -1 and nc).
template <int S>
struct CoarseStage {
    static constexpr int CS = S / 2 + 3;
    __device__ static void load(double *cs, const double *__restrict__ e, int nc, int cI0, int cJ0)
    {
        for (int q = threadIdx.x; q < CS * CS; q += NT) {
            const int cj = q / CS, ci = q - cj * CS;
            const int I = cI0 + ci, J = cJ0 + cj;
            cs[q] = (I >= -1 && I <= nc && J >= -1 && J <= nc) ? codd(e, nc, I, J) : 0.0;
        }
    }
    // P e at in-domain fine cell (gi, gj)
    __device__ static double at(const double *cs, int cI0, int cJ0, int gi, int gj)
    {
        const int I = (gi >> 1) - cI0, J = (gj >> 1) - cJ0;
        const int sx = (gi & 1) ? 1 : -1, sy = (gj & 1) ? CS : -CS;
        const int q = I + CS * J;
        return (9.0 * cs[q] + 3.0 * cs[q + sx] + 3.0 * cs[q + sy] + cs[q + sx + sy]) / 16.0;
    }
};

// Per-cell stencil kept in registers.
struct Cell {
    int l;                        // LDS index li + S*lj, -1 if not owned / outside
    double wE, wW, wN, wS, d, inv, rhs;   // d = sum of face weights, rhs = h^2 f
};

template <int S>
__device__ __forceinline__ void make_cell(Cell &c, const double *a_s, int li, int lj, int gi, int gj,
                                          int n, double rhs)
{
    const int l = li + S * lj;
    const double ap = a_s[l];
    double d = 0.0;
    c.wE = c.wW = c.wN = c.wS = 0.0;
    if (gi + 1 < n) { c.wE = hm(ap, a_s[l + 1]); d += c.wE; } else d += 2.0 * ap;
    if (gi > 0)     { c.wW = hm(ap, a_s[l - 1]); d += c.wW; } else d += 2.0 * ap;
    if (gj + 1 < n) { c.wN = hm(ap, a_s[l + S]); d += c.wN; } else d += 2.0 * ap;
    if (gj > 0)     { c.wS = hm(ap, a_s[l - S]); d += c.wS; } else d += 2.0 * ap;
    c.d = d;
    c.inv = frcp(d);
    c.rhs = rhs;
    c.l = l;
}

template <int S>
__device__ __forceinline__ void relax(const Cell &c, double *u_s)
{
    const int l = c.l;
    double num = c.rhs;
    num += c.wE * u_s[l + 1];
    num += c.wW * u_s[l - 1];
    num += c.wN * u_s[l + S];
    num += c.wS * u_s[l - S];
    u_s[l] = num * c.inv;
}

// Owned cells of one colour inside the square ring [lo, S-lo)^2 of the region.
// q-th cell: row r = q / half, column 2*(q % half) + parity.
template <int S, int LO, int COLOUR>
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

// ---------------------------------------------------------------------------
// Pre pass: mu1 red-black sweeps + residual + restriction on one tile.
// init: 0 = read u, 1 = zero initial guess, 2 = FMG interpolation from uc.
template <int MU>
__global__ __launch_bounds__(NT) void k_pre_tile(const double *__restrict__ a,
                                                 const double *__restrict__ f, double *__restrict__ u,
                                                 const double *__restrict__ uc, int n, int64_t Bc,
                                                 int init, double *__restrict__ fc,
                                                 const int32_t *__restrict__ active)
{
    constexpr int H = 2 * MU + 1;
    constexpr int S = TILE + 2 * H;
    using Red = OwnSet<S, 1, 0>;              // red cells are updated within ring H-1
    using Blk = OwnSet<S, 2, 1>;              // black cells within ring H-2
    using CSt = CoarseStage<S>;
    __shared__ double u_s[S * S];
    __shared__ double a_s[S * S];
    __shared__ double c_s[CSt::CS * CSt::CS];

    const int tiles_side = n / TILE;
    const int tps = tiles_side * tiles_side;
    const int L = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t b = L / tps;
    if (b >= Bc) return;
    if (active && !active[b]) return;
    const int tile = L - (int)(b * tps);
    const int i0 = (tile % tiles_side) * TILE, j0 = (tile / tiles_side) * TILE;
    const int64_t cells = (int64_t)n * n;
    const double *ab = a + b * cells;
    double *ub = u + b * cells;
    const double *fb = f ? f + b * cells : nullptr;
    const int nc = n / 2;
    const double h2 = 1.0 / ((double)n * (double)n);
    const int cI0 = i0 / 2 - (H + 1) / 2 - 1, cJ0 = j0 / 2 - (H + 1) / 2 - 1;
    if (init == 2) {
        CSt::load(c_s, uc + b * (int64_t)nc * nc, nc, cI0, cJ0);
        __syncthreads();
    }

    // all global loads of the region first (memory-level parallelism), then LDS
    constexpr int PERT = (S * S + NT - 1) / NT;
    double av[PERT], uv[PERT];
#pragma unroll
    for (int k = 0; k < PERT; ++k) {
        const int e = threadIdx.x + NT * k;
        const int lj = e / S, li = e - lj * S;
        const int gi = i0 - H + li, gj = j0 - H + lj;
        av[k] = 0.0;
        uv[k] = 0.0;
        if (e < S * S && gi >= 0 && gi < n && gj >= 0 && gj < n) {
            const int64_t p = gi + (int64_t)n * gj;
            av[k] = ab[p];
            if (init == 0) uv[k] = ub[p];
            else if (init == 2) uv[k] = CSt::at(c_s, cI0, cJ0, gi, gj);
        }
    }
#pragma unroll
    for (int k = 0; k < PERT; ++k) {
        const int e = threadIdx.x + NT * k;
        if (e < S * S) {
            a_s[e] = av[k];
            u_s[e] = uv[k];
        }
    }
    __syncthreads();

    Cell red[Red::PER], blk[Blk::PER];
#pragma unroll
    for (int k = 0; k < Red::PER; ++k) {
        const int q = threadIdx.x + NT * k;
        red[k].l = -1;
        if (q < Red::COUNT) {
            int li, lj;
            Red::coords(q, li, lj);
            const int gi = i0 - H + li, gj = j0 - H + lj;
            if (gi >= 0 && gi < n && gj >= 0 && gj < n)
                make_cell<S>(red[k], a_s, li, lj, gi, gj, n, h2 * (fb ? fb[gi + (int64_t)n * gj] : 1.0));
        }
    }
#pragma unroll
    for (int k = 0; k < Blk::PER; ++k) {
        const int q = threadIdx.x + NT * k;
        blk[k].l = -1;
        if (q < Blk::COUNT) {
            int li, lj;
            Blk::coords(q, li, lj);
            const int gi = i0 - H + li, gj = j0 - H + lj;
            if (gi >= 0 && gi < n && gj >= 0 && gj < n)
                make_cell<S>(blk[k], a_s, li, lj, gi, gj, n, h2 * (fb ? fb[gi + (int64_t)n * gj] : 1.0));
        }
    }
    // half-sweep t (1-based) covers ring H - t around the tile
#pragma unroll
    for (int t = 1; t <= 2 * MU; ++t) {
        const int lo = t, hi = S - t;          // region index range [lo, hi)
        if (t & 1) {
#pragma unroll
            for (int k = 0; k < Red::PER; ++k) {
                const int l = red[k].l;
                if (l < 0) continue;
                const int lj = l / S, li = l - lj * S;
                if (li >= lo && li < hi && lj >= lo && lj < hi) relax<S>(red[k], u_s);
            }
        } else {
#pragma unroll
            for (int k = 0; k < Blk::PER; ++k) {
                const int l = blk[k].l;
                if (l < 0) continue;
                const int lj = l / S, li = l - lj * S;
                if (li >= lo && li < hi && lj >= lo && lj < hi) relax<S>(blk[k], u_s);
            }
        }
        __syncthreads();
    }
    // residual r = f - A u on the tile, into a_s (a is no longer read)
    const double inv_h2 = (double)n * (double)n;
    auto resid = [&](const Cell &c) {
        const int l = c.l;
        const int lj = l / S, li = l - lj * S;
        if (li < H || li >= H + TILE || lj < H || lj >= H + TILE) return;
        double off = c.wE * u_s[l + 1];
        off += c.wW * u_s[l - 1];
        off += c.wN * u_s[l + S];
        off += c.wS * u_s[l - S];
        // h^-2 (h^2 f - (D u - sum w u_nbr)); h^2, h^-2 are powers of two
        a_s[l] = inv_h2 * (c.rhs - (c.d * u_s[l] - off));
    };
#pragma unroll
    for (int k = 0; k < Red::PER; ++k)
        if (red[k].l >= 0) resid(red[k]);
#pragma unroll
    for (int k = 0; k < Blk::PER; ++k)
        if (blk[k].l >= 0) resid(blk[k]);
    __syncthreads();
    // restriction (mean of the 4 children) and write-back of the tile
    {
        constexpr int CT = TILE / 2;
        for (int e = threadIdx.x; e < CT * CT; e += NT) {
            const int J = e / CT, I = e - J * CT;
            const int l = (H + 2 * I) + S * (H + 2 * J);
            const double v = 0.25 * (a_s[l] + a_s[l + 1] + a_s[l + S] + a_s[l + S + 1]);
            fc[b * (int64_t)nc * nc + (i0 / 2 + I) + (int64_t)nc * (j0 / 2 + J)] = v;
        }
        for (int e = threadIdx.x; e < TILE * TILE; e += NT) {
            const int lj = e / TILE, li = e - lj * TILE;
            ub[(i0 + li) + (int64_t)n * (j0 + lj)] = u_s[(H + li) + S * (H + lj)];
        }
    }
}

// Post pass: u += P ec on the tile and its halo, then mu2 sweeps black first.
template <int MU>
__global__ __launch_bounds__(NT) void k_post_tile(const double *__restrict__ a,
                                                  const double *__restrict__ f,
                                                  double *__restrict__ u,
                                                  const double *__restrict__ ec, int n, int64_t Bc,
                                                  const int32_t *__restrict__ active)
{
    constexpr int H = 2 * MU;
    constexpr int S = TILE + 2 * H;
    using Blk = OwnSet<S, 1, 1>;              // first half-sweep (black): ring H-1
    using Red = OwnSet<S, 2, 0>;              // second (red): ring H-2
    using CSt = CoarseStage<S>;
    __shared__ double u_s[S * S];
    __shared__ double a_s[S * S];
    __shared__ double c_s[CSt::CS * CSt::CS];

    const int tiles_side = n / TILE;
    const int tps = tiles_side * tiles_side;
    const int L = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t b = L / tps;
    if (b >= Bc) return;
    if (active && !active[b]) return;
    const int tile = L - (int)(b * tps);
    const int i0 = (tile % tiles_side) * TILE, j0 = (tile / tiles_side) * TILE;
    const int64_t cells = (int64_t)n * n;
    const double *ab = a + b * cells;
    double *ub = u + b * cells;
    const double *fb = f ? f + b * cells : nullptr;
    const int nc = n / 2;
    const double h2 = 1.0 / ((double)n * (double)n);
    const int cI0 = i0 / 2 - (H + 1) / 2 - 1, cJ0 = j0 / 2 - (H + 1) / 2 - 1;
    CSt::load(c_s, ec + b * (int64_t)nc * nc, nc, cI0, cJ0);
    __syncthreads();

    constexpr int PERT = (S * S + NT - 1) / NT;
    double av[PERT], uv[PERT];
#pragma unroll
    for (int k = 0; k < PERT; ++k) {
        const int e = threadIdx.x + NT * k;
        const int lj = e / S, li = e - lj * S;
        const int gi = i0 - H + li, gj = j0 - H + lj;
        av[k] = 0.0;
        uv[k] = 0.0;
        if (e < S * S && gi >= 0 && gi < n && gj >= 0 && gj < n) {
            const int64_t p = gi + (int64_t)n * gj;
            av[k] = ab[p];
            uv[k] = ub[p] + CSt::at(c_s, cI0, cJ0, gi, gj);
        }
    }
#pragma unroll
    for (int k = 0; k < PERT; ++k) {
        const int e = threadIdx.x + NT * k;
        if (e < S * S) {
            a_s[e] = av[k];
            u_s[e] = uv[k];
        }
    }
    __syncthreads();

    Cell blk[Blk::PER], red[Red::PER];
#pragma unroll
    for (int k = 0; k < Blk::PER; ++k) {
        const int q = threadIdx.x + NT * k;
        blk[k].l = -1;
        if (q < Blk::COUNT) {
            int li, lj;
            Blk::coords(q, li, lj);
            const int gi = i0 - H + li, gj = j0 - H + lj;
            if (gi >= 0 && gi < n && gj >= 0 && gj < n)
                make_cell<S>(blk[k], a_s, li, lj, gi, gj, n, h2 * (fb ? fb[gi + (int64_t)n * gj] : 1.0));
        }
    }
#pragma unroll
    for (int k = 0; k < Red::PER; ++k) {
        const int q = threadIdx.x + NT * k;
        red[k].l = -1;
        if (q < Red::COUNT) {
            int li, lj;
            Red::coords(q, li, lj);
            const int gi = i0 - H + li, gj = j0 - H + lj;
            if (gi >= 0 && gi < n && gj >= 0 && gj < n)
                make_cell<S>(red[k], a_s, li, lj, gi, gj, n, h2 * (fb ? fb[gi + (int64_t)n * gj] : 1.0));
        }
    }
#pragma unroll
    for (int t = 1; t <= 2 * MU; ++t) {
        const int lo = t, hi = S - t;
        if (t & 1) {
#pragma unroll
            for (int k = 0; k < Blk::PER; ++k) {
                const int l = blk[k].l;
                if (l < 0) continue;
                const int lj = l / S, li = l - lj * S;
                if (li >= lo && li < hi && lj >= lo && lj < hi) relax<S>(blk[k], u_s);
            }
        } else {
#pragma unroll
            for (int k = 0; k < Red::PER; ++k) {
                const int l = red[k].l;
                if (l < 0) continue;
                const int lj = l / S, li = l - lj * S;
                if (li >= lo && li < hi && lj >= lo && lj < hi) relax<S>(red[k], u_s);
            }
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < TILE * TILE; e += NT) {
        const int lj = e / TILE, li = e - lj * TILE;
        ub[(i0 + li) + (int64_t)n * (j0 + lj)] = u_s[(H + li) + S * (H + lj)];
    }
}

// ---------------------------------------------------------------------------
// LDS-resident hierarchy 2^2 .. 2^(GS+1) for one sample per workgroup.
constexpr int LT = 256;                 // threads per LDS workgroup

template <int GS>
struct LdsHier {
    static constexpr int TOTAL = (int)(4 * ((1LL << (2 * (GS + 1))) - 1) / 3);
    static __device__ constexpr int off(int g) { return (int)(4 * ((1LL << (2 * g)) - 1) / 3); }
};

__device__ __forceinline__ void lds_stencil(const double *a, int n, int i, int j, double &wE,
                                            double &wW, double &wN, double &wS, double &d)
{
    const int p = i + n * j;
    const double ap = a[p];
    d = 0.0;
    wE = wW = wN = wS = 0.0;
    if (i + 1 < n) { wE = hm(ap, a[p + 1]); d += wE; } else d += 2.0 * ap;
    if (i > 0)     { wW = hm(ap, a[p - 1]); d += wW; } else d += 2.0 * ap;
    if (j + 1 < n) { wN = hm(ap, a[p + n]); d += wN; } else d += 2.0 * ap;
    if (j > 0)     { wS = hm(ap, a[p - n]); d += wS; } else d += 2.0 * ap;
}

__device__ __forceinline__ double lds_nb(const double *u, int n, int i, int j)
{
    return (i < 0 || j < 0 || i >= n || j >= n) ? 0.0 : u[i + n * j];
}

// one colour; f == nullptr means f = 1
__device__ void lds_sweep(const double *a, const double *f, double *u, int n, int colour)
{
    const int half = n / 2;
    const double h2 = 1.0 / ((double)n * (double)n);
    for (int q = threadIdx.x; q < n * half; q += LT) {
        const int j = q / half;
        const int i = 2 * (q - j * half) + ((j + colour) & 1);
        double wE, wW, wN, wS, d;
        lds_stencil(a, n, i, j, wE, wW, wN, wS, d);
        double num = h2 * (f ? f[i + n * j] : 1.0);
        num += wE * lds_nb(u, n, i + 1, j);
        num += wW * lds_nb(u, n, i - 1, j);
        num += wN * lds_nb(u, n, i, j + 1);
        num += wS * lds_nb(u, n, i, j - 1);
        u[i + n * j] = num * frcp(d);
    }
    __syncthreads();
}

__device__ __forceinline__ double lds_resid(const double *a, const double *f, const double *u,
                                            int n, int i, int j)
{
    double wE, wW, wN, wS, d;
    lds_stencil(a, n, i, j, wE, wW, wN, wS, d);
    double off = wE * lds_nb(u, n, i + 1, j);
    off += wW * lds_nb(u, n, i - 1, j);
    off += wN * lds_nb(u, n, i, j + 1);
    off += wS * lds_nb(u, n, i, j - 1);
    return (f ? f[i + n * j] : 1.0) - (double)n * (double)n * (d * u[i + n * j] - off);
}

__device__ void lds_coarse_solve(const double *a, const double *f, double *u)
{
    if (threadIdx.x == 0) {
        double w01 = hm(a[0], a[1]), w02 = hm(a[0], a[2]), w13 = hm(a[1], a[3]), w23 = hm(a[2], a[3]);
        double A[4][4] = {{w01 + w02 + 4.0 * a[0], -w01, -w02, 0.0},
                          {-w01, w01 + w13 + 4.0 * a[1], 0.0, -w13},
                          {-w02, 0.0, w02 + w23 + 4.0 * a[2], -w23},
                          {0.0, -w13, -w23, w13 + w23 + 4.0 * a[3]}};
        double L[4][4] = {}, v[4];
        for (int p = 0; p < 4; ++p)
            for (int q = 0; q <= p; ++q) {
                double s = A[p][q];
                for (int t = 0; t < q; ++t) s -= L[p][t] * L[q][t];
                L[p][q] = (p == q) ? sqrt(s) : s / L[q][q];
            }
        for (int p = 0; p < 4; ++p) {
            double s = 0.25 * (f ? f[p] : 1.0);
            for (int q = 0; q < p; ++q) s -= L[p][q] * v[q];
            v[p] = s / L[p][p];
        }
        for (int p = 3; p >= 0; --p) {
            double s = v[p];
            for (int q = p + 1; q < 4; ++q) s -= L[q][p] * v[q];
            v[p] = s / L[p][p];
        }
        for (int p = 0; p < 4; ++p) u[p] = v[p];
    }
    __syncthreads();
}

__device__ __forceinline__ double lds_codd(const double *e, int nc, int I, int J)
{
    double sg = 1.0;
    if (I < 0) { I = 0; sg = -sg; }
    if (I >= nc) { I = nc - 1; sg = -sg; }
    if (J < 0) { J = 0; sg = -sg; }
    if (J >= nc) { J = nc - 1; sg = -sg; }
    return sg * e[I + nc * J];
}

// u = P e (add = false) or u += P e on the n x n grid
__device__ void lds_prolong(const double *e, double *u, int n, bool add)
{
    const int nc = n / 2;
    for (int p = threadIdx.x; p < n * n; p += LT) {
        const int j = p / n, i = p - j * n;
        const int I = i >> 1, J = j >> 1, sx = (i & 1) ? 1 : -1, sy = (j & 1) ? 1 : -1;
        const double v = (9.0 * lds_codd(e, nc, I, J) + 3.0 * lds_codd(e, nc, I + sx, J) +
                          3.0 * lds_codd(e, nc, I, J + sy) + lds_codd(e, nc, I + sx, J + sy)) / 16.0;
        u[p] = add ? u[p] + v : v;
    }
    __syncthreads();
}

template <int GS>
struct LdsVcycle {
    double *a, *u, *f;   // LDS bases, level g at LdsHier<GS>::off(g)
    int mu1, mu2;
    // V(mu1,mu2) at level g (one coarse-grid correction per level, so the
    // recursion unrolls into a descent and an ascent).  The top right-hand
    // side may be nullptr (f = 1); the coarser ones live in LDS.
    __device__ void run(int g, const double *ftop)
    {
        for (int l = g; l >= 1; --l) {
            const int n = 2 << l, nc = n / 2;
            double *al = a + LdsHier<GS>::off(l), *ul = u + LdsHier<GS>::off(l);
            const double *fl = (l == g) ? ftop : f + LdsHier<GS>::off(l);
            for (int it = 0; it < mu1; ++it) {
                lds_sweep(al, fl, ul, n, 0);
                lds_sweep(al, fl, ul, n, 1);
            }
            double *fcl = f + LdsHier<GS>::off(l - 1), *ucl = u + LdsHier<GS>::off(l - 1);
            for (int q = threadIdx.x; q < nc * nc; q += LT) {
                const int J = q / nc, I = q - J * nc;
                const double r00 = lds_resid(al, fl, ul, n, 2 * I, 2 * J);
                const double r10 = lds_resid(al, fl, ul, n, 2 * I + 1, 2 * J);
                const double r01 = lds_resid(al, fl, ul, n, 2 * I, 2 * J + 1);
                const double r11 = lds_resid(al, fl, ul, n, 2 * I + 1, 2 * J + 1);
                fcl[q] = 0.25 * (r00 + r10 + r01 + r11);
                ucl[q] = 0.0;
            }
            __syncthreads();
        }
        lds_coarse_solve(a, g == 0 ? ftop : f, u);
        for (int l = 1; l <= g; ++l) {
            const int n = 2 << l;
            double *al = a + LdsHier<GS>::off(l), *ul = u + LdsHier<GS>::off(l);
            const double *fl = (l == g) ? ftop : f + LdsHier<GS>::off(l);
            lds_prolong(u + LdsHier<GS>::off(l - 1), ul, n, true);
            for (int it = 0; it < mu2; ++it) {
                lds_sweep(al, fl, ul, n, 1);
                lds_sweep(al, fl, ul, n, 0);
            }
        }
    }
};

// deterministic block sum (Neumaier per thread, fixed pairwise tree)
__device__ double lds_block_sum(const double *v, int count, double *scratch)
{
    double s = 0.0, c = 0.0;
    for (int p = threadIdx.x; p < count; p += LT) {
        const double x = v[p];
        const double t = s + x;
        if (fabs(s) >= fabs(x)) c += (s - t) + x; else c += (x - t) + s;
        s = t;
    }
    scratch[2 * threadIdx.x] = s;
    scratch[2 * threadIdx.x + 1] = c;
    __syncthreads();
    for (int w = LT / 2; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const double s1 = scratch[2 * threadIdx.x], c1 = scratch[2 * threadIdx.x + 1];
            const double s2 = scratch[2 * (threadIdx.x + w)], c2 = scratch[2 * (threadIdx.x + w) + 1];
            const double t = s1 + s2, bb = t - s1;
            const double err = (s1 - (t - bb)) + (s2 - bb);
            scratch[2 * threadIdx.x] = t;
            scratch[2 * threadIdx.x + 1] = c1 + c2 + err;
        }
        __syncthreads();
    }
    const double r = scratch[0] + scratch[1];
    __syncthreads();
    return r;
}

// mode 0: FMG stages 0..G (G <= GS), QoI of stages g >= g0, final u to HBM.
// mode 1: one V-cycle at level G with zero initial guess and f read from HBM,
//         correction written to the u pool at level G.
template <int GS>
__global__ __launch_bounds__(LT) void k_lds_mg(const double *__restrict__ a_pool,
                                               const double *__restrict__ f_pool,
                                               double *__restrict__ u_pool, int64_t Bc, int G,
                                               int mode, int mu0, int mu1, int mu2, int g0,
                                               double *__restrict__ qoi, int nlev, uint32_t mask,
                                               const int32_t *__restrict__ active)
{
    constexpr int TOT = LdsHier<GS>::TOTAL;
    __shared__ double a_s[TOT], u_s[TOT], f_s[TOT];
    __shared__ double red_s[2 * LT];
    const int64_t b = blockIdx.x;
    if (b >= Bc) return;
    if (active && !active[b]) return;
    for (int g = 0; g <= G; ++g) {
        const int cnt = 4 << (2 * g);
        const double *src = a_pool + Bc * level_offset(g) + b * (int64_t)cnt;
        for (int p = threadIdx.x; p < cnt; p += LT) a_s[LdsHier<GS>::off(g) + p] = src[p];
    }
    const int cntG = 4 << (2 * G);
    if (mode == 1) {
        const double *src = f_pool + Bc * level_offset(G) + b * (int64_t)cntG;
        for (int p = threadIdx.x; p < cntG; p += LT) {
            f_s[LdsHier<GS>::off(G) + p] = src[p];
            u_s[LdsHier<GS>::off(G) + p] = 0.0;
        }
    }
    __syncthreads();
    LdsVcycle<GS> V{a_s, u_s, f_s, mu1, mu2};
    const int nq = (mask & 1u ? 1 : 0) + (mask & 2u ? 1 : 0);
    if (mode == 1) {
        V.run(G, f_s + LdsHier<GS>::off(G));
    } else {
        for (int g = 0; g <= G; ++g) {
            const int n = 2 << g;
            double *ug = u_s + LdsHier<GS>::off(g);
            if (g == 0) {
                V.run(0, nullptr);
            } else {
                lds_prolong(u_s + LdsHier<GS>::off(g - 1), ug, n, false);
                for (int c = 0; c < mu0; ++c) V.run(g, nullptr);
            }
            if (g >= g0) {
                double qm = 0.0;
                if (mask & 1u) qm = lds_block_sum(ug, n * n, red_s) / ((double)n * n);
                if (threadIdx.x == 0) {
                    double *qb = qoi + (b * nlev + (g - g0)) * nq;
                    int q = 0;
                    if (mask & 1u) qb[q++] = qm;
                    if (mask & 2u) {
                        const int c = n / 2;
                        qb[q] = 0.25 * (ug[(c - 1) + n * (c - 1)] + ug[c + n * (c - 1)] +
                                        ug[(c - 1) + n * c] + ug[c + n * c]);
                    }
                }
            }
        }
    }
    double *dst = u_pool + Bc * level_offset(G) + b * (int64_t)cntG;
    for (int p = threadIdx.x; p < cntG; p += LT) dst[p] = u_s[LdsHier<GS>::off(G) + p];
}

inline unsigned nblocks(int64_t n) { return (unsigned)(n < 1 ? 1 : n); }

}  // namespace

// ---------------------------------------------------------------------------
bool fused_supported(int mu1, int mu2) { return mu1 >= 1 && mu1 <= 2 && mu2 >= 1 && mu2 <= 2; }

void launch_pre_tile(hipStream_t st, int mu1, const double *a, const double *f, double *u,
                     const double *uc, int n, int64_t Bc, int init, double *fc,
                     const int32_t *active)
{
    const int64_t blocks = Bc * (int64_t)(n / TILE) * (n / TILE);
    if (mu1 == 2)
        hipLaunchKernelGGL(k_pre_tile<2>, dim3(nblocks(blocks)), dim3(NT), 0, st, a, f, u, uc, n, Bc,
                           init, fc, active);
    else
        hipLaunchKernelGGL(k_pre_tile<1>, dim3(nblocks(blocks)), dim3(NT), 0, st, a, f, u, uc, n, Bc,
                           init, fc, active);
}

void launch_post_tile(hipStream_t st, int mu2, const double *a, const double *f, double *u,
                      const double *ec, int n, int64_t Bc, const int32_t *active)
{
    const int64_t blocks = Bc * (int64_t)(n / TILE) * (n / TILE);
    if (mu2 == 2)
        hipLaunchKernelGGL(k_post_tile<2>, dim3(nblocks(blocks)), dim3(NT), 0, st, a, f, u, ec, n,
                           Bc, active);
    else
        hipLaunchKernelGGL(k_post_tile<1>, dim3(nblocks(blocks)), dim3(NT), 0, st, a, f, u, ec, n,
                           Bc, active);
}

void launch_lds_mg(hipStream_t st, const double *a_pool, const double *f_pool, double *u_pool,
                   int64_t Bc, int G, int mode, int mu0, int mu1, int mu2, int g0, double *qoi,
                   int nlev, uint32_t mask, const int32_t *active)
{
    hipLaunchKernelGGL(k_lds_mg<kLdsMaxLevel>, dim3(nblocks(Bc)), dim3(LT), 0, st, a_pool, f_pool,
                       u_pool, Bc, G, mode, mu0, mu1, mu2, g0, qoi, nlev, mask, active);
}

}  // namespace mlmc
