// Host side of the MI355X MG-MLQMC library: context, argument checking, KL
// tables, the full-multigrid schedule (Section 4) driven from the host over
// batched kernels, and the estimators (Sections 2-3).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <type_traits>
#include <new>
#include <string>
#include <vector>

#include "internal.hpp"

using namespace mlmc;

struct mlmc_ctx_s {
    mlmc_config cfg{};
    int device = 0;
    int g0 = 0, Gmax = 0, nq = 0;
    bool have_lattice = false;
    bool broken = false;
    bool host_only = false;      // device < 0: tables and schedule only
    std::string err;

    // KL mode table (host)
    std::vector<int32_t> mi, mj;
    std::vector<double> theta2;

    // device memory
    uint32_t *d_z = nullptr;
    uint64_t *d_shifts = nullptr;
    double *d_basis = nullptr;   // [s][Mmax]
    // mixed mode: bf16 digit arrays [rows_pad][sp] and per-row scale exponents
    uint16_t *d_bdig[kDigits] = {};    // basis, rows = field columns (Mpad)
    uint16_t *d_ydig[kDigits] = {};    // a chunk's Y, rows = samples (chunk_pad)
    int32_t *d_bexp = nullptr, *d_yexp = nullptr;
    int sp = 0;                  // s rounded up to the matrix-core K step
    double *d_a64 = nullptr;     // mixed mode: FP64 copy of the a pool (CG operator)
    double *d_ua = nullptr;      // tile levels: pre-pass output (V-cycle type, pool elements)
    int64_t Mmax = 0;
    int64_t pool = 0;            // doubles per pool
    double *d_a = nullptr, *d_u = nullptr, *d_f = nullptr;
    double *d_fcg = nullptr;     // rtol on grids >= 64^2: second iterate buffer (FP64), r_old
                                 // and two search directions (V-cycle type) of a chunk's top level
    int64_t fcg_cells = 0;       // cells per vector (samples x top-level cells)
    double *d_part = nullptr;    // per-block partial sums of those passes
    double *d_fs = nullptr;      // per-sample CG scalars (4 doubles)
    int64_t chunk_max = 0;       // upper bound of samples per chunk
    double *d_y = nullptr;       // [chunk_max][s]
    double *d_qoi = nullptr;     // [chunk_max][num_levels][nq]
    double *d_state = nullptr;   // [max shifts][nq][num_levels][4]
    int64_t state_tuples = 0;
    double *d_rho = nullptr;
    double *d_rho_hist = nullptr;    // [chunk_max][4]: CG stagnation state (best rho, steps since)
    double *d_qpart = nullptr;       // chunk sums of the QoI mean on grids >= 128^2
    int32_t *d_active = nullptr, *d_iters = nullptr;
    double *d_w = nullptr;           // refinement modes: FP64 stage solutions (pool elements)
    int32_t *d_st_iters = nullptr, *d_st_bad = nullptr;
    double *d_st_rho = nullptr;      // per-sample refinement statistics of a chunk
    int elem = 8;                    // bytes per pool element (4 in the mixed mode)
    // pass kinds of the tile grids: [MG level g][batch class], with the
    // durations mlmc_autotune measured for them (0: not measured)
    int8_t pre_kind[kMaxMgLevels][MLMC_BATCH_CLASSES] = {};
    int8_t post_kind[kMaxMgLevels][MLMC_BATCH_CLASSES] = {};
    double pre_ms[kMaxMgLevels][MLMC_BATCH_CLASSES] = {};
    double post_ms[kMaxMgLevels][MLMC_BATCH_CLASSES] = {};
    int32_t *h_active = nullptr, *h_iters = nullptr;
    double *h_rho = nullptr;
    std::vector<void *> allocs;

    // live per-kernel timing (mlmc_profile_begin/end)
    struct {
        int kind = -1;
        std::vector<hipEvent_t> ev;   // start/stop pairs, reused across sessions
        size_t used = 0;
        int64_t launches = 0;
        double bytes = 0.0, flops = 0.0;
    } prof;
};

namespace {

thread_local std::string g_create_error;

// Device memory of mlmc_field_static, for callers that cannot allocate: one
// copy per GPU, held until the process ends.  Its host-side name is not a
// device address: kernels get the address resolved per device at context
// creation (static_scratch_ptr), never the symbol.
constexpr size_t kStaticScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_ptr;      // device -> address of its copy

// resolve (once per device, with that device current) the device address of
// the static scratch; "" on success
std::string resolve_static_scratch(int device)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr.count(device)) return "";
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
    g_scratch_ptr[device] = p;
    return "";
}

void *static_scratch_ptr(int device)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    return it == g_scratch_ptr.end() ? nullptr : it->second;
}

const char *kStatusText[] = {"ok", "invalid argument", "out of device memory", "HIP error",
                             "not converged", "context unusable"};

#define HIPCHK(ctx, call)                                                            \
    do {                                                                             \
        hipError_t _e = (call);                                                      \
        if (_e != hipSuccess) {                                                      \
            (ctx)->err = std::string(#call) + ": " + hipGetErrorString(_e);          \
            (ctx)->broken = true;                                                    \
            return MLMC_E_HIP;                                                       \
        }                                                                            \
    } while (0)

mlmc_status inval(mlmc_ctx ctx, const char *msg)
{
    if (ctx)
        ctx->err = msg;
    return MLMC_E_INVAL;
}

int ilog2_exact(int v)
{
    int r = 0;
    while ((1 << r) < v) ++r;
    return (1 << r) == v ? r : -1;
}

// ---- Section 5: eigenpairs of exp(-|x-t|/lam) on [0,1] ---------------------
// Characteristic equation F(w) = (lam^2 w^2 - 1) sin w - 2 lam w cos w = 0 with
// one root in each ((k-1) pi, k pi); found by Newton's method kept inside a
// shrinking sign bracket.
double char_eq(double lam, double w, double *deriv)
{
    double sw = std::sin(w), cw = std::cos(w), l2w2 = lam * lam * w * w;
    *deriv = (2.0 * lam * lam * w + 2.0 * lam * w) * sw + (l2w2 - 1.0 - 2.0 * lam) * cw;
    return (l2w2 - 1.0) * sw - 2.0 * lam * w * cw;
}

double kl_root(double lam, int k)
{
    const double pi = 3.14159265358979323846;
    double lo = (k - 1) * pi, hi = k * pi;
    const bool lo_pos = (k % 2 == 0);   // F just above (k-1) pi: < 0 for k = 1, sign (-1)^k else
    double w = 0.5 * (lo + hi);
    for (int it = 0; it < 200; ++it) {
        double d;
        double f = char_eq(lam, w, &d);
        if (f == 0.0)
            return w;
        if ((f > 0.0) == lo_pos) lo = w; else hi = w;
        double wn = (d != 0.0) ? w - f / d : 0.5 * (lo + hi);
        if (!(wn > lo && wn < hi))
            wn = 0.5 * (lo + hi);
        if (std::fabs(wn - w) <= 2.0 * std::nextafter(w, 2.0 * hi) - 2.0 * w || hi <= std::nextafter(lo, hi))
            return wn;
        w = wn;
    }
    return w;
}

double kl_eigenvalue(double lam, double w) { return 2.0 * lam / (1.0 + lam * lam * w * w); }

double kl_eigenfunction(double lam, double w, double x)
{
    return (std::sin(w * x) + lam * w * std::cos(w * x)) /
           std::sqrt(lam + 0.5 * (1.0 + lam * lam * w * w));
}

int64_t field_size_g(int G) { return level_offset(G + 1); }

void free_all(mlmc_ctx c)
{
    for (hipEvent_t e : c->prof.ev) (void)hipEventDestroy(e);
    c->prof.ev.clear();
    for (void *p : c->allocs) (void)hipFree(p);
    c->allocs.clear();
    if (c->h_active) (void)hipHostFree(c->h_active);
    if (c->h_iters) (void)hipHostFree(c->h_iters);
    if (c->h_rho) (void)hipHostFree(c->h_rho);
    c->h_active = nullptr;
    c->h_iters = nullptr;
    c->h_rho = nullptr;
}

template <typename T>
hipError_t dev_alloc(mlmc_ctx c, T **p, int64_t count)
{
    *p = nullptr;
    if (count <= 0)
        return hipSuccess;
    void *v = nullptr;
    hipError_t e = hipMalloc(&v, (size_t)count * sizeof(T));
    if (e == hipSuccess) {
        c->allocs.push_back(v);
        *p = (T *)v;
    }
    return e;
}

// samples per chunk for finest MLMC level k
int64_t chunk_capacity(mlmc_ctx c, int k)
{
    int G = c->g0 + k;
    int64_t cap = c->pool / field_size_g(G);
    if (c->cfg.rtol > 0.0 && G > kLdsMaxLevel)
        cap = std::min(cap, c->fcg_cells / level_cells(G));
    return std::max<int64_t>(1, std::min(cap, c->chunk_max));
}

}  // namespace

int64_t mlmc::level_capacity(mlmc_ctx c, int k) { return chunk_capacity(c, k); }

namespace {

mlmc_status check_points(mlmc_ctx c, const mlmc_points *p, int64_t *B, int64_t *npts, int *nsh)
{
    if (!p)
        return inval(c, "points is NULL");
    if (p->level < 0 || p->level >= c->cfg.num_levels)
        return inval(c, "points.level out of range");
    if (p->n_begin < 0 || p->n_end < p->n_begin)
        return inval(c, "points range must satisfy 0 <= n_begin <= n_end");
    if (p->kind == MLMC_POINTS_LATTICE) {
        if (!c->have_lattice)
            return inval(c, "lattice points need genvec and shifts at create");
        if (p->n_end > ((int64_t)1 << 32))
            return inval(c, "lattice index beyond 2^32");
        if (p->shift_begin < 0 || p->shift_end <= p->shift_begin ||
            p->shift_end > c->cfg.num_shifts)
            return inval(c, "shift range out of [0, num_shifts)");
    } else if (p->kind == MLMC_POINTS_EXPLICIT) {
        if (p->shift_end - p->shift_begin != 1)
            return inval(c, "explicit points take exactly one replica (shift_end - shift_begin == 1)");
        if (!p->y_dev && p->n_end > p->n_begin)
            return inval(c, "explicit points need y_dev");
    } else {
        return inval(c, "unknown points.kind");
    }
    *npts = p->n_end - p->n_begin;
    *nsh = p->shift_end - p->shift_begin;
    *B = *npts * *nsh;
    return MLMC_OK;
}

// y of samples [b0, b0+Bc) of a point set, on the device
const double *chunk_y(mlmc_ctx c, hipStream_t st, const mlmc_points *p, int64_t npts, int64_t b0,
                      int64_t Bc, uint64_t *x_out)
{
    if (p->kind == MLMC_POINTS_EXPLICIT)
        return p->y_dev + b0 * c->cfg.s;
    launch_points(st, c->d_z, c->d_shifts, c->cfg.s, c->cfg.num_shifts, p->level, p->shift_begin,
                  p->n_begin, npts, b0, Bc, x_out, c->d_y);
    return c->d_y;
}

Hier make_hier(mlmc_ctx c, int G, int64_t Bc)
{
    Hier h;
    h.G = G;
    h.Bc = Bc;
    for (int g = 0; g <= G; ++g) {
        int64_t off = Bc * level_offset(g);
        h.a[g] = c->d_a + off;
        h.u[g] = c->d_u + off;
        h.f[g] = c->d_f + off;
    }
    return h;
}

// Brackets one launch with events when its kind is being profiled.
struct ProfScope {
    mlmc_ctx c;
    hipStream_t st;
    bool on = false;
    size_t idx = 0;
    ProfScope(mlmc_ctx c_, hipStream_t st_, int kind, double bytes, double flops) : c(c_), st(st_)
    {
        if (c->prof.kind != kind) return;
        idx = c->prof.used;
        while (c->prof.ev.size() < 2 * (idx + 1)) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return;
            c->prof.ev.push_back(e);
        }
        on = hipEventRecord(c->prof.ev[2 * idx], st) == hipSuccess;
        if (!on) return;
        c->prof.launches++;
        c->prof.bytes += bytes;
        c->prof.flops += flops;
    }
    ~ProfScope()
    {
        if (!on) return;
        (void)hipEventRecord(c->prof.ev[2 * idx + 1], st);
        c->prof.used++;
    }
};

// ---- Section 4: correction scheme / V-cycle / FMG --------------------------
struct Trace {
    std::vector<int32_t> lev, mark;
    void visit(int g)
    {
        if (!lev.empty() && lev.back() == g) return;
        lev.push_back(g);
        mark.push_back(0);
    }
    void record()
    {
        if (!mark.empty()) mark.back() = 1;
    }
};

struct Runner {
    mlmc_ctx c;
    hipStream_t st;
    Hier h;
    Trace *tr;                 // dry run when non-null
    const int32_t *active;     // refinement: skip converged samples

    double cells(int n) const { return (double)h.Bc * n * n; }

    void smooth(int g, const double *f, double *x, int colour)
    {
        const int n = 2 << g;
        ProfScope ps(c, st, MLMC_KERNEL_SMOOTH, 8.0 * cells(n) * (f ? 2.5 : 2.0), 0.0);
        launch_rbgs(st, h.a[g], f, x, n, h.Bc, colour, active);
    }
    void restrict_to(int g, const double *f, const double *x)
    {
        const int n = 2 << g;
        ProfScope ps(c, st, MLMC_KERNEL_RESTRICT, 8.0 * cells(n) * ((f ? 3.0 : 2.0) + 0.5), 0.0);
        launch_resid_restrict(st, h.a[g], f, x, n, h.Bc, h.f[g - 1], h.u[g - 1], active);
    }
    void prolong(int g, const double *ec, double *x, int add, const int32_t *act)
    {
        const int n = 2 << g;
        ProfScope ps(c, st, MLMC_KERNEL_PROLONG, 8.0 * cells(n) * (add ? 2.25 : 1.25), 0.0);
        launch_prolong(st, ec, x, n, h.Bc, add, act);
    }
    void coarse(const double *f, double *x)
    {
        ProfScope ps(c, st, MLMC_KERNEL_COARSE, 8.0 * h.Bc * 4 * (f ? 3 : 2), 0.0);
        launch_coarse_solve(st, h.a[0], f, x, h.Bc, active);
    }

    // V(mu1,mu2) on level g for the iterate x[g] (x = u pool below the top).
    // top_x / top_f override the iterate and rhs of level g (nullptr f = 1).
    void vcycle(int g, double *top_x, const double *top_f)
    {
        if (tr) tr->visit(g);
        double *x = top_x ? top_x : h.u[g];
        const double *f = top_x ? top_f : h.f[g];
        if (g == 0) {
            if (!tr) coarse(f, x);
            return;
        }
        for (int it = 0; it < c->cfg.mu1; ++it) {
            if (!tr) {
                smooth(g, f, x, 0);
                smooth(g, f, x, 1);
            }
        }
        if (!tr) restrict_to(g, f, x);
        vcycle(g - 1, nullptr, nullptr);
        if (tr) tr->visit(g);
        if (!tr) prolong(g, h.u[g - 1], x, 1, active);
        for (int it = 0; it < c->cfg.mu2; ++it) {
            if (!tr) {
                smooth(g, f, x, 1);
                smooth(g, f, x, 0);
            }
        }
    }
};

struct StageStats {
    int max_iters = 0;
    double max_rho = -1.0;
    int64_t noconv = 0;            // samples with any stage stopped above rtol
    std::vector<uint8_t> bad;      // per sample of the current chunk
    int32_t *sample_bad = nullptr; // optional host [B]: per-sample flag of the whole call
    double *sample_rho = nullptr;  // optional host [B]: per-sample largest final ratio
    int64_t b0 = 0;                // first sample of the current chunk
};

// FMG for one chunk; qoi rows of the chunk at qoi [Bc][k+1][nq].
mlmc_status run_fmg(mlmc_ctx c, hipStream_t st, const Hier &h, int k, double *qoi, Trace *tr,
                    StageStats *stats)
{
    const int G = h.G, g0 = c->g0, nlev = k + 1;
    Runner R{c, st, h, tr, nullptr};
    if (stats) stats->bad.assign((size_t)h.Bc, 0);
    if (tr)
        for (int g = G; g > 0; --g) tr->visit(g);   // initial descent: set-up
    // stage 0: exact solve with f = 1 on the 2x2 grid
    R.vcycle(0, h.u[0], nullptr);
    if (tr) tr->record();
    if (!tr && g0 == 0) {
        ProfScope ps(c, st, MLMC_KERNEL_QOI, 8.0 * h.Bc * 4, 0.0);
        launch_qoi(st, h.u[0], 2, h.Bc, qoi, nlev, 0, c->cfg.qoi_mask, c->d_qpart);
    }
    for (int g = 1; g <= G; ++g) {
        const int n = 2 << g;
        if (tr) tr->visit(g);
        // nested iteration: interpolate the previous stage's solution
        if (!tr) R.prolong(g, h.u[g - 1], h.u[g], 0, nullptr);
        // fixed cycles (rtol mode needs the fused passes, checked at create)
        for (int cyc = 0; cyc < c->cfg.mu0; ++cyc) R.vcycle(g, h.u[g], nullptr);
        if (stats) stats->max_iters = std::max(stats->max_iters, c->cfg.mu0);
        if (tr) tr->record();
        if (!tr && g >= g0) {
            ProfScope ps(c, st, MLMC_KERNEL_QOI, 8.0 * R.cells(n), 0.0);
            launch_qoi(st, h.u[g], n, h.Bc, qoi, nlev, g - g0, c->cfg.qoi_mask, c->d_qpart);
        }
    }
    if (stats)
        for (uint8_t v : stats->bad) stats->noconv += v;
    return MLMC_OK;
}

// ---- pass kinds of the tile grids (mlmc_autotune) --------------------------
// batch class of a chunk of Bc samples: 4^(c-1) < Bc <= 4^c, c = 0 for one
int batch_class(int64_t Bc)
{
    int c = 0;
    while (c + 1 < MLMC_BATCH_CLASSES && ((int64_t)1 << (2 * c)) < Bc) ++c;
    return c;
}
// top MG level of the LDS-resident grids; the tile grids lie above it
int lds_top(mlmc_ctx c) { return c->cfg.rtol > 0.0 ? kLdsMaxLevel : kLdsMaxLevelFixed; }
bool kind_allowed(mlmc_ctx c, int g, int kind)
{
    if (kind == kTile32 || kind == kTile16) return true;
    // the row-streaming passes exist for FP64 and FP32 V-cycles
    return kind == kStream && stream_supported(2 << g);
}

// Defaults: the choices mlmc_autotune made on MI355X for the FP64 s = 100
// workload (grids 32^2 .. 256^2) and for both V-cycle types of the s = 400
// workloads (64^2 .. 2048^2), batch classes up to 16384 samples, as a rule in
// the batch class c, the number of 32 x 32 tiles a pass covers, t = 4^c
// (n/32)^2, and the lanes the row-streaming passes would run, 4^c n/2: up to
// 256 tiles (one per CU or fewer) 16 x 16 tiles, which give four times the
// workgroups; 32 x 32 tiles otherwise; the row-streaming passes take both
// passes once they have 131072 lanes and t >= 65536 (FP64 from t = 16384 on
// 32^2 and 64^2, where a workgroup packs 4 or 2 samples) and the smallest
// chunk of the class still gives every CU a workgroup (a streaming workgroup
// holds one sample from 128^2 up, so 128 samples of 2048^2 streamed leave
// half the CUs idle), in FP64 up to 1024^2 (the 2048^2 FP64
// workgroup of 1024 lanes spills registers and measured slower than tiles).
void default_tuning(mlmc_ctx c)
{
    const bool fp64 = c->cfg.precision == MLMC_FP64;
    for (int g = 0; g < kMaxMgLevels; ++g) {
        const int n = 2 << g;
        const int64_t side = std::max(1, n / 32);
        const int64_t spb = n >= 128 ? 1 : 64 / (n / 2);
        const bool stream = kind_allowed(c, g, kStream) && (!fp64 || n <= 1024);
        for (int cl = 0; cl < MLMC_BATCH_CLASSES; ++cl) {
            const int64_t tiles = ((int64_t)1 << (2 * cl)) * side * side;
            const int64_t lanes = ((int64_t)1 << (2 * cl)) * (n / 2);
            const int64_t smallest = cl == 0 ? 1 : ((int64_t)1 << (2 * (cl - 1))) + 1;
            const int8_t tile = tiles <= 256 ? kTile16 : kTile32;
            const bool big = (tiles >= 65536 || (fp64 && n <= 64 && tiles >= 16384)) &&
                             lanes >= 131072 && smallest / spb >= 256;
            c->pre_kind[g][cl] = stream && big ? kStream : tile;
            c->post_kind[g][cl] = stream && big ? kStream : tile;
        }
    }
}

// ---- fused schedule: LDS-resident grids (<= 16^2 fixed, <= 32^2 rtol), tile passes above
// Typed views of one chunk's pools: a, u, f in the V-cycle type T; w holds the
// FP64 stage solutions of the refinement modes.
template <typename T>
struct HierT {
    int G = 0;
    int64_t Bc = 0;
    T *a[kMaxMgLevels] = {};
    T *u[kMaxMgLevels] = {};
    T *f[kMaxMgLevels] = {};
    double *w[kMaxMgLevels] = {};
    const double *a64[kMaxMgLevels] = {};   // FP64 coefficients (a itself when T = double)
    T *ua[kMaxMgLevels] = {};               // pre-pass output of a tile level
};

template <typename T>
HierT<T> make_hier_t(mlmc_ctx c, int G, int64_t Bc)
{
    HierT<T> h;
    h.G = G;
    h.Bc = Bc;
    for (int g = 0; g <= G; ++g) {
        const int64_t off = Bc * level_offset(g);
        h.a[g] = (T *)c->d_a + off;
        h.u[g] = (T *)c->d_u + off;
        h.f[g] = (T *)c->d_f + off;
        h.w[g] = c->d_w ? c->d_w + off : nullptr;
        h.a64[g] = sizeof(T) == sizeof(double) ? (const double *)h.a[g]
                                               : (c->d_a64 ? c->d_a64 + off : nullptr);
        h.ua[g] = c->d_ua ? (T *)c->d_ua + off : nullptr;
    }
    return h;
}

template <typename T>
struct FusedRunner {
    mlmc_ctx c;
    hipStream_t st;
    HierT<T> h;
    int Gs;
    static constexpr double W = sizeof(T);
    // samples the masked passes work on (the active ones of a refinement
    // step; -1: the whole chunk), for the profiled byte counts
    int64_t nact = -1;

    double samples() const { return (double)(nact >= 0 ? nact : h.Bc); }
    double cells(int n) const { return samples() * n * n; }

    // one V-cycle on the LDS-resident levels <= Gs (zero guess, f from the pool)
    void lds_vcycle(const int32_t *active)
    {
        const int n = 2 << Gs;
        ProfScope ps(c, st, MLMC_KERNEL_LDS, W * samples() * level_offset(Gs + 1) + W * cells(n) * 2.0, 0.0);
        launch_lds_vcycle<T>(st, h.a[0], h.f[0], h.u[0], h.Bc, Gs, c->cfg.mu1, c->cfg.mu2, active);
    }

    // V(mu1,mu2) at level g > Gs.  init_top: 0 read u, 1 zero, 2 interpolate
    // the previous stage's solution.  top_f nullptr means f = 1.  On every
    // tile level the pre pass writes ua and the post pass reads ua and writes
    // u (top_u on the top level), so no pass reads the array it writes.
    void vcycle(int g, T *top_u, int init_top, const T *top_f, const int32_t *active)
    {
        // the pass kinds of the samples the masked passes work on: in a
        // refinement step only the active ones have workgroups with work, so
        // a chunk whose active set has shrunk takes the kinds of that smaller
        // class (every kind gives the same bits)
        const int cls = batch_class(nact >= 0 ? nact : h.Bc);
        for (int l = g; l > Gs; --l) {
            const int n = 2 << l;
            const int init = (l == g) ? init_top : 1;
            const T *f = (l == g) ? top_f : h.f[l];
            T *u = (l == g) ? top_u : h.u[l];
            double words = 1.0 + (init == 0 ? 1.0 : 0.0) + (f ? 1.0 : 0.0) + 1.0 + 0.25 +
                           (init == 2 ? 0.25 : 0.0);
            ProfScope ps(c, st, MLMC_KERNEL_PRE, W * cells(n) * words, 0.0);
            const int kind = c->pre_kind[l][cls];
            if (kind == kStream) {
                launch_pre_stream<T>(st, c->cfg.mu1, h.a[l], f, u, h.ua[l], h.u[l - 1], n, h.Bc,
                                     init, h.f[l - 1], active);
                continue;
            }
            launch_pre_tile<T>(st, kind, c->cfg.mu1, h.a[l], f, u, h.ua[l], h.u[l - 1], n, h.Bc,
                               init, h.f[l - 1], active);
        }
        lds_vcycle(active);
        for (int l = Gs + 1; l <= g; ++l) {
            const int n = 2 << l;
            const T *f = (l == g) ? top_f : h.f[l];
            T *u = (l == g) ? top_u : h.u[l];
            ProfScope ps(c, st, MLMC_KERNEL_POST, W * cells(n) * (3.25 + (f ? 1.0 : 0.0)), 0.0);
            const int kind = c->post_kind[l][cls];
            if (kind == kStream) {
                launch_post_stream<T>(st, c->cfg.mu2, h.a[l], f, h.ua[l], u, h.u[l - 1], n, h.Bc,
                                      active);
                continue;
            }
            launch_post_tile<T>(st, kind, c->cfg.mu2, h.a[l], f, h.ua[l], u, h.u[l - 1], n, h.Bc,
                                active);
        }
    }
};

bool use_fused(mlmc_ctx c) { return fused_supported(c->cfg.mu1, c->cfg.mu2); }

// Fixed mu0 cycles per stage (FP64).
mlmc_status run_fmg_fixed(mlmc_ctx c, hipStream_t st, int G, int64_t Bc, int k, double *qoi,
                          StageStats *stats)
{
    const int nlev = k + 1;
    FusedRunner<double> R{c, st, make_hier_t<double>(c, G, Bc), std::min(G, kLdsMaxLevelFixed)};
    {
        const int n = 2 << R.Gs;
        ProfScope ps(c, st, MLMC_KERNEL_LDS, 8.0 * Bc * level_offset(R.Gs + 1) + 8.0 * R.cells(n), 0.0);
        launch_lds_fmg_fixed(st, c->d_a, c->d_u, Bc, R.Gs, c->cfg.mu0, c->cfg.mu1, c->cfg.mu2,
                             c->g0, qoi, nlev, c->cfg.qoi_mask);
    }
    for (int g = R.Gs + 1; g <= G; ++g) {
        const int n = 2 << g;
        for (int cyc = 0; cyc < c->cfg.mu0; ++cyc)
            R.vcycle(g, R.h.u[g], cyc == 0 ? 2 : 0, nullptr, nullptr);
        if (g >= c->g0) {
            ProfScope ps(c, st, MLMC_KERNEL_QOI, 8.0 * R.cells(n), 0.0);
            launch_qoi(st, R.h.u[g], n, Bc, qoi, nlev, g - c->g0, c->cfg.qoi_mask, c->d_qpart);
        }
    }
    if (stats) stats->max_iters = std::max(stats->max_iters, c->cfg.mu0);
    return MLMC_OK;
}

// Refinement to rtol with an FP64 residual and V-cycles of type T (double:
// FP64 path, float: mixed path).  Per stage: u64 = P u64_prev; repeat
// { r = 1 - A u64 ; stop at rtol or max_iters ; e = V_T(0; r) ; u64 += e }.
template <typename T>
mlmc_status run_fmg_refine(mlmc_ctx c, hipStream_t st, int G, int64_t Bc, int k, double *qoi,
                           StageStats *stats)
{
    const int nlev = k + 1;
    FusedRunner<T> R{c, st, make_hier_t<T>(c, G, Bc), std::min(G, kLdsMaxLevel)};
    const auto &h = R.h;
    {
        const int n = 2 << R.Gs;
        // a (and its FP64 copy in the mixed mode) of the LDS levels read, x of the top one written
        const double wa = R.W + (sizeof(T) == sizeof(double) ? 0.0 : 8.0);
        ProfScope ps(c, st, MLMC_KERNEL_LDS, wa * Bc * level_offset(R.Gs + 1) + 8.0 * R.cells(n), 0.0);
        launch_lds_fmg_refine<T>(st, h.a[0], h.a64[0], c->d_w, Bc, R.Gs, c->cfg.mu1, c->cfg.mu2,
                                 c->cfg.rtol,
                                 c->cfg.max_iters, c->g0, qoi, nlev, c->cfg.qoi_mask, c->d_st_iters,
                                 c->d_st_rho, c->d_st_bad);
    }
    for (int g = R.Gs + 1; g <= G; ++g) {
        const int n = 2 << g;
        {
            ProfScope ps(c, st, MLMC_KERNEL_PROLONG, 8.0 * R.cells(n) * 1.25, 0.0);
            launch_prolong(st, h.w[g - 1], h.w[g], n, Bc, 0, nullptr);
        }
        // flexible CG on level g from x = P x_prev, preconditioner z = V(0; r)
        const int64_t cells = Bc * (int64_t)n * n;
        FcgBufs<T> v;
        v.a = h.a[g];
        v.a64 = h.a64[g];
        v.z = h.u[g];
        v.f = h.f[g];
        v.x0 = h.w[g];
        v.x1 = c->d_fcg;
        v.fo = (T *)(c->d_fcg + cells);
        v.p0 = v.fo + cells;
        v.p1 = v.p0 + cells;
        v.part = c->d_part;
        v.fs = c->d_fs;
        v.rho = c->d_rho;
        v.hist = c->d_rho_hist;
        v.active = c->d_active;
        v.iters = c->d_iters;
        const double vec = R.cells(n);   // cells of all samples of the chunk
        {
            // a (FP64), x read; f written
            ProfScope ps(c, st, MLMC_KERNEL_REFINE, vec * (16.0 + R.W), 0.0);
            launch_fcg_resid<T>(st, h.a64[g], h.w[g], n, Bc, h.f[g], c->d_part);
        }
        launch_fcg_fin_rho(st, c->d_part, n, Bc, c->d_rho, c->d_rho_hist, c->d_active, c->d_iters,
                           c->cfg.rtol, c->cfg.max_iters, 1);
        for (int step = 1;; ++step) {
            HIPCHK(c, hipMemcpyAsync(c->h_active, c->d_active, sizeof(int32_t) * Bc,
                                     hipMemcpyDeviceToHost, st));
            HIPCHK(c, hipStreamSynchronize(st));
            int64_t nact = 0;
            for (int64_t b = 0; b < Bc; ++b) nact += c->h_active[b];
            if (nact == 0) break;
            // every active sample is at this step; its residual r_{step-1}
            // is in f for odd steps and in fo for even ones
            R.nact = nact;
            R.vcycle(g, h.u[g], 1, (step & 1) ? v.f : v.fo, c->d_active);
            {
                // per cell of the active samples: dots: z, r, r_old read; p:
                // a, z, p_prev read, p written; x: a (FP64), x_prev, p read,
                // x and r written (no r_old or p_prev at the first step)
                ProfScope ps(c, st, MLMC_KERNEL_REFINE,
                             R.cells(n) * (24.0 + (step > 1 ? 9.0 : 7.0) * R.W), 0.0);
                launch_fcg_step<T>(st, v, n, Bc, c->cfg.rtol, c->cfg.max_iters);
            }
            R.nact = -1;
        }
        launch_fcg_copyback(st, h.w[g], v.x1, n, Bc, c->d_iters);
        launch_refine_stats(st, c->d_iters, c->d_rho, Bc, c->cfg.rtol, c->d_st_iters, c->d_st_rho,
                            c->d_st_bad);
        if (g >= c->g0) {
            ProfScope ps(c, st, MLMC_KERNEL_QOI, 8.0 * R.cells(n), 0.0);
            launch_qoi(st, h.w[g], n, Bc, qoi, nlev, g - c->g0, c->cfg.qoi_mask, c->d_qpart);
        }
    }
    if (stats) {
        HIPCHK(c, hipMemcpyAsync(c->h_iters, c->d_st_iters, sizeof(int32_t) * Bc,
                                 hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipMemcpyAsync(c->h_rho, c->d_st_rho, sizeof(double) * Bc, hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipMemcpyAsync(c->h_active, c->d_st_bad, sizeof(int32_t) * Bc,
                                 hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        for (int64_t b = 0; b < Bc; ++b) {
            stats->max_iters = std::max(stats->max_iters, (int)c->h_iters[b]);
            stats->max_rho = std::max(stats->max_rho, c->h_rho[b]);
            stats->noconv += c->h_active[b] != 0;
            if (stats->sample_bad) stats->sample_bad[stats->b0 + b] = c->h_active[b] != 0;
            if (stats->sample_rho) stats->sample_rho[stats->b0 + b] = c->h_rho[b];
        }
    }
    return MLMC_OK;
}

// Neumaier summation on the host
struct HostSum {
    double s = 0.0, c = 0.0;
    void add(double v)
    {
        double t = s + v;
        if (std::fabs(s) >= std::fabs(v)) c += (s - t) + v; else c += (v - t) + s;
        s = t;
    }
    double value() const { return s + c; }
};

}  // namespace

// ===========================================================================
extern "C" {

const char *mlmc_status_str(mlmc_status st)
{
    int i = -(int)st;
    if (i < 0 || i > 5) return "unknown status";
    return kStatusText[i];
}

const char *mlmc_last_error(mlmc_ctx ctx)
{
    if (!ctx) return g_create_error.c_str();
    return ctx->err.c_str();
}

}  // extern "C"

// A context whose read-only tables (KL basis or its digits, generating vector,
// shifts) are those of `parent` when parent is not NULL: same device and the
// same field, level and lattice configuration; the parent must outlive it.
mlmc_status mlmc::create_ctx(const mlmc_config *cfg, int device, mlmc_ctx parent, mlmc_ctx *out)
{
    g_create_error.clear();
    if (!out) { g_create_error = "out is NULL"; return MLMC_E_INVAL; }
    *out = nullptr;
    if (!cfg) { g_create_error = "cfg is NULL"; return MLMC_E_INVAL; }
    const mlmc_config &c = *cfg;
    auto bad = [](const char *m) { g_create_error = m; return MLMC_E_INVAL; };
    int lg = ilog2_exact(c.n0);
    if (c.n0 < 2 || lg < 0) return bad("n0 must be a power of two >= 2");
    if (c.num_levels < 1) return bad("num_levels must be >= 1");
    int g0 = lg - 1, Gmax = g0 + c.num_levels - 1;
    if (Gmax >= kMaxMgLevels) return bad("finest grid beyond 4096 cells per side");
    if (c.s < 1 || c.s > 4096) return bad("s must be in 1..4096");
    if (!(c.corr_len > 0.0) || !std::isfinite(c.corr_len)) return bad("corr_len must be > 0");
    if (!(c.sigma2 >= 0.0) || !std::isfinite(c.sigma2)) return bad("sigma2 must be >= 0");
    if (c.mu1 < 0 || c.mu2 < 0 || c.mu1 + c.mu2 < 1) return bad("need mu1, mu2 >= 0 and mu1 + mu2 >= 1");
    if (!(c.rtol >= 0.0) || !std::isfinite(c.rtol)) return bad("rtol must be >= 0");
    if (c.rtol == 0.0 && c.mu0 < 1) return bad("mu0 must be >= 1 in fixed-cycle mode");
    if (c.rtol > 0.0 && c.max_iters < 1) return bad("max_iters must be >= 1 when rtol > 0");
    if (c.precision != MLMC_FP64 && c.precision != MLMC_MIXED) return bad("unknown precision");
    if (c.precision == MLMC_MIXED && !(c.rtol > 0.0))
        return bad("MLMC_MIXED refines an FP64 residual: it needs rtol > 0");
    if (c.rtol > 0.0 && !fused_supported(c.mu1, c.mu2))
        return bad("rtol > 0 supports mu1, mu2 in {1, 2}");
    if (c.qoi_mask == 0 || (c.qoi_mask & ~3u)) return bad("qoi_mask must be a non-empty subset of {MEAN, CENTER}");
    if (c.max_batch < 1) return bad("max_batch must be >= 1");
    bool lattice = c.genvec && c.shifts;
    if (lattice && c.num_shifts < 1) return bad("num_shifts must be >= 1 with shifts");
    if (c.field_kind != MLMC_FIELD_SEPARABLE_EXP && c.field_kind != MLMC_FIELD_MATERN)
        return bad("unknown field_kind");
    const bool matern = c.field_kind == MLMC_FIELD_MATERN;
    const int nq_nodes = c.nystrom_q == 0 ? 32 : c.nystrom_q;
    if (matern) {
        if (!(c.nu > 0.0 && c.nu <= 8.0)) return bad("Matern nu must be in (0, 8]");
        if (nq_nodes < 4 || nq_nodes > 96) return bad("nystrom_q must be 0 or in 4..96");
        if (c.s > nq_nodes * nq_nodes) return bad("s exceeds nystrom_q^2 Nystrom eigenpairs");
        if (device < 0) return bad("the Matern field's Nystrom eigensolve needs a device");
    }
    if (parent) {
        const mlmc_config &q = parent->cfg;
        if (parent->host_only || parent->device != device || q.n0 != c.n0 ||
            q.num_levels != c.num_levels || q.s != c.s || q.corr_len != c.corr_len ||
            q.sigma2 != c.sigma2 || q.precision != c.precision || q.field_kind != c.field_kind ||
            (matern && (q.nu != c.nu || q.nystrom_q != c.nystrom_q)) ||
            parent->have_lattice != lattice || (lattice && q.num_shifts != c.num_shifts))
            return bad("parent context has another field, level or lattice configuration");
    }

    mlmc_ctx ctx = new (std::nothrow) mlmc_ctx_s();
    if (!ctx) { g_create_error = "host allocation failed"; return MLMC_E_NOMEM; }
    ctx->cfg = c;
    if (matern) ctx->cfg.nystrom_q = nq_nodes;
    ctx->cfg.genvec = nullptr;
    ctx->cfg.shifts = nullptr;
    if (!lattice) ctx->cfg.num_shifts = std::max(ctx->cfg.num_shifts, 1);
    ctx->device = device;
    ctx->g0 = g0;
    ctx->Gmax = Gmax;
    ctx->nq = (c.qoi_mask & 1u ? 1 : 0) + (c.qoi_mask & 2u ? 1 : 0);
    ctx->have_lattice = lattice;

    auto fail = [&](mlmc_status s) {
        g_create_error = ctx->err;
        free_all(ctx);
        delete ctx;
        return s;
    };
#define CHK(call)                                                                    \
    do {                                                                             \
        hipError_t _e = (call);                                                      \
        if (_e != hipSuccess) {                                                      \
            ctx->err = std::string(#call) + ": " + hipGetErrorString(_e);            \
            return fail(_e == hipErrorOutOfMemory ? MLMC_E_NOMEM : MLMC_E_HIP);      \
        }                                                                            \
    } while (0)

    ctx->host_only = device < 0;
    if (!ctx->host_only) {
        CHK(hipSetDevice(device));
        const std::string serr = resolve_static_scratch(device);
        if (!serr.empty()) {
            ctx->err = serr;
            return fail(MLMC_E_HIP);
        }
    }

    // KL mode table: the s largest products theta_i theta_j (i, j <= s),
    // descending, exact ties ordered by i ascending (separable kernel; the
    // Matern eigenvalues come from the Nystrom eigensolve below).
    const int s = c.s;
    const double lam = c.corr_len;
    const int s1 = matern ? 0 : s;          // 1-D eigenpairs needed
    std::vector<double> w(s1), th(s1);
    for (int k = 1; k <= s1; ++k) {
        w[k - 1] = kl_root(lam, k);
        th[k - 1] = kl_eigenvalue(lam, w[k - 1]);
    }
    struct Pair { double t; int32_t i, j; };
    std::vector<Pair> pairs;
    pairs.reserve((size_t)s1 * s1);
    for (int i = 1; i <= s1; ++i)
        for (int j = 1; j <= s1; ++j) pairs.push_back({th[i - 1] * th[j - 1], i, j});
    std::partial_sort(pairs.begin(), pairs.begin() + s1, pairs.end(), [](const Pair &a, const Pair &b) {
        if (a.t != b.t) return a.t > b.t;
        if (a.i != b.i) return a.i < b.i;
        return a.j < b.j;
    });
    ctx->mi.assign(s, 0);
    ctx->mj.assign(s, 0);
    ctx->theta2.assign(s, 0.0);
    int pmax = 1;
    for (int m = 0; m < s1; ++m) {
        ctx->mi[m] = pairs[m].i;
        ctx->mj[m] = pairs[m].j;
        ctx->theta2[m] = pairs[m].t;
        pmax = std::max(pmax, std::max(pairs[m].i, pairs[m].j));
    }
    std::vector<Pair>().swap(pairs);
    const double sigma = std::sqrt(c.sigma2);
    std::vector<double> coef(s1);
    for (int m = 0; m < s1; ++m)
        coef[m] = sigma * std::sqrt(th[ctx->mi[m] - 1]) * std::sqrt(th[ctx->mj[m] - 1]);
    // 1-D eigenfunctions at the cell centres of every level
    std::vector<int64_t> psi_off(Gmax + 2);
    std::vector<double> psi;
    for (int g = 0; g <= Gmax && !matern; ++g) {
        int n = 2 << g;
        psi_off[g] = (int64_t)psi.size();
        for (int k = 0; k < pmax; ++k)
            for (int cc = 0; cc < n; ++cc)
                psi.push_back(kl_eigenfunction(lam, w[k], (cc + 0.5) / n));
    }

    ctx->Mmax = field_size_g(Gmax);
    default_tuning(ctx);
    if (ctx->host_only) {
        *out = ctx;
        return MLMC_OK;
    }
    // workspace sizes
    ctx->pool = c.max_batch * ctx->Mmax;          // elements per pool
    ctx->elem = c.precision == MLMC_MIXED ? 4 : 8;
    ctx->chunk_max = std::max<int64_t>(c.max_batch, 65536);
    const int64_t wcap = c.rtol > 0.0 ? ctx->pool : 0;
    if (c.rtol > 0.0 && Gmax > kLdsMaxLevel) ctx->fcg_cells = c.max_batch * level_cells(Gmax);
    // partial sums: 4 doubles per 1024-cell block, blocks of at most chunk_max samples
    const int64_t parts = ctx->fcg_cells > 0 ? fcg_partials(64, ctx->chunk_max) +
                                                   4 * (ctx->fcg_cells / 1024 + 1)
                                             : 0;
    int nshift_max = std::max(ctx->cfg.num_shifts, 1);
    ctx->state_tuples = (int64_t)nshift_max * ctx->nq * c.num_levels;
    const bool mixed = c.precision == MLMC_MIXED;
    if (mixed) ctx->sp = mixed_pad_k(s);
    const int64_t brows = mixed ? mixed_pad_cols(ctx->Mmax) : 0;
    const int64_t yrows = mixed ? mixed_pad_rows(ctx->chunk_max) : 0;
    const int64_t a64 = mixed ? ctx->pool : 0;
    const bool tile_levels = fused_supported(c.mu1, c.mu2) &&
                             Gmax > (c.rtol > 0.0 ? kLdsMaxLevel : kLdsMaxLevelFixed);
    const size_t own_tables = parent ? 0 : 1;
    size_t need = (size_t)ctx->elem * (tile_levels ? 4 : 3) * (size_t)ctx->pool +
                  (2 * kDigits * (size_t)ctx->sp + 4) * (size_t)(own_tables * brows + yrows) +
                  8 * (size_t)a64 +
                  sizeof(double) * (own_tables * (size_t)s * ctx->Mmax + 4 * ctx->fcg_cells + parts + wcap +
                                    (size_t)ctx->chunk_max * (s + c.num_levels * ctx->nq + 6) +
                                    qoi_partials(ctx->pool) +
                                    4 * ctx->state_tuples) +
                  sizeof(int32_t) * 4 * ctx->chunk_max;
    size_t free_b = 0, total_b = 0;
    CHK(hipMemGetInfo(&free_b, &total_b));
    if (need > free_b) {
        char msg[200];
        snprintf(msg, sizeof msg, "workspace needs %.3g GB, %.3g GB free", need / 1e9, free_b / 1e9);
        ctx->err = msg;
        return fail(MLMC_E_NOMEM);
    }
    if (!parent) CHK(dev_alloc(ctx, &ctx->d_basis, (int64_t)s * ctx->Mmax));
    {
        char *pa = nullptr, *pu = nullptr, *pf = nullptr;
        CHK(dev_alloc(ctx, &pa, ctx->pool * ctx->elem));
        CHK(dev_alloc(ctx, &pu, ctx->pool * ctx->elem));
        CHK(dev_alloc(ctx, &pf, ctx->pool * ctx->elem));
        ctx->d_a = (double *)pa;      // float storage in the mixed mode
        ctx->d_u = (double *)pu;
        ctx->d_f = (double *)pf;
    }
    for (int i = 0; i < kDigits && mixed; ++i) {
        if (!parent) CHK(dev_alloc(ctx, &ctx->d_bdig[i], brows * ctx->sp));
        CHK(dev_alloc(ctx, &ctx->d_ydig[i], yrows * ctx->sp));
    }
    if (!parent) CHK(dev_alloc(ctx, &ctx->d_bexp, brows));
    CHK(dev_alloc(ctx, &ctx->d_yexp, yrows));
    CHK(dev_alloc(ctx, &ctx->d_a64, a64));
    if (tile_levels) {
        char *pa2 = nullptr;
        CHK(dev_alloc(ctx, &pa2, ctx->pool * ctx->elem));
        ctx->d_ua = (double *)pa2;    // float storage in the mixed mode
    }
    CHK(dev_alloc(ctx, &ctx->d_fcg, 4 * ctx->fcg_cells));
    CHK(dev_alloc(ctx, &ctx->d_part, parts));
    CHK(dev_alloc(ctx, &ctx->d_fs, ctx->fcg_cells > 0 ? 4 * ctx->chunk_max : 0));
    CHK(dev_alloc(ctx, &ctx->d_w, wcap));
    CHK(dev_alloc(ctx, &ctx->d_st_iters, ctx->chunk_max));
    CHK(dev_alloc(ctx, &ctx->d_st_bad, ctx->chunk_max));
    CHK(dev_alloc(ctx, &ctx->d_st_rho, ctx->chunk_max));
    CHK(dev_alloc(ctx, &ctx->d_y, ctx->chunk_max * s));
    CHK(dev_alloc(ctx, &ctx->d_qoi, ctx->chunk_max * c.num_levels * ctx->nq));
    CHK(dev_alloc(ctx, &ctx->d_state, 4 * ctx->state_tuples));
    CHK(dev_alloc(ctx, &ctx->d_rho, ctx->chunk_max));
    CHK(dev_alloc(ctx, &ctx->d_rho_hist, ctx->fcg_cells > 0 ? 4 * ctx->chunk_max : 0));
    CHK(dev_alloc(ctx, &ctx->d_qpart, qoi_partials(ctx->pool)));
    CHK(dev_alloc(ctx, &ctx->d_active, ctx->chunk_max));
    CHK(dev_alloc(ctx, &ctx->d_iters, ctx->chunk_max));
    CHK(hipHostMalloc((void **)&ctx->h_active, sizeof(int32_t) * ctx->chunk_max, hipHostMallocDefault));
    CHK(hipHostMalloc((void **)&ctx->h_iters, sizeof(int32_t) * ctx->chunk_max, hipHostMallocDefault));
    CHK(hipHostMalloc((void **)&ctx->h_rho, sizeof(double) * ctx->chunk_max, hipHostMallocDefault));
    if (parent) {
        const mlmc_config &q = parent->cfg;
        if (q.precision == c.precision && (q.rtol > 0.0) == (c.rtol > 0.0) && q.mu1 == c.mu1 &&
            q.mu2 == c.mu2) {
            std::memcpy(ctx->pre_kind, parent->pre_kind, sizeof(ctx->pre_kind));
            std::memcpy(ctx->post_kind, parent->post_kind, sizeof(ctx->post_kind));
            std::memcpy(ctx->pre_ms, parent->pre_ms, sizeof(ctx->pre_ms));
            std::memcpy(ctx->post_ms, parent->post_ms, sizeof(ctx->post_ms));
        }
        ctx->d_basis = parent->d_basis;
        for (int i = 0; i < kDigits; ++i) ctx->d_bdig[i] = parent->d_bdig[i];
        ctx->d_bexp = parent->d_bexp;
        ctx->d_z = parent->d_z;
        ctx->d_shifts = parent->d_shifts;
        *out = ctx;
        return MLMC_OK;
    }
    if (lattice) {
        CHK(dev_alloc(ctx, &ctx->d_z, s));
        CHK(dev_alloc(ctx, &ctx->d_shifts, (int64_t)c.num_levels * c.num_shifts * s));
        CHK(hipMemcpy(ctx->d_z, c.genvec, sizeof(uint32_t) * s, hipMemcpyHostToDevice));
        CHK(hipMemcpy(ctx->d_shifts, c.shifts, sizeof(uint64_t) * (size_t)c.num_levels * c.num_shifts * s,
                      hipMemcpyHostToDevice));
    }
    if (matern) {
        const std::string merr = matern_basis(nq_nodes, c.nu, lam, sigma, s, Gmax, ctx->d_basis,
                                              ctx->Mmax, ctx->theta2);
        if (!merr.empty()) {
            ctx->err = merr;
            return fail(merr.find("out of memory") != std::string::npos ? MLMC_E_NOMEM : MLMC_E_HIP);
        }
        if (mixed) {
            launch_digits_cols(nullptr, ctx->d_basis, ctx->Mmax, s, ctx->Mmax, brows, ctx->sp,
                               ctx->d_bdig, ctx->d_bexp);
            CHK(hipGetLastError());
            CHK(hipDeviceSynchronize());
            void *fb = ctx->d_basis;
            ctx->d_basis = nullptr;
            (void)hipFree(fb);
            ctx->allocs.erase(std::find(ctx->allocs.begin(), ctx->allocs.end(), fb));
        }
        *out = ctx;
        return MLMC_OK;
    }
    // build the dense basis on the device from the 1-D tables
    double *d_psi = nullptr, *d_coef = nullptr;
    int64_t *d_psi_off = nullptr;
    int32_t *d_mi = nullptr, *d_mj = nullptr;
    CHK(hipMalloc((void **)&d_psi, sizeof(double) * psi.size()));
    ctx->allocs.push_back(d_psi);
    CHK(hipMalloc((void **)&d_coef, sizeof(double) * s));
    ctx->allocs.push_back(d_coef);
    CHK(hipMalloc((void **)&d_psi_off, sizeof(int64_t) * psi_off.size()));
    ctx->allocs.push_back(d_psi_off);
    CHK(hipMalloc((void **)&d_mi, sizeof(int32_t) * s));
    ctx->allocs.push_back(d_mi);
    CHK(hipMalloc((void **)&d_mj, sizeof(int32_t) * s));
    ctx->allocs.push_back(d_mj);
    CHK(hipMemcpy(d_psi, psi.data(), sizeof(double) * psi.size(), hipMemcpyHostToDevice));
    CHK(hipMemcpy(d_coef, coef.data(), sizeof(double) * s, hipMemcpyHostToDevice));
    CHK(hipMemcpy(d_psi_off, psi_off.data(), sizeof(int64_t) * psi_off.size(), hipMemcpyHostToDevice));
    CHK(hipMemcpy(d_mi, ctx->mi.data(), sizeof(int32_t) * s, hipMemcpyHostToDevice));
    CHK(hipMemcpy(d_mj, ctx->mj.data(), sizeof(int32_t) * s, hipMemcpyHostToDevice));
    launch_build_basis(nullptr, d_psi, d_psi_off, d_mi, d_mj, d_coef, s, Gmax, ctx->d_basis, ctx->Mmax);
    CHK(hipGetLastError());
    if (mixed) {   // basis row m of the split = field column m, K = KL mode
        launch_digits_cols(nullptr, ctx->d_basis, ctx->Mmax, s, ctx->Mmax, brows, ctx->sp,
                           ctx->d_bdig, ctx->d_bexp);
        CHK(hipGetLastError());
    }
    CHK(hipDeviceSynchronize());
    // the 1-D tables are no longer needed, nor, in the mixed mode, the FP64
    // basis (the field is formed from its digits)
    std::vector<void *> done{d_psi, d_coef, d_psi_off, d_mi, d_mj};
    if (mixed) {
        done.push_back(ctx->d_basis);
        ctx->d_basis = nullptr;
    }
    for (void *p : done) {
        (void)hipFree(p);
        ctx->allocs.erase(std::find(ctx->allocs.begin(), ctx->allocs.end(), p));
    }
#undef CHK
    *out = ctx;
    return MLMC_OK;
}

namespace {

// Durations of one pre and one post pass of every allowed kind on tile grid g
// for the largest (Bc) and the smallest (Blo) chunk of batch class cls, on
// the workspace (a = f = 1, u = 0: the time does not depend on the values).
// Each: one warm-up launch, then the best of two runs of `reps` launches
// between events.  A pass takes the kind whose larger ratio to the fastest
// kind at the two chunk sizes is smallest (ties: the faster at Bc), so that
// no chunk of the class gets a kind that leaves most of the GPU idle (a
// streaming workgroup holds one sample on grids from 128^2).
template <typename T>
mlmc_status tune_grid(mlmc_ctx c, hipStream_t st, int g, int64_t Bc, int64_t Blo, int cls,
                      hipEvent_t e0, hipEvent_t e1)
{
    const int n = 2 << g;
    const int64_t all = Bc * level_offset(g + 1);     // levels 0..g, level-major
    {
        HierT<T> h = make_hier_t<T>(c, g, Bc);        // its fill covers the Blo layout too
        if constexpr (std::is_same<T, double>::value) {
            launch_fill(st, h.a[0], all, 1.0);
            launch_fill(st, h.f[0], all, 1.0);
            launch_fill(st, h.u[0], all, 0.0);
        } else {
            launch_fill_f32(st, h.a[0], all, 1.0f);
            launch_fill_f32(st, h.f[0], all, 1.0f);
            launch_fill_f32(st, h.u[0], all, 0.0f);
        }
    }
    double ms_best = 0.0;
    auto time_it = [&](auto launch, int reps) -> hipError_t {
        launch();
        ms_best = 1e300;
        for (int r = 0; r < 2; ++r) {
            hipError_t e = hipEventRecord(e0, st);
            for (int i = 0; i < reps && e == hipSuccess; ++i) launch();
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e == hipSuccess) e = hipGetLastError();
            if (e != hipSuccess) return e;
            ms_best = std::min(ms_best, (double)ms / reps);
        }
        return hipSuccess;
    };
    const int kinds[] = {kTile32, kTile16, kStream};
    // [size: 0 = Bc, 1 = Blo][kind] -> ms (infinite where not allowed)
    double pre_ms[2][3], post_ms[2][3];
    const int64_t sizes[2] = {Bc, Blo};
    const int nsizes = Blo < Bc ? 2 : 1;
    for (int z = 0; z < nsizes; ++z) {
        const int64_t B = sizes[z];
        HierT<T> h = make_hier_t<T>(c, g, B);
        const int reps = B * (int64_t)n * n >= ((int64_t)1 << 22) ? 3 : 10;
        for (int q = 0; q < 3; ++q) {
            const int kind = kinds[q];
            pre_ms[z][q] = post_ms[z][q] = 1e300;
            if (!kind_allowed(c, g, kind)) continue;
            auto pre = [&] {
                if (kind == kStream) {
                    launch_pre_stream<T>(st, c->cfg.mu1, h.a[g], h.f[g], h.u[g], h.ua[g], h.u[g - 1],
                                         n, B, 1, h.f[g - 1], nullptr);
                    return;
                }
                launch_pre_tile<T>(st, kind, c->cfg.mu1, h.a[g], h.f[g], h.u[g], h.ua[g], h.u[g - 1],
                                   n, B, 1, h.f[g - 1], nullptr);
            };
            auto post = [&] {
                if (kind == kStream) {
                    launch_post_stream<T>(st, c->cfg.mu2, h.a[g], h.f[g], h.ua[g], h.u[g], h.u[g - 1],
                                          n, B, nullptr);
                    return;
                }
                launch_post_tile<T>(st, kind, c->cfg.mu2, h.a[g], h.f[g], h.ua[g], h.u[g], h.u[g - 1],
                                    n, B, nullptr);
            };
            HIPCHK(c, time_it(pre, reps));
            pre_ms[z][q] = ms_best;
            HIPCHK(c, time_it(post, reps));
            post_ms[z][q] = ms_best;
        }
    }
    auto choose = [&](double (*t)[3], int8_t &kind_out, double &ms_out) {
        double best[2] = {1e300, 1e300};
        for (int z = 0; z < nsizes; ++z)
            for (int q = 0; q < 3; ++q) best[z] = std::min(best[z], t[z][q]);
        int pick = -1;
        double pick_score = 1e300;
        for (int q = 0; q < 3; ++q) {
            if (t[0][q] >= 1e300) continue;
            double score = 0.0;
            for (int z = 0; z < nsizes; ++z) score = std::max(score, t[z][q] / best[z]);
            if (pick < 0 || score < pick_score || (score == pick_score && t[0][q] < t[0][pick])) {
                pick = q;
                pick_score = score;
            }
        }
        kind_out = (int8_t)kinds[pick];
        ms_out = t[0][pick];
    };
    choose(pre_ms, c->pre_kind[g][cls], c->pre_ms[g][cls]);
    choose(post_ms, c->post_kind[g][cls], c->post_ms[g][cls]);
    return MLMC_OK;
}

// tile grids of a context: MG levels lds_top < g <= Gmax (none without the
// fused passes)
int first_tile_grid(mlmc_ctx c) { return lds_top(c) + 1; }
int tile_grid_count(mlmc_ctx c)
{
    return use_fused(c) ? std::max(0, c->Gmax - lds_top(c)) : 0;
}

}  // namespace

extern "C" {

mlmc_status mlmc_autotune(mlmc_ctx ctx, int32_t level, void *hip_stream)
{
    if (!ctx) return MLMC_E_INVAL;
    if (ctx->broken || ctx->host_only) return MLMC_E_STATE;
    if (level < 0 || level >= ctx->cfg.num_levels) return inval(ctx, "level out of range");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    if (tile_grid_count(ctx) == 0) return MLMC_OK;
    hipStream_t st = (hipStream_t)hip_stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(ctx, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        ctx->err = "hipEventCreate failed";
        ctx->broken = true;
        return MLMC_E_HIP;
    }
    mlmc_status r = MLMC_OK;
    for (int g = first_tile_grid(ctx); g <= ctx->g0 + level && r == MLMC_OK; ++g) {
        const int64_t cap = chunk_capacity(ctx, std::max(0, g - ctx->g0));
        for (int cl = 0; cl < MLMC_BATCH_CLASSES && r == MLMC_OK; ++cl) {
            const int64_t lo = cl == 0 ? 1 : ((int64_t)1 << (2 * (cl - 1))) + 1;
            if (lo > cap) break;
            const int64_t Bc = cl + 1 == MLMC_BATCH_CLASSES
                                   ? cap
                                   : std::min<int64_t>((int64_t)1 << (2 * cl), cap);
            r = ctx->cfg.precision == MLMC_MIXED
                    ? tune_grid<float>(ctx, st, g, Bc, std::min(lo, Bc), cl, e0, e1)
                    : tune_grid<double>(ctx, st, g, Bc, std::min(lo, Bc), cl, e0, e1);
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return r;
}

mlmc_status mlmc_tuning_get(mlmc_ctx ctx, mlmc_tune_entry *out, int32_t max_entries,
                            int32_t *count)
{
    if (!ctx || !count || max_entries < 0 || (max_entries > 0 && !out)) return MLMC_E_INVAL;
    int32_t k = 0;
    const int g1 = first_tile_grid(ctx);
    for (int g = g1; g < g1 + tile_grid_count(ctx); ++g)
        for (int cl = 0; cl < MLMC_BATCH_CLASSES; ++cl, ++k) {
            if (k >= max_entries) continue;
            mlmc_tune_entry &e = out[k];
            e.n = 2 << g;
            e.batch_class = cl;
            e.pre = ctx->pre_kind[g][cl];
            e.post = ctx->post_kind[g][cl];
            e.pre_ms = ctx->pre_ms[g][cl];
            e.post_ms = ctx->post_ms[g][cl];
        }
    *count = k;
    return MLMC_OK;
}

mlmc_status mlmc_tuning_set(mlmc_ctx ctx, const mlmc_tune_entry *in, int32_t count)
{
    if (!ctx || count < 0 || (count > 0 && !in)) return MLMC_E_INVAL;
    const int g1 = first_tile_grid(ctx), g2 = g1 + tile_grid_count(ctx);
    for (int32_t i = 0; i < count; ++i) {
        const mlmc_tune_entry &e = in[i];
        const int g = ilog2_exact(e.n) - 1;
        if (g < g1 || g >= g2) return inval(ctx, "tuning entry: n is not a tile grid of this context");
        if (e.batch_class < 0 || e.batch_class >= MLMC_BATCH_CLASSES)
            return inval(ctx, "tuning entry: batch class out of range");
        if (!kind_allowed(ctx, g, e.pre) || !kind_allowed(ctx, g, e.post))
            return inval(ctx, "tuning entry: pass kind not available on this grid");
    }
    for (int32_t i = 0; i < count; ++i) {
        const mlmc_tune_entry &e = in[i];
        const int g = ilog2_exact(e.n) - 1;
        ctx->pre_kind[g][e.batch_class] = (int8_t)e.pre;
        ctx->post_kind[g][e.batch_class] = (int8_t)e.post;
        ctx->pre_ms[g][e.batch_class] = 0.0;
        ctx->post_ms[g][e.batch_class] = 0.0;
    }
    return MLMC_OK;
}

}  // extern "C"

extern "C" {

mlmc_status mlmc_create(const mlmc_config *cfg, int device, mlmc_ctx *out)
{
    return create_ctx(cfg, device, nullptr, out);
}

mlmc_status mlmc_destroy(mlmc_ctx ctx)
{
    if (!ctx) return MLMC_OK;
    if (!ctx->host_only) {
        (void)hipSetDevice(ctx->device);
        (void)hipDeviceSynchronize();
    }
    free_all(ctx);
    delete ctx;
    return MLMC_OK;
}

int64_t mlmc_field_size(mlmc_ctx ctx, int32_t level)
{
    if (!ctx || level < 0 || level >= ctx->cfg.num_levels) return 0;
    return field_size_g(ctx->g0 + level);
}

int32_t mlmc_num_qoi(mlmc_ctx ctx) { return ctx ? ctx->nq : 0; }

mlmc_status mlmc_points_gen(mlmc_ctx ctx, const mlmc_points *pts, uint64_t *x_dev, double *y_dev,
                            void *hip_stream)
{
    if (!ctx) return MLMC_E_INVAL;
    if (ctx->broken || ctx->host_only) return MLMC_E_STATE;
    int64_t B, npts;
    int nsh;
    mlmc_status st = check_points(ctx, pts, &B, &npts, &nsh);
    if (st) return st;
    if (x_dev && pts->kind != MLMC_POINTS_LATTICE) return inval(ctx, "x_dev only for lattice points");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)hip_stream;
    if (B == 0) return MLMC_OK;
    if (pts->kind == MLMC_POINTS_EXPLICIT) {
        if (y_dev)
            HIPCHK(ctx, hipMemcpyAsync(y_dev, pts->y_dev, sizeof(double) * B * ctx->cfg.s,
                                       hipMemcpyDeviceToDevice, s));
        return MLMC_OK;
    }
    for (int64_t b0 = 0; b0 < B; b0 += ctx->chunk_max) {
        int64_t Bc = std::min(ctx->chunk_max, B - b0);
        launch_points(s, ctx->d_z, ctx->d_shifts, ctx->cfg.s, ctx->cfg.num_shifts, pts->level,
                      pts->shift_begin, pts->n_begin, npts, b0, Bc,
                      x_dev ? x_dev + b0 * ctx->cfg.s : nullptr,
                      y_dev ? y_dev + b0 * ctx->cfg.s : ctx->d_y);
    }
    HIPCHK(ctx, hipGetLastError());
    return MLMC_OK;
}

namespace {
// mixed mode: split the chunk's Y into bf16 terms, then the matrix-core product
void field_digits(mlmc_ctx ctx, hipStream_t s, const double *Y, int64_t M, int64_t Bc, void *out,
                  double *out64, int mode)
{
    const int sd = ctx->cfg.s;
    launch_digits_rows(s, Y, Bc, sd, sd, mixed_pad_rows(Bc), ctx->sp, ctx->d_ydig, ctx->d_yexp);
    launch_field_digits(s, ctx->d_ydig, ctx->d_yexp, ctx->d_bdig, ctx->d_bexp, ctx->sp, M, Bc, out,
                        out64, mode);
}
}  // namespace

mlmc_status mlmc_field(mlmc_ctx ctx, const mlmc_points *pts, double *z_dev, void *hip_stream)
{
    if (!ctx) return MLMC_E_INVAL;
    if (ctx->broken || ctx->host_only) return MLMC_E_STATE;
    int64_t B, npts;
    int nsh;
    mlmc_status st = check_points(ctx, pts, &B, &npts, &nsh);
    if (st) return st;
    if (!z_dev && B > 0) return inval(ctx, "z_dev is NULL");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)hip_stream;
    const int64_t M = field_size_g(ctx->g0 + pts->level);
    for (int64_t b0 = 0; b0 < B; b0 += ctx->chunk_max) {
        int64_t Bc = std::min(ctx->chunk_max, B - b0);
        const double *Y = chunk_y(ctx, s, pts, npts, b0, Bc, nullptr);
        if (ctx->cfg.precision == MLMC_MIXED)
            field_digits(ctx, s, Y, M, Bc, z_dev + b0 * M, nullptr, 0);
        else
            launch_field_gemm(s, Y, ctx->cfg.s, ctx->d_basis, ctx->Mmax, M, Bc, z_dev + b0 * M, 0);
    }
    HIPCHK(ctx, hipGetLastError());
    return MLMC_OK;
}

// mlmc_field with the staging of the points (Y for lattice points) and, in
// a mixed context, of their bf16 digits and scale exponents in the static
// scratch instead of the context's workspace.  Layout (each part aligned to
// 256 bytes): Y [B][s] FP64 (lattice points only), then kDigits digit arrays
// [B_pad][sp] and the exponents [B_pad].
static int64_t static_field_bytes(mlmc_ctx c, int64_t B, bool lattice)
{
    auto up = [](int64_t v) { return (v + 255) / 256 * 256; };
    int64_t bytes = lattice ? up(8 * B * c->cfg.s) : 0;
    if (c->cfg.precision == MLMC_MIXED) {
        const int64_t rows = mixed_pad_rows(B);
        bytes += kDigits * up(2 * rows * c->sp) + up(4 * rows);
    }
    return bytes;
}

mlmc_status mlmc_field_static(mlmc_ctx ctx, const mlmc_points *pts, double *z_dev,
                              void *hip_stream)
{
    if (!ctx) return MLMC_E_INVAL;
    if (ctx->broken || ctx->host_only) return MLMC_E_STATE;
    int64_t B, npts;
    int nsh;
    mlmc_status st = check_points(ctx, pts, &B, &npts, &nsh);
    if (st) return st;
    if (!z_dev && B > 0) return inval(ctx, "z_dev is NULL");
    const bool lattice = pts->kind == MLMC_POINTS_LATTICE;
    if (static_field_bytes(ctx, B, lattice) > (int64_t)kStaticScratchBytes) {
        char msg[160];
        snprintf(msg, sizeof msg, "mlmc_field_static: %lld samples need %lld bytes of scratch, "
                 "more than its %zu", (long long)B, (long long)static_field_bytes(ctx, B, lattice),
                 kStaticScratchBytes);
        ctx->err = msg;
        return MLMC_E_INVAL;
    }
    if (B == 0) return MLMC_OK;
    unsigned char *base = (unsigned char *)static_scratch_ptr(ctx->device);
    if (!base) {
        ctx->err = "static scratch not resolved on this device";
        return MLMC_E_STATE;
    }
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)hip_stream;
    auto up = [](int64_t v) { return (v + 255) / 256 * 256; };
    const int sd = ctx->cfg.s;
    const int64_t M = field_size_g(ctx->g0 + pts->level);
    const double *Y = pts->y_dev;
    int64_t off = 0;
    if (lattice) {
        double *y = (double *)base;
        launch_points(s, ctx->d_z, ctx->d_shifts, sd, ctx->cfg.num_shifts, pts->level,
                      pts->shift_begin, pts->n_begin, npts, 0, B, nullptr, y);
        Y = y;
        off = up(8 * B * sd);
    }
    if (ctx->cfg.precision == MLMC_MIXED) {
        const int64_t rows = mixed_pad_rows(B);
        uint16_t *dig[kDigits];
        for (int q = 0; q < kDigits; ++q) {
            dig[q] = (uint16_t *)(base + off);
            off += up(2 * rows * ctx->sp);
        }
        int32_t *ey = (int32_t *)(base + off);
        launch_digits_rows(s, Y, B, sd, sd, rows, ctx->sp, dig, ey);
        launch_field_digits(s, dig, ey, ctx->d_bdig, ctx->d_bexp, ctx->sp, M, B, z_dev, nullptr,
                            0);
    } else {
        launch_field_gemm(s, Y, sd, ctx->d_basis, ctx->Mmax, M, B, z_dev, 0);
    }
    HIPCHK(ctx, hipGetLastError());
    return MLMC_OK;
}

mlmc_status mlmc_fmg_solve(mlmc_ctx ctx, const mlmc_points *pts, const double *z_dev,
                           double *qoi_dev, double *sums_dev, mlmc_solve_info *info,
                           void *hip_stream)
{
    return mlmc::fmg_solve_ex(ctx, pts, z_dev, qoi_dev, sums_dev, info, hip_stream, nullptr,
                              nullptr);
}

}  // extern "C"

mlmc_status mlmc::fmg_solve_ex(mlmc_ctx ctx, const mlmc_points *pts, const double *z_dev,
                               double *qoi_dev, double *sums_dev, mlmc_solve_info *info,
                               void *hip_stream, int32_t *sample_bad, double *sample_rho)
{
    if (!ctx) return MLMC_E_INVAL;
    if (ctx->broken || ctx->host_only) return MLMC_E_STATE;
    int64_t B, npts;
    int nsh;
    mlmc_status st = check_points(ctx, pts, &B, &npts, &nsh);
    if (st) return st;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)hip_stream;
    const int k = pts->level, G = ctx->g0 + k, nlev = k + 1, nq = ctx->nq;
    const int64_t M = field_size_g(G);
    const int64_t cap = chunk_capacity(ctx, k);
    const int64_t ntup = (int64_t)nsh * nq * nlev;
    if (sums_dev) launch_fill(s, ctx->d_state, 4 * ntup, 0.0);
    StageStats stats;
    stats.sample_bad = sample_bad;
    stats.sample_rho = sample_rho;
    if (sample_bad) std::fill(sample_bad, sample_bad + B, 0);
    if (sample_rho) std::fill(sample_rho, sample_rho + B, -1.0);
    mlmc_solve_info local_info;
    if (!info && (sample_bad || sample_rho)) info = &local_info;
    for (int64_t b0 = 0; b0 < B; b0 += cap) {
        const int64_t Bc = std::min(cap, B - b0);
        stats.b0 = b0;
        Hier h = make_hier(ctx, G, Bc);
        const bool mixed = ctx->cfg.precision == MLMC_MIXED;
        if (z_dev) {
            launch_exp_to_levels(s, z_dev + b0 * M, M, Bc, ctx->d_a, mixed, ctx->d_a64);
        } else {
            const double *Y;
            {
                ProfScope ps(ctx, s, MLMC_KERNEL_POINTS, 16.0 * Bc * ctx->cfg.s, 0.0);
                Y = chunk_y(ctx, s, pts, npts, b0, Bc, nullptr);
            }
            const double sd = ctx->cfg.s;
            if (mixed) {
                // fifteen bf16 digit products per term; operands 5 x 2 bytes, a
                // stored as float and double
                ProfScope ps(ctx, s, MLMC_KERNEL_FIELD,
                             8.0 * Bc * sd + 2.0 * kDigits * (Bc + (double)M) * sd + 12.0 * Bc * M,
                             30.0 * Bc * sd * M);
                field_digits(ctx, s, Y, M, Bc, ctx->d_a, ctx->d_a64, 2);
            } else {
                ProfScope ps(ctx, s, MLMC_KERNEL_FIELD, 8.0 * (Bc * sd + sd * M + (double)Bc * M),
                             2.0 * Bc * sd * M);
                launch_field_gemm(s, Y, ctx->cfg.s, ctx->d_basis, ctx->Mmax, M, Bc, ctx->d_a, 1);
            }
        }
        double *q = qoi_dev ? qoi_dev + b0 * nlev * nq : ctx->d_qoi;
        if (!use_fused(ctx))
            st = run_fmg(ctx, s, h, k, q, nullptr, &stats);
        else if (ctx->cfg.rtol <= 0.0)
            st = run_fmg_fixed(ctx, s, G, Bc, k, q, &stats);
        else if (mixed)
            st = run_fmg_refine<float>(ctx, s, G, Bc, k, q, &stats);
        else
            st = run_fmg_refine<double>(ctx, s, G, Bc, k, q, &stats);
        if (st) return st;
        if (sums_dev) {
            ProfScope ps(ctx, s, MLMC_KERNEL_SUMS, 8.0 * Bc * nlev * nq, 0.0);
            launch_sums(s, q, nlev, nq, b0, Bc, npts, nsh, ctx->d_state);
        }
    }
    if (sums_dev) launch_sums_final(s, ctx->d_state, ntup, sums_dev);
    HIPCHK(ctx, hipGetLastError());
    if (info) {
        HIPCHK(ctx, hipStreamSynchronize(s));
        info->samples = B;
        info->max_iters_used = stats.max_iters;
        info->max_rel_residual = ctx->cfg.rtol > 0.0 ? stats.max_rho : -1.0;
        info->not_converged = stats.noconv;
        if (stats.noconv > 0) {
            ctx->err = "refinement stopped above rtol (max_iters or the rounding floor)";
            return MLMC_E_NOCONV;
        }
    }
    return MLMC_OK;
}

extern "C" {

mlmc_status mlmc_kl_modes(mlmc_ctx ctx, int32_t *i_out, int32_t *j_out, double *theta_out)
{
    if (!ctx) return MLMC_E_INVAL;
    const int s = ctx->cfg.s;
    if (i_out) std::memcpy(i_out, ctx->mi.data(), sizeof(int32_t) * s);
    if (j_out) std::memcpy(j_out, ctx->mj.data(), sizeof(int32_t) * s);
    if (theta_out) std::memcpy(theta_out, ctx->theta2.data(), sizeof(double) * s);
    return MLMC_OK;
}

mlmc_status mlmc_fmg_trace(mlmc_ctx ctx, int32_t level, int32_t *levels, int32_t *marks,
                           int64_t cap, int64_t *len)
{
    if (!ctx) return MLMC_E_INVAL;
    if (level < 0 || level >= ctx->cfg.num_levels) return inval(ctx, "level out of range");
    if (ctx->cfg.rtol > 0.0) return inval(ctx, "trace is data dependent in rtol mode");
    if (cap < 0 || (cap > 0 && (!levels || !marks))) return inval(ctx, "bad trace buffers");
    Trace tr;
    Hier h;
    h.G = ctx->g0 + level;
    run_fmg(ctx, nullptr, h, level, nullptr, &tr, nullptr);
    int64_t n = (int64_t)tr.lev.size();
    for (int64_t i = 0; i < std::min(n, cap); ++i) {
        levels[i] = tr.lev[i];
        marks[i] = tr.mark[i];
    }
    if (len) *len = n;
    return MLMC_OK;
}

mlmc_status mlmc_profile_begin(mlmc_ctx ctx, int32_t kernel_kind)
{
    if (!ctx) return MLMC_E_INVAL;
    if (ctx->host_only) return MLMC_E_STATE;
    if (kernel_kind < MLMC_KERNEL_POINTS || kernel_kind > MLMC_KERNEL_REFINE)
        return inval(ctx, "unknown kernel kind");
    ctx->prof.kind = kernel_kind;
    ctx->prof.used = 0;
    ctx->prof.launches = 0;
    ctx->prof.bytes = ctx->prof.flops = 0.0;
    return MLMC_OK;
}

mlmc_status mlmc_profile_end(mlmc_ctx ctx, mlmc_profile_result *out)
{
    if (!ctx || !out) return MLMC_E_INVAL;
    if (ctx->host_only) return MLMC_E_STATE;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    HIPCHK(ctx, hipDeviceSynchronize());
    double ms_total = 0.0;
    for (size_t i = 0; i < ctx->prof.used; ++i) {
        float ms = 0.0f;
        HIPCHK(ctx, hipEventElapsedTime(&ms, ctx->prof.ev[2 * i], ctx->prof.ev[2 * i + 1]));
        ms_total += ms;
    }
    out->launches = ctx->prof.launches;
    out->total_ms = ms_total;
    out->bytes = ctx->prof.bytes;
    out->flops = ctx->prof.flops;
    ctx->prof.kind = -1;
    ctx->prof.used = 0;
    return MLMC_OK;
}

mlmc_status mlmc_estimate(const mlmc_est_input *in, mlmc_est_output *out)
{
    if (!in || !out || !in->n_per_level || !in->sums) return MLMC_E_INVAL;
    const int L1 = in->num_levels, R = in->num_shifts, nq = in->nq;
    if (L1 < 1 || R < 1 || nq < 1 || nq > 2) return MLMC_E_INVAL;
    for (int k = 0; k < L1; ++k)
        if (in->n_per_level[k] < 0) return MLMC_E_INVAL;
    if (!out->upsilon || !out->upsilon_bar || !out->var_level || !out->q_shift || !out->q_bar ||
        !out->var_q)
        return MLMC_E_INVAL;
    const bool reuse = in->reuse != 0;
    const double nan = std::nan("");
    // sums[k][r][q][l][2]
    auto S = [&](int k, int r, int q, int l, int w) {
        return in->sums[((((int64_t)k * R + r) * nq + q) * L1 + l) * 2 + w];
    };
    for (int q = 0; q < nq; ++q) {
        double *ups = out->upsilon + (int64_t)q * L1 * R;
        for (int l = 0; l < L1; ++l) {
            int64_t den = 0;
            for (int k = (reuse ? l : l); k <= (reuse ? L1 - 1 : l); ++k) den += in->n_per_level[k];
            for (int r = 0; r < R; ++r) {
                HostSum num;
                for (int k = l; k <= (reuse ? L1 - 1 : l); ++k) num.add(S(k, r, q, l, 0));
                ups[(int64_t)l * R + r] = den > 0 ? num.value() / (double)den : 0.0;
            }
        }
        double *qs = out->q_shift + (int64_t)q * R;
        for (int r = 0; r < R; ++r) {
            HostSum t;
            for (int l = 0; l < L1; ++l) t.add(ups[(int64_t)l * R + r]);
            qs[r] = t.value();
        }
        HostSum qb;
        for (int r = 0; r < R; ++r) qb.add(qs[r]);
        out->q_bar[q] = qb.value() / R;
        for (int l = 0; l < L1; ++l) {
            HostSum ub;
            for (int r = 0; r < R; ++r) ub.add(ups[(int64_t)l * R + r]);
            out->upsilon_bar[(int64_t)q * L1 + l] = ub.value() / R;
        }
        if (R >= 2) {
            HostSum v;
            for (int r = 0; r < R; ++r) {
                double d = qs[r] - out->q_bar[q];
                v.add(d * d);
            }
            out->var_q[q] = v.value() / ((double)R * (R - 1));
            for (int l = 0; l < L1; ++l) {
                HostSum vl;
                double m = out->upsilon_bar[(int64_t)q * L1 + l];
                for (int r = 0; r < R; ++r) {
                    double d = ups[(int64_t)l * R + r] - m;
                    vl.add(d * d);
                }
                out->var_level[(int64_t)q * L1 + l] = vl.value() / ((double)R * (R - 1));
            }
        } else if (!reuse) {
            // eq. vardecomp: V = sum_l s_l^2 / N_l from sum dF and sum dF^2
            HostSum v;
            for (int l = 0; l < L1; ++l) {
                int64_t N = in->n_per_level[l];
                double vl = nan;
                if (N > 1) {
                    // (s2 - s1^2/N) / (N-1) with s1^2/N carried to about one
                    // rounding: m = s1/N with its exact remainder s1 - m N,
                    // s1 m split into its rounded value and exact error (fma),
                    // so that only the cancellation against s2 is left, and
                    // that subtraction is exact when the two are close
                    const double s1 = S(l, 0, q, l, 0), s2 = S(l, 0, q, l, 1);
                    const double Nd = (double)N;
                    const double m = s1 / Nd;
                    const double rem = std::fma(-m, Nd, s1);
                    const double p = s1 * m;
                    const double perr = std::fma(s1, m, -p);
                    const double num = ((s2 - p) - perr) - s1 * (rem / Nd);
                    vl = std::max(num, 0.0) / (Nd - 1.0) / Nd;
                }
                out->var_level[(int64_t)q * L1 + l] = vl;
                v.add(vl);
            }
            out->var_q[q] = v.value();
        } else {
            for (int l = 0; l < L1; ++l) out->var_level[(int64_t)q * L1 + l] = nan;
            out->var_q[q] = nan;
        }
    }
    return MLMC_OK;
}

}  // extern "C"
