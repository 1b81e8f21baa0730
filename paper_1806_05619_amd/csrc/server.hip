// Serving loop: a FIFO of (level, lattice range, shift range) solve requests,
// served by a fixed set of slots.  Each slot is one context (its own
// workspace, sized at create; the KL tables are the first slot's, held once),
// one HIP stream and one host thread; a free slot takes the oldest queued
// request and every queued request of the same level that still fits the
// workspace at that level, generates their points into one explicit batch,
// solves it (the SampleAndSolve body of Algorithm 1) and hands back the QoIs,
// the per-shift level-difference sums a request asks for (formed on the
// device, compensated) and the request's unconverged samples.
// Slots run concurrently, so batches of different levels overlap on the
// device.
#include "internal.hpp"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

using Clock = std::chrono::steady_clock;

namespace {

struct Pending {
    mlmc_request req;
    int64_t samples;
    Clock::time_point submitted;
};

struct Slot {
    mlmc_ctx ctx = nullptr;
    hipStream_t stream = nullptr;
    double *y_dev = nullptr;      // [cap][s]
    double *q_dev = nullptr;      // [cap][num_levels][nq]
    double *q_host = nullptr;     // pinned copy of q_dev
    int64_t *seg_host = nullptr;  // pinned [cap][2]: (first sample, count) per requested sum
    int64_t *seg_dev = nullptr;
    double *s_dev = nullptr;      // [cap][nq][num_levels][2] segment sums
    double *s_host = nullptr;     // pinned copy of s_dev
    std::vector<int32_t> bad;     // per sample of the batch: stopped above rtol
    std::vector<double> rho;      // per sample: largest final residual ratio
    std::thread worker;
};

double ms_between(Clock::time_point a, Clock::time_point b)
{
    return std::chrono::duration<double, std::milli>(b - a).count();
}

}  // namespace

struct mlmc_server_s {
    mlmc_config cfg{};
    int device = 0;
    int nq = 1;
    int64_t slot_samples = 0;
    std::vector<int64_t> cap;     // samples per batch at each level (HBM footprint)
    std::vector<Slot> slots;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Pending> queue;
    std::deque<mlmc_result> done;
    bool stopping = false;

    // statistics of completed requests
    std::vector<double> latencies;
    int64_t n_samples = 0, n_batches = 0;
    bool started = false;
    Clock::time_point first_submit, last_done;

    void work(int slot_index);
    mlmc_status solve(Slot &sl, int level, std::vector<Pending> &batch, int64_t total);
    void report(const Slot &sl, const std::vector<Pending> &batch, mlmc_status st, int level,
                int64_t total, Clock::time_point t_start, Clock::time_point t_end);
};

mlmc_status mlmc_server_s::solve(Slot &sl, int level, std::vector<Pending> &batch, int64_t total)
{
    const int s = cfg.s;
    int64_t off = 0;
    for (auto &p : batch) {
        mlmc_points pts{MLMC_POINTS_LATTICE, level, p.req.shift_begin, p.req.shift_end,
                        p.req.n_begin, p.req.n_end, nullptr};
        mlmc_status st = mlmc_points_gen(sl.ctx, &pts, nullptr, sl.y_dev + off * s, sl.stream);
        if (st) return st;
        off += p.samples;
    }
    mlmc_points all{MLMC_POINTS_EXPLICIT, level, 0, 1, 0, total, sl.y_dev};
    // per-sample convergence flags (synchronises the slot's stream in rtol mode)
    mlmc_status st = mlmc::fmg_solve_ex(sl.ctx, &all, nullptr, sl.q_dev, nullptr, nullptr,
                                        sl.stream, sl.bad.data(), sl.rho.data());
    if (st && st != MLMC_E_NOCONV) return st;
    // level-difference sums of every (request, shift) that asked for them:
    // one segment of the batch's QoI table each, one launch for the batch
    const int nlev = level + 1;
    int64_t nseg = 0;
    off = 0;
    for (auto &p : batch) {
        const int64_t npts = p.req.n_end - p.req.n_begin;
        if (p.req.sums_out)
            for (int r = p.req.shift_begin; r < p.req.shift_end; ++r) {
                sl.seg_host[2 * nseg] = off + (int64_t)(r - p.req.shift_begin) * npts;
                sl.seg_host[2 * nseg + 1] = npts;
                ++nseg;
            }
        off += p.samples;
    }
    const size_t srow = sizeof(double) * (size_t)nq * nlev * 2;
    if (nseg > 0) {
        if (hipMemcpyAsync(sl.seg_dev, sl.seg_host, sizeof(int64_t) * 2 * nseg,
                           hipMemcpyHostToDevice, sl.stream) != hipSuccess)
            return MLMC_E_HIP;
        mlmc::launch_seg_sums(sl.stream, sl.q_dev, nlev, nq, sl.seg_dev, nseg, sl.s_dev);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(sl.s_host, sl.s_dev, srow * nseg, hipMemcpyDeviceToHost, sl.stream) !=
                hipSuccess)
            return MLMC_E_HIP;
    }
    const size_t row = sizeof(double) * (size_t)nlev * nq;
    if (hipMemcpyAsync(sl.q_host, sl.q_dev, row * total, hipMemcpyDeviceToHost, sl.stream) !=
            hipSuccess ||
        hipStreamSynchronize(sl.stream) != hipSuccess)
        return MLMC_E_HIP;
    off = 0;
    nseg = 0;
    for (auto &p : batch) {
        std::memcpy(p.req.qoi_out, (const char *)sl.q_host + row * off, row * p.samples);
        if (p.req.sums_out) {
            const int nsh = p.req.shift_end - p.req.shift_begin;
            std::memcpy(p.req.sums_out, (const char *)sl.s_host + srow * nseg, srow * nsh);
            nseg += nsh;
        }
        off += p.samples;
    }
    return st;
}

void mlmc_server_s::report(const Slot &sl, const std::vector<Pending> &batch, mlmc_status st,
                           int level, int64_t total, Clock::time_point t_start,
                           Clock::time_point t_end)
{
    std::lock_guard<std::mutex> lk(mu);
    int64_t off = 0;
    for (auto &p : batch) {
        mlmc_result r{};
        r.tag = p.req.tag;
        r.level = level;
        r.samples = p.samples;
        r.batch_samples = total;
        r.queued_ms = ms_between(p.submitted, t_start);
        r.latency_ms = ms_between(p.submitted, t_end);
        r.max_rel_residual = -1.0;
        if (st == MLMC_OK || st == MLMC_E_NOCONV) {
            for (int64_t b = off; b < off + p.samples; ++b) {
                r.not_converged += sl.bad[b] != 0;
                r.max_rel_residual = std::max(r.max_rel_residual, sl.rho[b]);
            }
            r.status = r.not_converged ? MLMC_E_NOCONV : MLMC_OK;
        } else {
            r.status = st;
        }
        off += p.samples;
        done.push_back(r);
        latencies.push_back(r.latency_ms);
        n_samples += p.samples;
    }
    ++n_batches;
    last_done = t_end;
}

void mlmc_server_s::work(int slot_index)
{
    Slot &sl = slots[slot_index];
    (void)hipSetDevice(device);
    for (;;) {
        std::vector<Pending> batch;
        int level = 0;
        int64_t total = 0;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] { return stopping || !queue.empty(); });
            if (queue.empty()) return;          // stopping and drained
            level = queue.front().req.level;
            for (auto it = queue.begin(); it != queue.end();) {
                if (it->req.level == level && total + it->samples <= cap[level]) {
                    total += it->samples;
                    batch.push_back(*it);
                    it = queue.erase(it);
                } else {
                    ++it;
                }
            }
        }
        const Clock::time_point t_start = Clock::now();
        const mlmc_status st = solve(sl, level, batch, total);
        const Clock::time_point t_end = Clock::now();
        report(sl, batch, st, level, total, t_start, t_end);
        cv_done.notify_all();
    }
}

namespace {

// slots in reverse order: the first slot's context owns the shared tables
void free_slots(mlmc_server srv)
{
    for (auto it = srv->slots.rbegin(); it != srv->slots.rend(); ++it) {
        if (it->q_host) (void)hipHostFree(it->q_host);
        if (it->s_host) (void)hipHostFree(it->s_host);
        if (it->seg_host) (void)hipHostFree(it->seg_host);
        if (it->s_dev) (void)hipFree(it->s_dev);
        if (it->seg_dev) (void)hipFree(it->seg_dev);
        if (it->q_dev) (void)hipFree(it->q_dev);
        if (it->y_dev) (void)hipFree(it->y_dev);
        if (it->stream) (void)hipStreamDestroy(it->stream);
        if (it->ctx) mlmc_destroy(it->ctx);
    }
    srv->slots.clear();
}

}  // namespace

extern "C" {

mlmc_status mlmc_server_create(const mlmc_config *cfg, int device, int32_t num_slots,
                               int64_t slot_samples, mlmc_server *out)
{
    if (!out) return MLMC_E_INVAL;
    *out = nullptr;
    if (!cfg || device < 0 || num_slots < 1 || slot_samples < 1 || !cfg->genvec || !cfg->shifts)
        return MLMC_E_INVAL;
    auto *srv = new (std::nothrow) mlmc_server_s();
    if (!srv) return MLMC_E_NOMEM;
    srv->cfg = *cfg;
    srv->cfg.max_batch = slot_samples;
    srv->device = device;
    srv->slot_samples = slot_samples;
    srv->slots.resize(num_slots);
    mlmc_status st = MLMC_OK;
    int64_t cap_max = 1;
    for (auto &sl : srv->slots) {
        st = mlmc::create_ctx(&srv->cfg, device, srv->slots[0].ctx, &sl.ctx);
        if (st) break;
        if (srv->cap.empty()) {      // the same workspace in every slot
            srv->nq = mlmc_num_qoi(sl.ctx);
            for (int l = 0; l < cfg->num_levels; ++l) {
                srv->cap.push_back(mlmc::level_capacity(sl.ctx, l));
                cap_max = std::max(cap_max, srv->cap.back());
            }
        }
        const size_t qsize = sizeof(double) * (size_t)cap_max * cfg->num_levels * srv->nq;
        const size_t ssize = 2 * qsize;       // one segment per sample at most
        const size_t gsize = sizeof(int64_t) * 2 * (size_t)cap_max;
        try {
            sl.bad.assign((size_t)cap_max, 0);
            sl.rho.assign((size_t)cap_max, -1.0);
        } catch (...) {
            st = MLMC_E_NOMEM;
            break;
        }
        if (hipSetDevice(device) != hipSuccess || hipStreamCreate(&sl.stream) != hipSuccess ||
            hipMalloc((void **)&sl.y_dev, sizeof(double) * (size_t)cap_max * cfg->s) !=
                hipSuccess ||
            hipMalloc((void **)&sl.q_dev, qsize) != hipSuccess ||
            hipHostMalloc((void **)&sl.q_host, qsize, hipHostMallocDefault) != hipSuccess ||
            hipMalloc((void **)&sl.s_dev, ssize) != hipSuccess ||
            hipHostMalloc((void **)&sl.s_host, ssize, hipHostMallocDefault) != hipSuccess ||
            hipMalloc((void **)&sl.seg_dev, gsize) != hipSuccess ||
            hipHostMalloc((void **)&sl.seg_host, gsize, hipHostMallocDefault) != hipSuccess) {
            st = MLMC_E_NOMEM;
            break;
        }
    }
    if (st) {
        free_slots(srv);
        delete srv;
        return st;
    }
    for (int i = 0; i < num_slots; ++i) srv->slots[i].worker = std::thread(&mlmc_server_s::work, srv, i);
    *out = srv;
    return MLMC_OK;
}

mlmc_status mlmc_server_destroy(mlmc_server srv)
{
    if (!srv) return MLMC_OK;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stopping = true;
    }
    srv->cv_work.notify_all();
    for (auto &sl : srv->slots)
        if (sl.worker.joinable()) sl.worker.join();
    free_slots(srv);
    delete srv;
    return MLMC_OK;
}

mlmc_status mlmc_server_submit(mlmc_server srv, const mlmc_request *req)
{
    if (!srv || !req || !req->qoi_out) return MLMC_E_INVAL;
    const mlmc_config &c = srv->cfg;
    if (req->level < 0 || req->level >= c.num_levels || req->n_begin < 0 ||
        req->n_end <= req->n_begin || req->n_end > ((int64_t)1 << 32) || req->shift_begin < 0 ||
        req->shift_end <= req->shift_begin || req->shift_end > c.num_shifts)
        return MLMC_E_INVAL;
    const int64_t samples = (req->n_end - req->n_begin) * (req->shift_end - req->shift_begin);
    if (samples > srv->cap[req->level]) return MLMC_E_INVAL;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->stopping) return MLMC_E_STATE;
        const Clock::time_point now = Clock::now();
        if (!srv->started) {
            srv->started = true;
            srv->first_submit = now;
        }
        srv->queue.push_back(Pending{*req, samples, now});
    }
    srv->cv_work.notify_one();
    return MLMC_OK;
}

mlmc_status mlmc_server_poll(mlmc_server srv, mlmc_result *out, int32_t max_results,
                             int32_t wait_ms, int32_t *count)
{
    if (!srv || !count || max_results < 0 || (max_results > 0 && !out)) return MLMC_E_INVAL;
    std::unique_lock<std::mutex> lk(srv->mu);
    if (srv->done.empty() && wait_ms > 0)
        srv->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms),
                              [&] { return !srv->done.empty(); });
    int32_t n = 0;
    while (n < max_results && !srv->done.empty()) {
        out[n++] = srv->done.front();
        srv->done.pop_front();
    }
    *count = n;
    return MLMC_OK;
}

int64_t mlmc_server_capacity(mlmc_server srv, int32_t level)
{
    if (!srv || level < 0 || level >= srv->cfg.num_levels) return 0;
    return srv->cap[level];
}

mlmc_status mlmc_server_stats_get(mlmc_server srv, mlmc_server_stats *out)
{
    if (!srv || !out) return MLMC_E_INVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    *out = mlmc_server_stats{};
    out->requests = (int64_t)srv->latencies.size();
    out->samples = srv->n_samples;
    out->batches = srv->n_batches;
    if (!srv->latencies.empty()) {
        std::vector<double> v = srv->latencies;
        std::sort(v.begin(), v.end());
        auto pct = [&](double p) {
            const double x = p * (double)(v.size() - 1);
            const size_t i = (size_t)x;
            const double w = x - (double)i;
            return i + 1 < v.size() ? v[i] * (1.0 - w) + v[i + 1] * w : v[i];
        };
        out->p50_ms = pct(0.5);
        out->p99_ms = pct(0.99);
        out->max_ms = v.back();
        out->busy_s = ms_between(srv->first_submit, srv->last_done) * 1e-3;
    }
    return MLMC_OK;
}

}  // extern "C"
