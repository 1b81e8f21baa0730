"""Benchmark of the MG-MLQMC per-sample hot path on one MI355X.

One step = one pass of the whole path over one batch: lattice points, KL field
(dense product + exp), FMG with the QoI of every stage, level-difference sums,
their device-to-host copy and the estimator.  The batch is the finest level of
the MLQMC FP64 workload: 2^10 Korobov lattice points x 16 random shifts =
16384 samples solved on 4^2 .. 256^2 (s = 100 KL terms, lambda = 0.3,
sigma = 1, FMG with 2 V(2,2) cycles per stage, QoI mean of u and u(1/2,1/2)).
Inputs (generating vector, shifts, KL basis) are resident in HBM before the
timed region.

Prints one JSON line (rank 0) with the throughput, the roofline of the
dominant kernel measured live with HIP events on the library's stream, the
per-level throughput, request latency percentiles and the oracle timed on the
host's cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("samples/s per level (KL+FMG) mixed vs FP64 at equal QoI error; p50/p99 latency")
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
BF16_PEAK_TFLOPS = 2500.0


KINDS = ("points", "field", "smooth", "restrict", "prolong", "coarse", "qoi", "sums", "pre", "post",
         "lds", "refine")
KIND_NAMES = {0: "tile32", 1: "tile16", 2: "stream"}
KERNEL_NAMES = dict(
    points="k_points", field="k_field_mfma64", smooth="k_rbgs (one colour)",
    restrict="k_resid_restrict", prolong="k_prolong", coarse="k_coarse_solve", qoi="k_qoi",
    sums="k_sums",
    pre="pre pass (2 red-black sweeps + residual + restriction): k_stream<2,pre> on 32^2.."
        "256^2 (2 and 4 samples per workgroup on 64^2 and 32^2)",
    post="post pass (prolongation + correction + 2 sweeps): k_stream<2,post> on 32^2..256^2 "
         "(2 and 4 samples per workgroup on 64^2 and 32^2)",
    lds="k_lds_fmg_fixed, k_lds_vcycle (LDS-resident grids <= 16^2)",
    refine="k_fcg_* (flexible-CG vector passes, grids >= 64^2)")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# HBM bytes per launch of a kernel from two rocprofv3 --pmc passes (FETCH_SIZE,
# WRITE_SIZE), scaled by the same counters on a 1 GiB copy; valid only while
# the kernel source is the one the counters were taken on.
TRAFFIC_RECORDS = dict(pre="profiles/pre_pass_mlqmc_fp64_s100_256_traffic.txt",
                       post="profiles/post_pass_mlqmc_fp64_s100_256_traffic.txt")


def measured_traffic(kind):
    import hashlib
    rec = TRAFFIC_RECORDS.get(kind)
    if not rec or not os.path.exists(os.path.join(ROOT, rec)):
        return None, "no counter record"
    with open(os.path.join(ROOT, rec)) as fh:
        r = json.load(fh)
    h = hashlib.sha256()
    for src in r["sources"]:
        with open(os.path.join(ROOT, src), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != r["sources_sha256"]:
        return None, f"{rec}: kernel source changed since the counters were taken"
    return r["hbm_bytes_per_launch"], rec


def make_context(m, w, max_batch):
    import synth
    return m.Context(w["n0"], w["num_levels"], w["s"], w["corr_len"], w["sigma2"],
                     mu0=w["mu0"], mu1=w["mu1"], mu2=w["mu2"], rtol=w["rtol"],
                     max_iters=w["max_iters"], precision=m.MLMC_FP64,
                     qoi_mask=m.MLMC_QOI_MEAN | m.MLMC_QOI_CENTER,
                     genvec=synth.korobov_vector(w["seed"], w["s"]),
                     shifts=synth.shift_table(w["seed"], w["num_levels"], w["num_shifts"], w["s"]),
                     max_batch=max_batch, device=0)


def mixed_vs_fp64(m, torch, dev, max_batch=64, min_seconds=0.25):
    """The s = 400 workload (lambda 0.1, sigma^2 2, 4^2 .. 1024^2) with both
    paths run to the same stopping rule (relative residual 1e-10 per FMG
    stage): FP64 CG with FP64 V-cycles and an FP64 product field, against
    FP64 CG with FP32 V-cycles and the bf16 digit-product field.  Per level:
    samples/s of each (lattice points of shift 0, 2^26 / n^2 of them, at most
    65536), their ratio, the largest relative QoI difference between the two,
    step counts and unconverged samples; the field product's time and
    TFLOP/s (issued digit-product flops in the mixed path, 20 s M per sample,
    against the bf16 matrix-core peak; 2 s M in FP64)."""
    import synth
    w = synth.workload("mlqmc_mixed_s400")
    out = dict(workload="mlqmc_mixed_s400: lambda 0.1, sigma^2 2, s = 400, levels 4^2..1024^2, "
                        "FMG with every stage solved to relative residual 1e-10 by V(2,2)-"
                        "preconditioned flexible CG", rtol=w["rtol"], levels={})
    ctxs = {}
    for name, prec in (("fp64", m.MLMC_FP64), ("mixed", m.MLMC_MIXED)):
        ctxs[name] = m.Context(w["n0"], w["num_levels"], w["s"], w["corr_len"], w["sigma2"],
                               mu0=w["mu0"], mu1=w["mu1"], mu2=w["mu2"], rtol=w["rtol"],
                               max_iters=w["max_iters"], precision=prec,
                               qoi_mask=m.MLMC_QOI_MEAN | m.MLMC_QOI_CENTER,
                               genvec=synth.korobov_vector(w["seed"], w["s"]),
                               shifts=synth.shift_table(w["seed"], w["num_levels"],
                                                        w["num_shifts"], w["s"]),
                               max_batch=max_batch, device=0)
    for k in range(w["num_levels"]):
        n = w["n0"] << k
        npts = int(min(65536, max(16, (1 << 26) // (n * n))))
        row = dict(samples=npts)
        q = {}
        for name, c in ctxs.items():
            p = c.lattice(k, 0, npts, 0, 1)
            qq = torch.zeros((npts, k + 1, 2), dtype=torch.float64, device=dev)
            info = c.fmg_solve(p, qoi=qq, want_info=True)
            torch.cuda.synchronize()
            reps, t0 = 0, time.perf_counter()
            while True:
                c.fmg_solve(p, qoi=qq)
                torch.cuda.synchronize()
                reps += 1
                if time.perf_counter() - t0 >= min_seconds:
                    break
            dt = (time.perf_counter() - t0) / reps
            c.profile_begin("field")
            c.fmg_solve(p, qoi=qq)
            fr = c.profile_end()
            row[f"{name}_field_ms"] = fr["total_ms"]
            row[f"{name}_field_tflops"] = fr["flops"] / (fr["total_ms"] * 1e-3) / 1e12
            row[f"{name}_samples_per_s"] = npts / dt
            row[f"{name}_max_steps"] = info["max_iters_used"]
            row[f"{name}_not_converged"] = info["not_converged"]
            q[name] = qq.cpu().numpy()
        row["ratio_mixed_over_fp64"] = row["mixed_samples_per_s"] / row["fp64_samples_per_s"]
        row["max_rel_qoi_diff"] = float(np.max(np.abs(q["mixed"] - q["fp64"]) / np.abs(q["fp64"])))
        out["levels"][f"{n}^2"] = row
        row["field_digits_frac_of_bf16_peak"] = row["mixed_field_tflops"] / BF16_PEAK_TFLOPS
        log(f"[bench] mixed vs fp64 {n}^2: {row['mixed_samples_per_s']:.0f} vs "
            f"{row['fp64_samples_per_s']:.0f} samples/s (x{row['ratio_mixed_over_fp64']:.2f}), "
            f"max rel diff {row['max_rel_qoi_diff']:.1e}")
    del ctxs
    return out


def serving(m, torch, seconds=4.0, rate=500.0, clients=4, slots=4, slot_samples=64,
            eps=1e-4):
    """The serving loop (mlmc_server) on the s = 1000 workload (lambda 0.05,
    4^2 .. 2048^2, FP64, 2 V(2,2) per FMG stage).  Open loop: jobs arrive as a
    Poisson process, each an adaptive MLQMC estimate (Algorithm 1) to RMSE
    `eps` on its own group of 16 random shifts, whose (level, lattice range,
    shift) requests go through the server while other jobs run; the job rate
    is set so that requests arrive at `rate` per second on average.  Reported:
    request latency p50/p99 (submit to QoIs on the host), job latency,
    samples/s.  Saturated: 4000 single-shift requests of 64 points (level l
    with probability ~2^-l) submitted at once, against the same requests
    solved one call at a time on one context."""
    import threading
    import synth
    from paper_1806_05619_amd.driver import ServerSampler, mg_mlqmc
    w = synth.workload("serving_fp64_s1000")
    L1, R = w["num_levels"], w["num_shifts"]
    kw = dict(n0=w["n0"], num_levels=L1, s=w["s"], corr_len=w["corr_len"], sigma2=w["sigma2"],
              mu0=w["mu0"], mu1=w["mu1"], mu2=w["mu2"], rtol=w["rtol"], max_iters=w["max_iters"],
              precision=m.MLMC_FP64, qoi_mask=m.MLMC_QOI_MEAN | m.MLMC_QOI_CENTER,
              genvec=synth.korobov_vector(w["seed"], w["s"]),
              shifts=synth.shift_table(w["seed"], L1, R * clients, w["s"]))
    rng = np.random.default_rng(11)
    out = dict(workload="serving_fp64_s1000: s = 1000, lambda 0.05, sigma^2 1, levels 4^2..2048^2, "
                        "FP64, 2 V(2,2) cycles per FMG stage",
               slots=slots, slot_samples=slot_samples, eps=eps)
    with m.Server(**kw, num_slots=slots, slot_samples=slot_samples, device=0) as srv:
        def job(c):
            t0 = time.perf_counter()
            r = mg_mlqmc(ServerSampler(srv, R, first_shift=R * (c % clients)), eps,
                         max_level=L1 - 1, max_points=1 << w["lattice_log2n"])
            return time.perf_counter() - t0, r

        job(0)                                   # warm-up; calibrates requests per job
        s0 = srv.stats()
        job(1)
        per_job = srv.stats()["requests"] - s0["requests"]
        job_rate = rate / max(per_job, 1)
        base = srv.stats()
        srv.take_latencies()
        results, threads = [], []
        lock = threading.Lock()

        def run(c):
            res = job(c)
            with lock:
                results.append(res)

        t0 = time.perf_counter()
        t_next, c = t0, 0
        while t_next < t0 + seconds:
            time.sleep(max(0.0, t_next - time.perf_counter()))
            th = threading.Thread(target=run, args=(c,))
            th.start()
            threads.append(th)
            c += 1
            t_next += rng.exponential(1.0 / job_rate)
        for th in threads:
            th.join()
        dt = max(time.perf_counter() - t0, seconds)   # arrival window, or longer if a job ran on
        st = srv.stats()
        rl = np.array(srv.take_latencies())
        jl = np.array([r[0] for r in results]) * 1e3
        q = np.array([r[1]["q_bar"] for r in results])
        out["open_loop"] = dict(
            request_rate_per_s=(st["requests"] - base["requests"]) / dt, jobs=len(results),
            requests_per_job=per_job, seconds=dt,
            samples_per_s=(st["samples"] - base["samples"]) / dt,
            batches=st["batches"] - base["batches"],
            request_p50_ms=float(np.percentile(rl, 50)), request_p99_ms=float(np.percentile(rl, 99)),
            request_max_ms=float(rl.max()),
            job_p50_ms=float(np.percentile(jl, 50)), job_p99_ms=float(np.percentile(jl, 99)),
            all_converged=all(r[1]["converged"] for r in results),
            finest_level=max(r[1]["L"] for r in results),
            estimate_mean=float(q.mean()), estimate_spread=float(q.std()),
            estimate_sd_predicted=float(np.mean([np.sqrt(r[1]["var"]) for r in results])))
        log(f"[bench] serving (s = 1000): {len(results)} jobs, "
            f"{out['open_loop']['request_rate_per_s']:.0f} req/s, request p50 "
            f"{np.percentile(rl, 50):.2f} ms p99 {np.percentile(rl, 99):.2f} ms, job p50 "
            f"{out['open_loop']['job_p50_ms']:.0f} ms")

        def draw(n):
            p = 2.0 ** -np.arange(L1)
            lv = rng.choice(L1, size=n, p=p / p.sum())
            r = rng.integers(0, R, size=n)
            n0 = rng.integers(0, 1 << 20, size=n)
            return [(int(a), int(b), int(b) + 64, int(c), int(c) + 1) for a, b, c in zip(lv, n0, r)]

        reqs = draw(4000)
        s1 = srv.stats()
        t0 = time.perf_counter()
        tags = [srv.submit(*q) for q in reqs]
        res = srv.collect(tags)
        dt = time.perf_counter() - t0
        lat = np.array([r["latency_ms"] for r in res])
        out["saturated"] = dict(requests=len(reqs), samples_per_s=len(reqs) * 64 / dt,
                                batches=srv.stats()["batches"] - s1["batches"],
                                p50_ms=float(np.percentile(lat, 50)),
                                p99_ms=float(np.percentile(lat, 99)))
    kw["shifts"] = synth.shift_table(w["seed"], L1, R, w["s"])
    ctx = m.Context(**kw, max_batch=64, device=0)
    qd = torch.zeros((64, L1, 2), dtype=torch.float64, device="cuda:0")
    t0 = time.perf_counter()
    for r in reqs[:400]:
        ctx.fmg_solve(ctx.lattice(*r), qoi=qd)
        qd.cpu()
    dt = time.perf_counter() - t0
    # one adaptive run on this context alone: recycled fractions against
    # Proposition 1 for the rates fitted to its costs and variances
    from paper_1806_05619_amd.driver import GpuSampler, recycling_report
    mg_mlqmc(GpuSampler(ctx), eps, max_level=L1 - 1, max_points=1 << w["lattice_log2n"])
    r1 = mg_mlqmc(GpuSampler(ctx), eps, max_level=L1 - 1, max_points=1 << w["lattice_log2n"])
    rep = recycling_report(r1["N"], r1["cost"], r1["estimate"]["var_level"][0][: r1["L"] + 1])
    out["recycling"] = dict(N=r1["N"].tolist(), cost_us=(r1["cost"] * 1e6).tolist(), **rep,
                            note="beta fitted to var_l * N_l (Monte Carlo rate), lam = 1")
    del ctx
    out["one_call_per_request_samples_per_s"] = 400 * 64 / dt
    out["saturated"]["speedup_over_one_call_per_request"] = (out["saturated"]["samples_per_s"] /
                                                             out["one_call_per_request_samples_per_s"])
    log(f"[bench] serving saturated: {out['saturated']['samples_per_s']:.0f} samples/s "
        f"(x{out['saturated']['speedup_over_one_call_per_request']:.1f} over one call per request)")
    return out


def methods(m, torch, eps_list=(2e-3, 1e-3, 5e-4, 2.5e-4)):
    """The four estimators of the paper on the s = 100 workload (4^2 ..
    256^2, FP64, 2 V(2,2) per FMG stage), each driven by Algorithm 1 to RMSE
    eps: MLMC and MG-MLMC (Monte Carlo points, 16 independent replicas),
    MLQMC and MG-MLQMC (Korobov lattice sequence, 16 random shifts); MG-
    means the coarse FMG solutions are recycled (eq. Upsilon-reuse).  Wall
    time on the GPU, points per level, finest level and the estimate."""
    import synth
    from paper_1806_05619_amd.driver import GpuMcSampler, GpuSampler, mg_mlqmc
    w = synth.workload("mlqmc_fp64_s100")
    L1, R = w["num_levels"], w["num_shifts"]
    ctx = make_context(m, w, max_batch=4096)
    seed = w["seed"]

    def normals(level, r, n0, n1):
        return synth.mc_normals(seed, level, n1, w["s"], replica=r)[n0:n1]

    samplers = dict(MLMC=(lambda: GpuMcSampler(ctx, normals, R), False),
                    MG_MLMC=(lambda: GpuMcSampler(ctx, normals, R), True),
                    MLQMC=(lambda: GpuSampler(ctx), False),
                    MG_MLQMC=(lambda: GpuSampler(ctx), True))
    out = dict(workload="mlqmc_fp64_s100 (s = 100, lambda 0.3, sigma 1, 4^2..256^2, FP64, "
                        "2 V(2,2) per FMG stage), QoI mean(u), 16 shifts / replicas",
               runs=[])
    mg_mlqmc(GpuSampler(ctx), eps_list[0], max_level=L1 - 1)      # warm-up
    for eps in eps_list:
        for name, (mk, reuse) in samplers.items():
            t0 = time.perf_counter()
            r = mg_mlqmc(mk(), eps, max_level=L1 - 1, reuse=reuse, max_points=1 << 16)
            dt = time.perf_counter() - t0
            out["runs"].append(dict(method=name, eps=eps, seconds=dt, L=r["L"],
                                    N=r["N"].tolist(), q_bar=r["q_bar"],
                                    sd=float(np.sqrt(r["var"])), bias=r["bias"],
                                    converged=r["converged"],
                                    samples=int(np.sum(r["N"]) * R)))
        row = {x["method"]: x["seconds"] for x in out["runs"] if x["eps"] == eps}
        log(f"[bench] methods eps {eps:g}: " + ", ".join(f"{k} {v:.3f} s" for k, v in row.items()))
    del ctx
    return out


def matern_fields(m, torch, Q=64, samples=1024, reps=3):
    """The paper's field families (Section 6): isotropic Matern covariance with
    lambda_c in {0.1, 0.3, 0.5} and nu in {0.5, 1, 2}, KL eigenpairs by the
    Nystrom method on Q x Q nodes, s the smallest number of terms that keeps
    99.8% of the variance (the eigenvalues of the Nystrom matrix sum to the
    area of the domain, 1), at most Q^2.  Per field: set-up time of the
    context (eigensolve and basis), and FP64 samples/s on the benchmark's
    grids (4^2 .. 256^2, 2 V(2,2) per FMG stage) for N(0,1) points."""
    out = {}
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(11)
    base = dict(n0=4, sigma2=1.0, mu0=2, mu1=2, mu2=2, field_kind=m.MLMC_FIELD_MATERN,
                nystrom_q=Q, qoi_mask=m.MLMC_QOI_MEAN, device=0)
    for lam in (0.1, 0.3, 0.5):
        for nu in (0.5, 1.0, 2.0):
            # all Q^2 eigenvalues from a context on the 2^2 .. 4^2 grids only
            probe = m.Context(**base, num_levels=1, s=Q * Q, corr_len=lam, nu=nu, max_batch=1)
            th = probe.kl_modes()[2]
            probe.close()
            s = int(min(Q * Q, np.searchsorted(np.cumsum(th), 0.998) + 1))
            t0 = time.perf_counter()
            ctx = m.Context(**base, num_levels=7, s=s, corr_len=lam, nu=nu, max_batch=samples)
            torch.cuda.synchronize()
            t_setup = time.perf_counter() - t0
            y = torch.tensor(rng.standard_normal((samples, s)), device=dev)
            pts = ctx.explicit(6, y)
            q = torch.zeros((samples, 7, 1), dtype=torch.float64, device=dev)
            ctx.fmg_solve(pts, qoi=q)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                ctx.fmg_solve(pts, qoi=q)
            torch.cuda.synchronize()
            rate = samples * reps / (time.perf_counter() - t0)
            key = f"lambda {lam} nu {nu}"
            out[key] = dict(s=s, variance_kept=float(np.sum(th[:s])), setup_s=t_setup,
                            samples_per_s=rate, mean_qoi_256=float(q[:, 6, 0].mean()))
            log(f"[bench] matern {key}: s {s} ({np.sum(th[:s]):.4f} of the variance), "
                f"set-up {t_setup:.2f} s, {rate:.0f} samples/s at 256^2")
            del ctx, y, q
            torch.cuda.empty_cache()
    return dict(workload=f"isotropic Matern fields, Nystrom on {Q}x{Q} nodes, sigma^2 1, FP64, "
                         f"4^2..256^2, 2 V(2,2) per stage, {samples} N(0,1) samples",
                fields=out)


def recycling_by_smoothness(m, torch, lam=0.3, nus=(0.5, 1.0, 2.0), eps_list=(2e-4, 1e-4, 5e-5),
                            Q=64):
    """Section 6's finding on this implementation: recycling the coarse FMG
    solutions pays more for rougher fields.  For Matern fields of correlation
    length lam and smoothness nu (s by the 99.8% rule on Q x Q Nystrom
    nodes), Algorithm 1 with lattice points (16 shifts) runs to RMSE eps
    without (MLQMC) and with (MG-MLQMC) recycling.  Per run: GPU wall time,
    points per level, finest level; for MG-MLQMC the recycled fractions and
    the cost of its own sample counts with recycling over without
    (Proposition 1's quantity, independent of timing noise)."""
    import synth
    from paper_1806_05619_amd.driver import GpuSampler, mg_mlqmc, recycling_report
    out = dict(workload=f"isotropic Matern, lambda_c {lam}, sigma^2 1, Nystrom {Q}x{Q}, "
                        "4^2..256^2, FP64, 2 V(2,2) per stage, QoI mean(u), 16 shifts",
               fields={})
    seed, L1, R = 5, 7, 16
    for nu in nus:
        probe = m.Context(n0=4, num_levels=1, s=Q * Q, corr_len=lam, sigma2=1.0,
                          field_kind=m.MLMC_FIELD_MATERN, nu=nu, nystrom_q=Q, max_batch=1,
                          device=0)
        th = probe.kl_modes()[2]
        probe.close()
        s = int(min(Q * Q, np.searchsorted(np.cumsum(th), 0.998) + 1))
        ctx = m.Context(n0=4, num_levels=L1, s=s, corr_len=lam, sigma2=1.0, mu0=2, mu1=2, mu2=2,
                        field_kind=m.MLMC_FIELD_MATERN, nu=nu, nystrom_q=Q,
                        qoi_mask=m.MLMC_QOI_MEAN | m.MLMC_QOI_CENTER,
                        genvec=synth.korobov_vector(seed, s),
                        shifts=synth.shift_table(seed, L1, R, s), max_batch=4096, device=0)
        mg_mlqmc(GpuSampler(ctx), eps_list[0], max_level=L1 - 1)      # warm-up
        runs = []
        for eps in eps_list:
            row = {}
            for name, reuse in (("MLQMC", False), ("MG_MLQMC", True)):
                t0 = time.perf_counter()
                r = mg_mlqmc(GpuSampler(ctx), eps, max_level=L1 - 1, reuse=reuse,
                             max_points=1 << 20)
                dt = time.perf_counter() - t0
                run = dict(method=name, eps=eps, seconds=dt, L=r["L"], N=r["N"].tolist(),
                           q_bar=r["q_bar"], converged=r["converged"])
                if reuse:
                    rep = recycling_report(r["N"], r["cost"])
                    run["new_fraction"] = rep["new_fraction"]
                    run["cost_with_over_without"] = rep["cost_ratio"]
                runs.append(run)
                row[name] = run
            log(f"[bench] recycling nu {nu} (s {s}) eps {eps:g}: MLQMC {row['MLQMC']['seconds']:.3f} s "
                f"(L {row['MLQMC']['L']}), MG-MLQMC {row['MG_MLQMC']['seconds']:.3f} s "
                f"(L {row['MG_MLQMC']['L']}), its cost with/without recycling "
                f"{row['MG_MLQMC']['cost_with_over_without']:.2f}, converged "
                f"{row['MLQMC']['converged'] and row['MG_MLQMC']['converged']}")
        out["fields"][f"nu {nu}"] = dict(s=s, runs=runs)
        del ctx
        torch.cuda.empty_cache()
    return out


def uneven(m, torch, slots=3, reps=2):
    """Uneven levels: 4^2 .. 2048^2 with 2^(16-l) samples on level l (all 16
    shifts), mixed path refined to 1e-10.  One context solving the levels one
    call after another, against the serving loop with `slots` slots given the
    whole mixed queue at once (one request per level and shift, finest levels
    first), whose batches of different levels overlap on the device.  Every
    sample's QoIs must be bitwise those of the one-context run."""
    import synth
    w = synth.workload("uneven_mixed_s400")
    L1, R = w["num_levels"], w["num_shifts"]
    counts = w["samples_per_level"]
    finest = counts[-1]
    kw = dict(n0=w["n0"], num_levels=L1, s=w["s"], corr_len=w["corr_len"], sigma2=w["sigma2"],
              mu0=w["mu0"], mu1=w["mu1"], mu2=w["mu2"], rtol=w["rtol"], max_iters=w["max_iters"],
              precision=m.MLMC_MIXED, qoi_mask=m.MLMC_QOI_MEAN | m.MLMC_QOI_CENTER,
              genvec=synth.korobov_vector(w["seed"], w["s"]),
              shifts=synth.shift_table(w["seed"], L1, R, w["s"]))
    dev = torch.device("cuda:0")
    out = dict(workload="uneven_mixed_s400: levels 4^2..2048^2, 2^(16-l) samples on level l "
                        f"({sum(counts)} in all, {R} shifts), s = 400, lambda 0.1, sigma^2 2, "
                        "mixed path, every FMG stage refined to relative residual 1e-10",
               slots=slots, levels={})
    ctx = m.Context(**kw, max_batch=finest, device=0)
    ref = {}
    for rep in range(reps):           # the last repetition is timed
        t_all = 0.0
        for l in range(L1):
            npts = counts[l] // R
            q = torch.empty((npts * R, l + 1, 2), dtype=torch.float64, device=dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = ctx.fmg_solve(ctx.lattice(l, 0, npts, 0, R), qoi=q, want_info=True)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            t_all += dt
            ref[l] = q.cpu().numpy()
            out["levels"][f"{w['n0'] << l}^2"] = dict(samples=counts[l], one_call_s=dt,
                                                       samples_per_s=counts[l] / dt,
                                                       not_converged=info["not_converged"],
                                                       max_steps=info["max_iters_used"])
        log(f"[bench] uneven, one context: {sum(counts) / t_all:.0f} samples/s ({t_all:.2f} s)")
    out["one_context"] = dict(seconds=t_all, samples_per_s=sum(counts) / t_all)
    del ctx
    torch.cuda.empty_cache()
    reqs = [(l, 0, counts[l] // R, r, r + 1) for l in reversed(range(L1)) for r in range(R)]
    with m.Server(**kw, num_slots=slots, slot_samples=finest, device=0) as srv:
        same = True
        for rep in range(reps):
            t0 = time.perf_counter()
            tags = {srv.submit(*q): q for q in reqs}
            done = []
            while srv.pending():
                done += srv.poll(wait_ms=50)
            dt = time.perf_counter() - t0
            for r in done:
                l, n0, n1, r0, r1 = tags[r["tag"]]
                same &= r["status"] == m.MLMC_OK and bool(
                    np.array_equal(r["qoi"], ref[l][r0 * (n1 - n0):(r0 + 1) * (n1 - n0)]))
        st = srv.stats()
        log(f"[bench] uneven, server ({slots} slots): {sum(counts) / dt:.0f} samples/s "
            f"({dt:.2f} s), bitwise equal to one context: {same}")
    out["server"] = dict(seconds=dt, samples_per_s=sum(counts) / dt, batches=st["batches"] // reps,
                         bitwise_equal_to_one_context=same,
                         speedup=out["one_context"]["seconds"] / dt)
    return out


def cpu_baseline(w, level, seconds):
    """The oracle (field by direct summation + CPU FMG + QoI) on the host's
    cores, over the first lattice points of shift 0 at the same level, run in
    batches until `seconds` of wall time have passed."""
    import oracle
    import synth
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
    threads = max(1, min(threads, 16))
    P = oracle.Problem(w["n0"], w["num_levels"], w["s"], w["corr_len"], w["sigma2"],
                       mu0=w["mu0"], mu1=w["mu1"], mu2=w["mu2"])
    z = synth.korobov_vector(w["seed"], w["s"])
    D = synth.shift_table(w["seed"], w["num_levels"], w["num_shifts"], w["s"])
    def run(nthreads, secs, n0):
        done = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < secs:
            nb = 2 * nthreads
            _, y = oracle.points(z, D[level, 0], n0 + done, n0 + done + nb)
            P.batch(level, y, 0, nthreads=nthreads)
            done += nb
        return done, time.perf_counter() - t0

    done, dt = run(threads, seconds, 0)
    done1, dt1 = run(1, max(1.0, seconds / 4), done)
    return dict(value=done / dt, unit="samples/s", cores=threads, kind="oracle",
                sample=f"{done} lattice samples (shift 0, points 0..{done - 1}) at level "
                       f"{level} ({w['n0'] << level}^2): direct-sum KL field + CPU FMG + QoI, "
                       f"{dt:.1f} s wall",
                single_thread_value=done1 / dt1,
                single_thread_sample=f"{done1} further samples on one thread, {dt1:.1f} s wall")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default pass kinds instead of measuring them first")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip per-level, latency and CPU-baseline measurements")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 1 GiB device copy (reference for HBM byte counters)")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-vs-FP64 comparison on the s = 400 workload")
    ap.add_argument("--only-mixed", action="store_true",
                    help="run only the mixed-vs-FP64 comparison (prints its JSON object)")
    ap.add_argument("--only-matern", action="store_true",
                    help="only the Matern field families and recycling against smoothness")
    ap.add_argument("--only-methods", action="store_true",
                    help="run only the MLMC / MLQMC / recycling comparison (prints its JSON object)")
    ap.add_argument("--only-serving", action="store_true",
                    help="run only the serving-loop measurement (prints its JSON object)")
    ap.add_argument("--only-uneven", action="store_true",
                    help="run only the uneven-level comparison (prints its JSON object)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the path "
              "shards by shift or lattice range with one small all-reduce of the sums, "
              "which this build does not run.", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_1806_05619_amd as m

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.only_mixed:
        print(json.dumps(mixed_vs_fp64(m, torch, dev)), flush=True)
        return
    if args.only_uneven:
        print(json.dumps(uneven(m, torch)), flush=True)
        return
    if args.only_serving:
        print(json.dumps(serving(m, torch)), flush=True)
        return
    if args.only_methods:
        print(json.dumps(methods(m, torch)), flush=True)
        return
    if args.only_matern:
        print(json.dumps(dict(matern=matern_fields(m, torch),
                              recycling=recycling_by_smoothness(m, torch))), flush=True)
        return
    w = synth.workload("mlqmc_fp64_s100")
    k = w["num_levels"] - 1
    npts = 1 << w["lattice_log2n"]
    R = w["num_shifts"]
    B = npts * R
    nq = 2
    ctx = make_context(m, w, max_batch=B)
    pts = ctx.lattice(k, 0, npts, 0, R)
    sums = torch.zeros((R, nq, k + 1, 2), dtype=torch.float64, device=dev)
    n_per_level = np.zeros(k + 1, dtype=np.int64)
    n_per_level[k] = npts
    host_sums = np.zeros((k + 1, R, nq, k + 1, 2))
    est = {}

    def step():
        ctx.fmg_solve(pts, sums=sums)
        host_sums[k] = sums.cpu().numpy()          # synchronising device-to-host copy
        est.update(m.mlmc_estimate(n_per_level, host_sums, R, nq, True))

    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("[bench] copy calibration: 1 GiB read + 1 GiB written")
        del src, dst
    tune = None
    if not args.no_autotune:
        # pass kinds of the tile grids measured on this device (setup, untimed)
        ta = time.perf_counter()
        table = ctx.autotune(k)
        tune = dict(seconds=time.perf_counter() - ta,
                    measured=[[e["n"], e["batch_class"], KIND_NAMES[e["pre"]], KIND_NAMES[e["post"]],
                               round(e["pre_ms"], 4), round(e["post_ms"], 4)]
                              for e in table if e["pre_ms"] > 0])
        log(f"[bench] autotune {tune['seconds']:.2f} s")
    log(f"[bench] workload mlqmc_fp64_s100 level {k}: {B} samples, warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # kernel-time breakdown of one (untimed) step; the kind with the most time
    # is the dominant kernel whose roofline is measured over the timed steps
    breakdown = {}
    for kind in KINDS:
        ctx.profile_begin(kind)
        step()
        r = ctx.profile_end()
        if r["launches"]:
            breakdown[kind] = dict(ms=r["total_ms"], launches=r["launches"],
                                   gbs=r["bytes"] / (r["total_ms"] * 1e-3) / 1e9 if r["total_ms"] > 0 else None,
                                   tflops=r["flops"] / (r["total_ms"] * 1e-3) / 1e12 if r["flops"] else None)
    dominant = max(breakdown, key=lambda kk: breakdown[kk]["ms"])

    ctx.profile_begin(dominant)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile_end()
    elapsed = t1 - t0
    value = B * args.steps / elapsed
    log(f"[bench] timed {args.steps} steps in {elapsed:.3f} s -> {value:.1f} samples/s")

    avg_ms = prof["total_ms"] / max(prof["launches"], 1)
    bytes_per_launch = prof["bytes"] / max(prof["launches"], 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    traffic, traffic_src = measured_traffic(dominant)
    roofline = dict(kernel=KERNEL_NAMES[dominant], bound="hbm",
                    achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=achieved / HBM_PEAK_GBS, traffic=traffic, traffic_source=traffic_src,
                    avg_launch_ms=avg_ms, launches_per_step=prof["launches"] / args.steps,
                    algorithmic_bytes_per_launch=bytes_per_launch,
                    share_of_step=prof["total_ms"] / (elapsed * 1e3))

    out = dict(metric=METRIC, value=value, unit="samples/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=elapsed * 1e3 / args.steps,
               higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f64",
               data="synthetic",
               config=dict(workload="mlqmc_fp64_s100: MLQMC FP64, lognormal KL field "
                                    "(separable exponential, lambda 0.3, sigma 1, s = 100), "
                                    "FMG 2 x V(2,2) from 2^2, finest level 256^2 "
                                    "(MLMC levels 4^2..256^2), 2^10 Korobov lattice points "
                                    "x 16 shifts = 16384 samples per step, QoI mean(u) and "
                                    "u(1/2,1/2)",
                           samples_per_step=B, level=k, finest_grid=f"{w['n0'] << k}^2",
                           precision="fp64"),
               roofline=roofline, mixed=None,
               estimate=dict(q_bar=float(est["q_bar"][0]), std=float(np.sqrt(est["var_q"][0]))))

    out["kernel_breakdown_one_step"] = breakdown
    out["autotune"] = tune
    if not args.no_extras:
        # samples/s per level, same batch size (16384 samples finest at each level)
        per_level = {}
        for lev in range(k + 1):
            p = ctx.lattice(lev, 0, npts, 0, R)
            s2 = torch.zeros((R, nq, lev + 1, 2), dtype=torch.float64, device=dev)
            ctx.fmg_solve(p, sums=s2)
            torch.cuda.synchronize()
            reps = 3
            ta = time.perf_counter()
            for _ in range(reps):
                ctx.fmg_solve(p, sums=s2)
                s2.cpu()
            torch.cuda.synchronize()
            per_level[f"{w['n0'] << lev}^2"] = B * reps / (time.perf_counter() - ta)
        out["samples_per_s_per_level"] = per_level
        # request latency: one (level, lattice range, shift) call, from the ABI
        # call to host-visible sums, per level and request size
        lat = {}
        for lev in range(k + 1):
            for nreq in (1, 64, 1024):
                p = ctx.lattice(lev, 0, nreq, 3, 4)
                s3 = torch.zeros((1, nq, lev + 1, 2), dtype=torch.float64, device=dev)
                reps = 1000 if nreq * 4 ** lev <= 64 * 4 ** 6 else 200
                times = []
                for i in range(reps + 10):
                    torch.cuda.synchronize()
                    ta = time.perf_counter()
                    ctx.fmg_solve(p, sums=s3)
                    s3.cpu()
                    times.append((time.perf_counter() - ta) * 1e3)
                times = np.array(times[10:])
                lat[f"level{lev}_{w['n0'] << lev}^2_n{nreq}"] = dict(
                    p50_ms=float(np.percentile(times, 50)), p99_ms=float(np.percentile(times, 99)),
                    repeats=reps)
        log("[bench] latency 256^2: " + ", ".join(
            f"n{q} {lat[f'level{k}_256^2_n{q}']['p50_ms']:.2f}/{lat[f'level{k}_256^2_n{q}']['p99_ms']:.2f} ms"
            for q in (1, 64, 1024)))
        out["latency"] = lat
        out["serving"] = serving(m, torch)
        out["methods"] = methods(m, torch)
        out["matern"] = matern_fields(m, torch)
        out["recycling_by_smoothness"] = recycling_by_smoothness(m, torch)
        if not args.no_mixed:
            del ctx
            torch.cuda.empty_cache()
            out["uneven"] = uneven(m, torch)
            torch.cuda.empty_cache()
            out["mixed"] = mixed_vs_fp64(m, torch, dev)
        log("[bench] extras done; CPU baseline ...")
        out["cpu_baseline"] = cpu_baseline(w, k, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
