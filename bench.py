"""Benchmark of the MG-MLQMC per-sample hot path on one MI355X.

One step = one pass of the whole path over one batch: lattice points, KL field
(dense product + exp), FMG with every stage refined to relative residual 1e-10
and the QoI of every stage, level-difference sums, their device-to-host copy
and the estimator.  The batch is 64 Korobov lattice points x 16 random shifts
= 1024 samples at the finest level (1024^2, MLMC levels 4^2 .. 1024^2) of the
mixed-precision workload (s = 400 KL terms, lambda = 0.1, sigma^2 = 2, QoI
mean of u and u(1/2,1/2)).  The mixed path (bf16 digit-product field, FP32
V-cycles inside FP64 flexible CG) is the headline; the FP64 path runs the same
steps on the same batch beside it.  Inputs (generating vector, shifts, KL
basis) are resident in HBM before the timed region.

The last line of stdout is one compact JSON object: mixed samples/s, the FP64
samples/s and their ratio, the per-level QoI difference between the paths,
the roofline of the dominant kernel (HIP events on the library's stream),
samples/s per level, one-point request latency percentiles, and the oracle
timed on the host's cores on the first samples of the same batch, with the
per-level error of each path against it.  Progress and detail go to stderr;
--only-* runs print the other measurements.
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


# algorithmic HBM bytes each profiled kind counts per launch (per cell of the
# grid it runs on, over all samples of the chunk; w = bytes per word of the
# V-cycle type, 4 in the mixed path)
BYTE_MODEL = dict(
    points="Y written, 16 B per sample and term",
    field="Y, Y digits and basis digits (10 B per term and cell) read, a written (12 B per cell)",
    smooth="unfused colour sweep", restrict="unfused", prolong="FMG interpolation: coarse "
    "solution read (n^2/4), fine written, 8 B words", coarse="2x2 solve", qoi="u read once",
    sums="QoI table read once",
    pre="a, u (unless zero or interpolated), f (unless 1) read, u written, f_c written (w/4)",
    post="e_c (w/4), a, u, f (unless 1) read, u written",
    lds="coefficients of the LDS grids read, top-level solution written",
    refine="24+9w B per cell of iterating samples (24+7w at a stage's first step), "
           "w = V-cycle word bytes")

KINDS = ("points", "field", "smooth", "restrict", "prolong", "coarse", "qoi", "sums", "pre", "post",
         "lds", "refine")
KERNEL_NAMES = dict(
    points="k_points", field="k_field_digits (mixed) / k_field_mfma64 (FP64)",
    smooth="k_rbgs (one colour)", restrict="k_resid_restrict", prolong="k_prolong",
    coarse="k_coarse_solve", qoi="k_qoi", sums="k_sums",
    pre="pre pass (2 red-black sweeps + residual + restriction): k_pre_tile / k_stream on "
        "every grid above the LDS-resident ones",
    post="post pass (prolongation + correction + 2 sweeps): k_post_tile / k_stream on every "
         "grid above the LDS-resident ones",
    lds="k_lds_fmg_refine, k_lds_vcycle (LDS-resident grids <= 32^2)",
    refine="one flexible-CG step (>= 64^2): k_fcg_dots+k_fcg_p+k_fcg_x+folds")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# HBM bytes per launch of a kernel from two rocprofv3 --pmc passes (FETCH_SIZE,
# WRITE_SIZE), scaled by the same counters on a 1 GiB copy; valid only while
# the kernel source is the one the counters were taken on.
TRAFFIC_RECORDS = dict(refine="profiles/refine_step_mlqmc_mixed_s400_1024_traffic.txt")


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


def make_context(m, w, max_batch, precision=None):
    import synth
    return m.Context(w["n0"], w["num_levels"], w["s"], w["corr_len"], w["sigma2"],
                     mu0=w["mu0"], mu1=w["mu1"], mu2=w["mu2"], rtol=w["rtol"],
                     max_iters=w["max_iters"],
                     precision=m.MLMC_FP64 if precision is None else precision,
                     qoi_mask=m.MLMC_QOI_MEAN | m.MLMC_QOI_CENTER,
                     genvec=synth.korobov_vector(w["seed"], w["s"]),
                     shifts=synth.shift_table(w["seed"], w["num_levels"], w["num_shifts"], w["s"]),
                     max_batch=max_batch, device=0)


def fp64_fixed_c2(m, torch, args):
    """The FP64 fixed-cycle workload (s = 100, 2^10 points x 16 shifts =
    16384 samples at 256^2, 2 V(2,2) per FMG stage): samples/s of the whole
    path, with the kernel-time breakdown of one step."""
    import synth
    w = synth.workload("mlqmc_fp64_s100")
    dev = torch.device("cuda:0")
    k = w["num_levels"] - 1
    npts, R = 1 << w["lattice_log2n"], w["num_shifts"]
    B = npts * R
    ctx = make_context(m, w, max_batch=B)
    if not args.no_autotune:
        ctx.autotune(k)
    pts = ctx.lattice(k, 0, npts, 0, R)
    sums = torch.zeros((R, 2, k + 1, 2), dtype=torch.float64, device=dev)
    rate = solve_rate(ctx, pts, torch, 1.0, sums=sums)
    breakdown = {}
    for kind in KINDS:
        ctx.profile_begin(kind)
        ctx.fmg_solve(pts, sums=sums)
        r = ctx.profile_end()
        if r["launches"]:
            breakdown[kind] = dict(ms=r["total_ms"], launches=r["launches"],
                                   gbs=r["bytes"] / (r["total_ms"] * 1e-3) / 1e9)
    log(f"[bench] C2 fp64 fixed cycles at 256^2: {rate:.0f} samples/s")
    return dict(workload="mlqmc_fp64_s100 at 256^2, 16384 samples, FP64, 2 V(2,2) per stage",
                samples_per_s=rate, breakdown=breakdown)


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


def speedup_table(runs, pairs=(("S1", "MLMC", "MLQMC"), ("S2", "MLMC", "MG_MLQMC"),
                                 ("S3", "MLQMC", "MG_MLQMC"))):
    """The paper's speedups (table speedup): S1 = time(MLMC) / time(MLQMC),
    S2 = time(MLMC) / time(MG-MLQMC), S3 = time(MLQMC) / time(MG-MLQMC), each
    averaged over the tolerances at which both runs finished."""
    t = {(r["method"], r["eps"]): r["seconds"] for r in runs if r["converged"]}
    out = {}
    for name, a, b in pairs:
        vals = [(e, t[(a, e)] / t[(b, e)]) for (mm, e) in t if mm == a and (b, e) in t]
        if vals:
            out[name] = dict(mean=float(np.mean([v for _, v in vals])),
                             per_eps={f"{e:g}": round(v, 3) for e, v in sorted(vals, reverse=True)})
    return out


def methods(m, torch, eps_list=(2e-3, 1e-3, 5e-4, 2.5e-4, 1.25e-4, 6.25e-5, 3.125e-5,
                                1.5625e-5, 7.8125e-6), budget_s=20.0):
    """The four estimators of the paper on the s = 100 workload (4^2 ..
    256^2, FP64, 2 V(2,2) per FMG stage), each driven to RMSE eps by the
    adaptive driver (Section 3.4): MLMC and MG-MLMC (Monte Carlo points, 16
    independent replicas), MLQMC and MG-MLQMC (Korobov lattice sequence, 16
    random shifts); MG- means the coarse FMG solutions are recycled (eq.
    Upsilon-reuse).  Each method walks down the tolerances until one run
    takes longer than budget_s (so the small tolerances are reached by the
    lattice methods only).  Wall time on the GPU, the share of it spent in
    the library's solves, points per level, finest level and the estimate;
    the paper's S1, S2, S3 averaged over the tolerances both methods reached."""
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
               runs=[], budget_s=budget_s)
    mg_mlqmc(GpuSampler(ctx), eps_list[0], max_level=L1 - 1)      # warm-up
    for name, (mk, reuse) in samplers.items():
        for eps in eps_list:
            sampler = mk()
            t0 = time.perf_counter()
            r = mg_mlqmc(sampler, eps, max_level=L1 - 1, reuse=reuse, max_points=1 << 20)
            dt = time.perf_counter() - t0
            out["runs"].append(dict(method=name, eps=eps, seconds=dt, L=r["L"],
                                    N=r["N"].tolist(), q_bar=r["q_bar"],
                                    sd=float(np.sqrt(r["var"])), bias=r["bias"],
                                    converged=r["converged"],
                                    solve_share=float(np.sum(r["cost"] * r["N"]) * R / dt),
                                    samples=int(np.sum(r["N"]) * R)))
            log(f"[bench] methods {name} eps {eps:g}: {dt:.3f} s, L {r['L']}, "
                f"converged {r['converged']}")
            if dt > budget_s or not r["converged"]:
                break
    out["speedups"] = speedup_table(out["runs"])
    log("[bench] methods speedups: " + json.dumps(out["speedups"]))
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


def recycling_by_smoothness(m, torch, lam=0.3, nus=(0.5, 1.0, 2.0),
                            eps_list=(2e-4, 1e-4, 5e-5, 2.5e-5, 1.25e-5), Q=64, budget_s=20.0):
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
            if runs and max(r["seconds"] for r in runs[-2:]) > budget_s:
                break
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
        out["fields"][f"nu {nu}"] = dict(s=s, runs=runs,
                                         speedups=speedup_table(runs, (("S3", "MLQMC", "MG_MLQMC"),)))
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
        same, noconv = True, 0
        for rep in range(reps):
            t0 = time.perf_counter()
            tags = {srv.submit(*q): q for q in reqs}
            done = []
            while srv.pending():
                done += srv.poll(wait_ms=50)
            dt = time.perf_counter() - t0
            for r in done:
                l, n0, n1, r0, r1 = tags[r["tag"]]
                # samples stopped by the rounding floor are reported (status
                # NOCONV); their QoIs are compared like the others
                same &= r["status"] in (m.MLMC_OK, m.MLMC_E_NOCONV) and bool(
                    np.array_equal(r["qoi"], ref[l][r0 * (n1 - n0):(r0 + 1) * (n1 - n0)]))
                noconv += r["not_converged"]
        st = srv.stats()
        log(f"[bench] uneven, server ({slots} slots): {sum(counts) / dt:.0f} samples/s "
            f"({dt:.2f} s), bitwise equal to one context: {same}")
    out["server"] = dict(seconds=dt, samples_per_s=sum(counts) / dt, batches=st["batches"] // reps,
                         bitwise_equal_to_one_context=same,
                         not_converged_reported=noconv // reps,
                         speedup=out["one_context"]["seconds"] / dt)
    return out


def oracle_baseline(w, level, y_batch, gpu_qoi, seconds, max_samples):
    """The oracle (field by direct summation + CPU FMG to the same rtol + QoI,
    built -O3 -march=native) on the host's cores, over the first samples of
    the GPU step's own batch (same lattice points and shifts), run in groups
    of `threads` samples until `seconds` of wall time have passed.  Its QoIs
    also give the error of each GPU path against the oracle, per level, on
    those samples.  This is the only part of the benchmark that runs the
    oracle."""
    import oracle
    oracle.select_build("fast")
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
    threads = max(1, min(threads, 16))
    P = oracle.Problem(w["n0"], w["num_levels"], w["s"], w["corr_len"], w["sigma2"],
                       mu0=w["mu0"], mu1=w["mu1"], mu2=w["mu2"], rtol=w["rtol"],
                       max_iters=w["max_iters"])
    done, bad, qs = 0, 0, []
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds and done < max_samples:
        nb = min(threads, max_samples - done)
        q, nbad = P.batch(level, y_batch[done:done + nb], 0, nthreads=threads)
        qs.append(q)
        bad += nbad
        done += nb
    dt = time.perf_counter() - t0
    qo = np.concatenate(qs)
    err = {}
    for name, qg in gpu_qoi.items():
        rel = np.abs(qg[:done] - qo) / np.abs(qo)          # [samples][level][nq]
        err[name] = [float(f"{v:.1e}") for v in rel.max(axis=(0, 2))]
    base = dict(value=round(done / dt, 3), unit="samples/s", cores=threads, kind="oracle",
                sample=f"{done} samples of the step's batch, {w['n0'] << level}^2: KL "
                       f"direct sum + CPU FMG to {w['rtol']:g} + QoI, {dt:.1f} s, -O3 "
                       f"-march=native",
                not_converged=bad)
    return base, err, done


def solve_rate(ctx, pts, torch, min_seconds, q=None, sums=None):
    """Samples/s of repeated solves of one point set (synchronised per call)."""
    B = ctx.count(pts)
    ctx.fmg_solve(pts, qoi=q, sums=sums)
    torch.cuda.synchronize()
    reps, t0 = 0, time.perf_counter()
    while True:
        ctx.fmg_solve(pts, qoi=q, sums=sums)
        torch.cuda.synchronize()
        reps += 1
        if time.perf_counter() - t0 >= min_seconds:
            break
    return B * reps / (time.perf_counter() - t0)


def levels_only(m, torch, args):
    """The per-level table of the s = 400 workload on its own (every level's
    own batch, both paths, the finest level included)."""
    import synth
    w = synth.workload("mlqmc_mixed_s400")
    lv = per_level(m, torch, w, torch.device("cuda:0"), autotune=not args.no_autotune)
    return {key: [round(r["mixed"]), round(r["fp64"]), round(r["mixed"] / r["fp64"], 2),
                  float(f"{r['max_rel_diff']:.1e}")] for key, r in lv.items()}


# samples a per-level context is sized for (chunk capacity scales from it)
LEVEL_CTX_BATCH = 1024


def per_level(m, torch, w, dev, min_seconds=0.25, skip_level=None, autotune=True):
    """Samples/s of each path on every level's own batch (2^26 / n^2 lattice
    points of shift 0, at most 65536) and the largest relative QoI difference
    between the paths on it; `skip_level` is measured by the timed steps.
    One path after the other, each on an autotuned context of its own."""
    levels = [k for k in range(w["num_levels"]) if k != skip_level]
    rate, noconv, q = {}, {}, {}
    for name, prec in (("mixed", m.MLMC_MIXED), ("fp64", m.MLMC_FP64)):
        c = make_context(m, w, LEVEL_CTX_BATCH, precision=prec)
        if autotune:
            c.autotune(max(levels))
        for k in levels:
            n = w["n0"] << k
            npts = int(min(65536, max(16, (1 << 26) // (n * n))))
            p = c.lattice(k, 0, npts, 0, 1)
            qq = torch.zeros((npts, k + 1, 2), dtype=torch.float64, device=dev)
            info = c.fmg_solve(p, qoi=qq, want_info=True)
            rate[(name, k)] = solve_rate(c, p, torch, min_seconds, q=qq)
            noconv[(name, k)] = info["not_converged"]
            q[(name, k)] = qq.cpu().numpy()
            del qq
        c.close()
        del c
        torch.cuda.empty_cache()
    rows = {}
    for k in levels:
        n = w["n0"] << k
        row = dict(samples=q[("mixed", k)].shape[0])
        for name in ("mixed", "fp64"):
            row[name] = rate[(name, k)]
            row[f"{name}_not_converged"] = noconv[(name, k)]
        row["max_rel_diff"] = float(np.max(np.abs(q[("mixed", k)] - q[("fp64", k)]) /
                                           np.abs(q[("fp64", k)])))
        rows[f"{n}^2"] = row
        log(f"[bench] level {n}^2: mixed {row['mixed']:.0f} fp64 {row['fp64']:.0f} samples/s "
            f"(x{row['mixed'] / row['fp64']:.2f}), max rel diff {row['max_rel_diff']:.1e}")
    return rows


def latency(m, torch, ctx, w, dev, levels, reps=200):
    """One-point request latency (ABI call to host-visible sums), p50/p99."""
    out = {}
    for k in levels:
        p = ctx.lattice(k, 0, 1, 3, 4)
        s3 = torch.zeros((1, 2, k + 1, 2), dtype=torch.float64, device=dev)
        nrep = reps if k < 7 else max(20, reps // 4)
        times = []
        for i in range(nrep + 5):
            torch.cuda.synchronize()
            ta = time.perf_counter()
            ctx.fmg_solve(p, sums=s3)
            s3.cpu()
            times.append((time.perf_counter() - ta) * 1e3)
        t = np.array(times[5:])
        out[f"{w['n0'] << k}^2"] = [round(float(np.percentile(t, 50)), 3),
                                    round(float(np.percentile(t, 99)), 3)]
    return out


def headline(m, torch, args):
    """Mixed vs FP64 on the s = 400 workload at its finest level (1024^2):
    a step is one batch of points x shifts solved through the whole path
    (points, field, FMG with every stage refined to rtol, QoI of every level,
    level-difference sums, their copy to the host and the estimator).  The
    two paths are measured one after the other, each on a context of its own
    that is released before the next is made (a 2304-sample context at
    1024^2 takes about 212 GB of the GPU's 288)."""
    import synth
    w = synth.workload("mlqmc_mixed_s400")
    dev = torch.device("cuda:0")
    k = w["num_levels"] - 1
    npts, R = args.points, args.shifts
    B = npts * R
    nq = 2
    n_per_level = np.zeros(k + 1, dtype=np.int64)
    n_per_level[k] = npts
    res, y = {}, None
    for name, prec in (("mixed", m.MLMC_MIXED), ("fp64", m.MLMC_FP64)):
        c = make_context(m, w, B, precision=prec)
        if not args.no_autotune:
            ta = time.perf_counter()
            c.autotune(k)
            log(f"[bench] {name} autotune {time.perf_counter() - ta:.2f} s")
        pts = c.lattice(k, 0, npts, 0, R)
        qoi = torch.zeros((B, k + 1, nq), dtype=torch.float64, device=dev)
        sums = torch.zeros((R, nq, k + 1, 2), dtype=torch.float64, device=dev)
        host_sums = np.zeros((k + 1, R, nq, k + 1, 2))
        est = {}

        def step(c=c, pts=pts, qoi=qoi, sums=sums, host_sums=host_sums, est=est):
            c.fmg_solve(pts, qoi=qoi, sums=sums)
            host_sums[k] = sums.cpu().numpy()          # synchronising device-to-host copy
            est.update(m.mlmc_estimate(n_per_level, host_sums, R, nq, True))

        info = c.fmg_solve(pts, qoi=qoi, want_info=True)
        log(f"[bench] {name} {B} samples at {w['n0'] << k}^2: not converged "
            f"{info['not_converged']}, largest residual ratio {info['max_rel_residual']:.2e}, "
            f"at most {info['max_iters_used']} steps per stage")
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        r = dict(info=info, est=est)
        if name == "mixed":
            # kernel-time breakdown of one (untimed) step; the kind with the
            # most time is the dominant kernel whose roofline is measured live
            breakdown = {}
            for kind in KINDS:
                c.profile_begin(kind)
                step()
                pr = c.profile_end()
                if pr["launches"]:
                    breakdown[kind] = dict(ms=round(pr["total_ms"], 3), launches=pr["launches"],
                                           gbs=round(pr["bytes"] / (pr["total_ms"] * 1e-3) / 1e9, 1)
                                           if pr["total_ms"] > 0 else None,
                                           tflops=round(pr["flops"] / (pr["total_ms"] * 1e-3) / 1e12, 1)
                                           if pr["flops"] else None)
            r["breakdown"] = breakdown
            r["dominant"] = max(breakdown, key=lambda kk: breakdown[kk]["ms"])
            c.profile_begin(r["dominant"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        r["elapsed"] = time.perf_counter() - t0
        if name == "mixed":
            r["prof"] = c.profile_end()
            # points of the step's batch, for the oracle (y = Phi^-1 of the lattice points)
            yd = torch.zeros((B, w["s"]), dtype=torch.float64, device=dev)
            c.points_gen(pts, y=yd)
            y = yd.cpu().numpy()
            del yd
        r["qoi"] = qoi.cpu().numpy()
        r["value"] = B * args.steps / r["elapsed"]
        log(f"[bench] {name}: {args.steps} steps in {r['elapsed']:.3f} s -> "
            f"{r['value']:.1f} samples/s")
        res[name] = r
        c.close()
        del c, qoi, sums, step
        torch.cuda.empty_cache()
    return w, k, B, res, y


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--points", type=int, default=144,
                    help="lattice points per shift in one step's batch")
    ap.add_argument("--shifts", type=int, default=16, help="random shifts in one step's batch")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default pass kinds instead of measuring them first")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--cpu-max-samples", type=int, default=64)
    ap.add_argument("--no-extras", action="store_true",
                    help="only the timed steps and their roofline (no per-level table, "
                         "latency or CPU baseline)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 1 GiB device copy (reference for HBM byte counters)")
    ap.add_argument("--only-c2", action="store_true",
                    help="only the FP64 fixed-cycle s = 100 workload at 256^2 (prints its JSON)")
    ap.add_argument("--only-matern", action="store_true",
                    help="only the Matern field families and recycling against smoothness")
    ap.add_argument("--only-methods", action="store_true",
                    help="run only the MLMC / MLQMC / recycling comparison (prints its JSON object)")
    ap.add_argument("--only-serving", action="store_true",
                    help="run only the serving-loop measurement (prints its JSON object)")
    ap.add_argument("--only-uneven", action="store_true",
                    help="run only the uneven-level comparison (prints its JSON object)")
    ap.add_argument("--only-levels", action="store_true",
                    help="run only the per-level mixed vs FP64 table (prints its JSON object)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the path "
              "shards by shift or lattice range with one small all-reduce of the sums, "
              "which this program does not run.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1806_05619_amd as m

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    for flag, fn in ((args.only_uneven, lambda: uneven(m, torch)),
                     (args.only_levels, lambda: levels_only(m, torch, args)),
                     (args.only_serving, lambda: serving(m, torch)),
                     (args.only_methods, lambda: methods(m, torch)),
                     (args.only_c2, lambda: fp64_fixed_c2(m, torch, args)),
                     (args.only_matern, lambda: dict(matern=matern_fields(m, torch),
                                                     recycling=recycling_by_smoothness(m, torch)))):
        if flag:
            print(json.dumps(fn()), flush=True)
            return
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("[bench] copy calibration: 1 GiB read + 1 GiB written")
        del src, dst

    w, k, B, res, y = headline(m, torch, args)
    mixed, fp64 = res["mixed"], res["fp64"]
    prof, dominant = mixed["prof"], mixed["dominant"]
    avg_ms = prof["total_ms"] / max(prof["launches"], 1)
    bytes_per_launch = prof["bytes"] / max(prof["launches"], 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    traffic, traffic_src = measured_traffic(dominant)
    qm, qf = mixed["qoi"], fp64["qoi"]
    diff = np.abs(qm - qf) / np.abs(qf)
    n = w["n0"] << k
    out = dict(metric=METRIC, value=round(mixed["value"], 2), unit="samples/s", n_gpus=1,
               steps=args.steps, warmup=args.warmup,
               ms_per_step=round(mixed["elapsed"] * 1e3 / args.steps, 3),
               higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype="bf16 field digits, f32 V-cycles, f64 CG and sums",
               data="synthetic",
               config=dict(workload=f"mlqmc_mixed_s400 at {n}^2 (s 400, lambda 0.1, sigma^2 2, "
                                    f"levels 4^2..{n}^2, FMG stages to rtol 1e-10)",
                           samples_per_step=B, points=args.points, shifts=args.shifts,
                           level=k),
               fp64_value=round(fp64["value"], 2),
               ratio_mixed_over_fp64=round(mixed["value"] / fp64["value"], 3),
               not_converged=dict(mixed=mixed["info"]["not_converged"],
                                  fp64=fp64["info"]["not_converged"]),
               roofline=dict(kernel=KERNEL_NAMES[dominant], bound="hbm",
                             achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                             frac=round(achieved / HBM_PEAK_GBS, 4),
                             traffic=None if traffic is None else round(traffic),
                             traffic_source=traffic_src, avg_launch_ms=round(avg_ms, 4),
                             launches_per_step=prof["launches"] / args.steps,
                             algorithmic_bytes_per_launch=round(bytes_per_launch),
                             byte_model=BYTE_MODEL[dominant],
                             share_of_step=round(prof["total_ms"] / (mixed["elapsed"] * 1e3), 3)))
    log(f"[bench] estimate of the step's batch: q_bar {mixed['est']['q_bar'][0]:.10g}, "
        f"std {np.sqrt(mixed['est']['var_q'][0]):.4g}")
    log("[bench] breakdown of one mixed step: " + json.dumps(mixed["breakdown"]))
    log("[bench] max rel diff mixed vs fp64 on the step's QoI table, per MLMC level: " +
        json.dumps([float(f"{v:.1e}") for v in diff.max(axis=(0, 2))]))
    if not args.no_extras:
        lv = per_level(m, torch, w, dev, skip_level=k, autotune=not args.no_autotune)
        lv[f"{n}^2"] = dict(samples=B, mixed=mixed["value"], fp64=fp64["value"],
                            max_rel_diff=float(diff.max()))
        out["per_level"] = {key: [round(r["mixed"]), round(r["fp64"]),
                                  round(r["mixed"] / r["fp64"], 2),
                                  float(f"{r['max_rel_diff']:.1e}")] for key, r in lv.items()}
        out["per_level_columns"] = "mixed/s, fp64/s, ratio, max rel diff"
        lc = make_context(m, w, 64, precision=m.MLMC_MIXED)
        out["latency_p50_p99_ms"] = latency(m, torch, lc, w, dev, (0, 4, 8))
        lc.close()
        del lc, res
        torch.cuda.empty_cache()
        log("[bench] CPU baseline (oracle) ...")
        base, err, ns = oracle_baseline(w, k, y, dict(mixed=qm, fp64=qf), args.cpu_seconds,
                                        args.cpu_max_samples)
        out["cpu_baseline"] = base
        out["max_rel_err_vs_oracle_per_level"] = dict(samples=ns, **err)
    print(json.dumps(out, separators=(",", ":")), flush=True)


if __name__ == "__main__":
    main()
