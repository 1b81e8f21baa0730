"""GPU tests of the serving loop (mlmc_server_*): requests of mixed levels and
sizes, batched by the server, give bitwise the QoIs of the same lattice
points solved alone through mlmc_fmg_solve; the batch-size dependent kernel
choices keep every sample's result independent of its batch."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1806_05619_amd as m  # noqa: E402


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _kw(w, precision):
    return dict(n0=w["n0"], num_levels=w["num_levels"], s=w["s"], corr_len=w["corr_len"],
                sigma2=w["sigma2"], mu0=w["mu0"], mu1=w["mu1"], mu2=w["mu2"], rtol=w["rtol"],
                max_iters=w["max_iters"], precision=precision,
                qoi_mask=m.MLMC_QOI_MEAN | m.MLMC_QOI_CENTER,
                genvec=synth.korobov_vector(w["seed"], w["s"]),
                shifts=synth.shift_table(w["seed"], w["num_levels"], w["num_shifts"], w["s"]))


def _direct(ctx, level, n0, n1, r0, r1):
    pts = ctx.lattice(level, n0, n1, r0, r1)
    q = torch.full((ctx.count(pts), level + 1, ctx.nq), float("nan"), dtype=torch.float64,
                   device="cuda:0")
    ctx.fmg_solve(pts, qoi=q)
    torch.cuda.synchronize()
    return q.cpu().numpy()


def _drain(srv, want, timeout_polls=600):
    got = []
    for _ in range(timeout_polls):
        got += srv.poll(max_results=256, wait_ms=100)
        if len(got) == want:
            break
    return got


def _requests(rng, num_levels, n_req, max_samples):
    reqs = []
    for i in range(n_req):
        level = int(rng.integers(0, num_levels))
        r0 = int(rng.integers(0, 16))
        r1 = min(16, r0 + int(rng.integers(1, 4)))
        npts = int(rng.integers(1, max_samples // (r1 - r0) + 1))
        n0 = int(rng.integers(0, 1000))
        reqs.append((level, n0, n0 + npts, r0, r1))
    return reqs


@pytest.mark.parametrize("name,precision,max_level,slots", [
    ("mlqmc_fp64_s100", m.MLMC_FP64, 6, 3),
    ("mlqmc_mixed_s400", m.MLMC_MIXED, 4, 2),
])
def test_server_results_equal_direct_solves(name, precision, max_level, slots):
    _dev()
    w = synth.workload(name)
    kw = _kw(w, precision)
    slot_samples = 96
    rng = np.random.default_rng(7)
    # two big finest-level requests keep the slots busy while the rest queue up
    reqs = [(max_level, 0, 48, 0, 2), (max_level, 100, 196, 5, 6)]
    reqs += _requests(rng, max_level + 1, 40, slot_samples)
    print(f"\n{name}: {len(reqs)} requests on {slots} slots of {slot_samples}", flush=True)
    with m.Server(**kw, num_slots=slots, slot_samples=slot_samples, device=0) as srv:
        for tag, r in enumerate(reqs):
            assert srv.submit(*r, tag=tag) == tag
        res = _drain(srv, len(reqs))
        assert len(res) == len(reqs)
        st = srv.stats()
    assert st["requests"] == len(reqs) and st["batches"] < len(reqs), st
    assert st["samples"] == sum((r[2] - r[1]) * (r[4] - r[3]) for r in reqs)
    assert 0 < st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
    assert any(r["batch_samples"] > r["samples"] for r in res)
    ctx = m.Context(**kw, max_batch=slot_samples, device=0)
    for r in res:
        assert r["status"] == m.MLMC_OK, r
        level, n0, n1, r0, r1 = reqs[r["tag"]]
        assert r["level"] == level and r["samples"] == (n1 - n0) * (r1 - r0)
        assert r["queued_ms"] <= r["latency_ms"]
        want = _direct(ctx, level, n0, n1, r0, r1)
        assert np.array_equal(r["qoi"], want), (r["tag"], reqs[r["tag"]])


def test_server_rejects_bad_requests_and_keeps_serving():
    _dev()
    w = synth.workload("mlqmc_fp64_s100")
    kw = _kw(w, m.MLMC_FP64)
    with m.Server(**kw, num_slots=1, slot_samples=32, device=0) as srv:
        # footprint admission: the finest level holds slot_samples, coarser
        # levels as many as fit the same workspace
        caps = [srv.capacity(l) for l in range(w["num_levels"])]
        assert caps[-1] == 32 and all(a >= b for a, b in zip(caps, caps[1:])) and caps[0] > 32
        assert srv.capacity(7) == 0 and srv.capacity(-1) == 0
        for bad in [(7, 0, 1, 0, 1), (-1, 0, 1, 0, 1), (0, 5, 5, 0, 1), (0, 0, 1, 3, 3),
                    (0, 0, 1, 15, 17), (6, 0, 33, 0, 1), (6, 0, 17, 0, 2),
                    (5, 0, caps[5] + 1, 0, 1)]:
            with pytest.raises(m.MlmcError):
                srv.submit(*bad)
        tag = srv.submit(2, 0, 32, 1, 2)
        res = _drain(srv, 1)
    assert len(res) == 1 and res[0]["tag"] == tag and res[0]["status"] == m.MLMC_OK
    ctx = m.Context(**kw, max_batch=32, device=0)
    assert np.array_equal(res[0]["qoi"], _direct(ctx, 2, 0, 32, 1, 2))


def test_large_batch_passes_equal_small_batch_passes():
    """At 256^2 a batch of 1100 samples takes the row-streaming post pass and a
    batch of one the tile post pass; both give the same bits."""
    _dev()
    w = synth.workload("mlqmc_fp64_s100")
    kw = _kw(w, m.MLMC_FP64)
    ctx = m.Context(**kw, max_batch=1100, device=0)
    k = w["num_levels"] - 1
    big = _direct(ctx, k, 0, 1100, 3, 4)
    for n in (0, 517, 1099):
        assert np.array_equal(_direct(ctx, k, n, n + 1, 3, 4)[0], big[n]), n


def test_server_concurrent_clients_collect_their_own_results():
    """Four host threads submit interleaved requests to one server and collect
    their own tags (results polled by one client are kept for the others);
    every result is bitwise the direct solve of its points."""
    import threading
    _dev()
    w = synth.workload("mlqmc_fp64_s100")
    kw = _kw(w, m.MLMC_FP64)
    got, errors = {}, []
    with m.Server(**kw, num_slots=2, slot_samples=64, device=0) as srv:
        def client(c):
            try:
                rng = np.random.default_rng(100 + c)
                reqs = _requests(rng, w["num_levels"], 15, 64)
                tags = [srv.submit(*r) for r in reqs]
                for r, res in zip(reqs, srv.collect(tags, timeout_s=120)):
                    got[(c, res["tag"])] = (r, res)
            except Exception as e:          # reported below, on the main thread
                errors.append(e)
        th = [threading.Thread(target=client, args=(c,)) for c in range(4)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        assert srv.pending() == 0
    assert not errors, errors
    assert len(got) == 60
    ctx = m.Context(**kw, max_batch=64, device=0)
    for (c, tag), (r, res) in got.items():
        assert res["status"] == m.MLMC_OK and res["tag"] == tag
        assert np.array_equal(res["qoi"], _direct(ctx, *r)), (c, tag, r)


def test_server_on_matern_field_equals_direct_solves():
    """Slots of a Matern configuration share the first slot's Nystrom basis;
    every served result is bitwise the direct solve of its points."""
    _dev()
    w = synth.workload("mlqmc_fp64_s100")
    s = 60
    kw = dict(n0=4, num_levels=5, s=s, corr_len=0.3, sigma2=1.0, mu0=2, mu1=2, mu2=2,
              qoi_mask=m.MLMC_QOI_MEAN | m.MLMC_QOI_CENTER, field_kind=m.MLMC_FIELD_MATERN,
              nu=1.0, nystrom_q=16, genvec=synth.korobov_vector(w["seed"], s),
              shifts=synth.shift_table(w["seed"], 5, 16, s))
    rng = np.random.default_rng(21)
    reqs = _requests(rng, 5, 24, 48)
    with m.Server(**kw, num_slots=2, slot_samples=48, device=0) as srv:
        tags = [srv.submit(*r) for r in reqs]
        res = srv.collect(tags, timeout_s=120)
    ctx = m.Context(**kw, max_batch=48, device=0)
    for r, out in zip(reqs, res):
        assert out["status"] == m.MLMC_OK
        assert np.array_equal(out["qoi"], _direct(ctx, *r)), r


@pytest.mark.parametrize("precision", [m.MLMC_FP64, m.MLMC_MIXED])
def test_served_results_against_oracle_and_device_sums(oracle_mod, precision):
    """Requests of several levels through the server (mixed workload, rtol
    1e-10): sampled served QoIs against the oracle's band solve (1e-8), each
    request's per-shift level sums against exactly rounded sums of its
    served QoIs (1e-13) and bitwise against mlmc_fmg_solve's sums for the
    same points alone, and no unconverged sample reported."""
    import math
    _dev()
    w = synth.workload("mlqmc_mixed_s400")
    w["num_levels"] = 6
    kw = _kw(w, precision)
    reqs = [(5, 0, 6, 0, 2), (2, 10, 41, 3, 4), (4, 7, 12, 5, 8), (0, 0, 200, 1, 2),
            (3, 100, 164, 15, 16), (5, 6, 9, 2, 3)]
    with m.Server(**kw, num_slots=2, slot_samples=16, device=0) as srv:
        tags = [srv.submit(*r, sums=True) for r in reqs]
        res = srv.collect(tags, timeout_s=300)
    ctx = m.Context(**kw, max_batch=256, device=0)
    P = oracle_mod.Problem(w["n0"], w["num_levels"], w["s"], w["corr_len"], w["sigma2"],
                           mu0=w["mu0"], mu1=w["mu1"], mu2=w["mu2"], rtol=w["rtol"],
                           max_iters=w["max_iters"])
    z = synth.korobov_vector(w["seed"], w["s"])
    D = synth.shift_table(w["seed"], w["num_levels"], w["num_shifts"], w["s"])
    for (level, n0, n1, r0, r1), out in zip(reqs, res):
        assert out["status"] == m.MLMC_OK and out["not_converged"] == 0, out
        assert 0 < out["max_rel_residual"] <= w["rtol"], out
        Q = out["qoi"]
        npts = n1 - n0
        # device sums: exactly rounded sums of the served QoIs, and the
        # library's own sums for the same points solved alone
        pts = ctx.lattice(level, n0, n1, r0, r1)
        s_dev = torch.zeros((r1 - r0, 2, level + 1, 2), dtype=torch.float64, device="cuda:0")
        ctx.fmg_solve(pts, sums=s_dev)
        assert np.array_equal(out["sums"], s_dev.cpu().numpy()), (level, n0, n1, r0, r1)
        for r in range(r1 - r0):
            Fr = Q[r * npts:(r + 1) * npts]
            d = np.diff(np.concatenate([np.zeros((npts, 1, 2)), Fr], axis=1), axis=1)
            for q in range(2):
                for l in range(level + 1):
                    s1 = math.fsum(d[:, l, q])
                    s2 = math.fsum(d[:, l, q] ** 2)
                    assert abs(out["sums"][r, q, l, 0] - s1) <= 1e-13 * math.fsum(np.abs(d[:, l, q]))
                    assert abs(out["sums"][r, q, l, 1] - s2) <= 1e-13 * s2
        # first and last sample of the request against the band solve
        for b in (0, len(Q) - 1):
            r, n = r0 + b // npts, n0 + b % npts
            _, y = oracle_mod.points(z, D[level, r], n, n + 1)
            qo = P.sample(level, y[0], 1)
            assert np.max(np.abs(Q[b] - qo) / np.abs(qo)) <= 1e-8, (level, r, n)


def test_server_reports_unconverged_samples():
    """An rtol no FP64 residual can reach: every served sample stops at the
    rounding floor, each request reports all its samples as not converged
    with status MLMC_E_NOCONV, and its QoIs are still written."""
    _dev()
    w = synth.workload("mlqmc_fp64_s100")
    kw = _kw(w, m.MLMC_FP64)
    kw.update(rtol=1e-30, max_iters=200, mu0=1, num_levels=5,
              shifts=synth.shift_table(w["seed"], 5, w["num_shifts"], w["s"]))
    reqs = [(4, 0, 3, 0, 1), (1, 5, 9, 2, 4)]
    with m.Server(**kw, num_slots=1, slot_samples=8, device=0) as srv:
        res = srv.collect([srv.submit(*r) for r in reqs], timeout_s=120)
    for (level, n0, n1, r0, r1), out in zip(reqs, res):
        assert out["status"] == m.MLMC_E_NOCONV, out
        assert out["not_converged"] == (n1 - n0) * (r1 - r0), out
        assert 0 < out["max_rel_residual"] <= 1e-12
        assert np.all(np.isfinite(out["qoi"])) and np.all(out["qoi"] > 0)
