"""GPU parity: the HIP path through the C ABI against the CPU oracle on the
same seeded inputs.

Tolerances (derived from the arithmetic, see the design notes):
  lattice points x ............ bit-exact (integer arithmetic)
  normals y ................... |dy| <= 4 ulp(|y|) (two independent FP64 inverse-CDF methods)
  field z (FP64) .............. |dz| <= 1e-13 (s-term dot products of O(1) terms)
  QoI, fixed-cycle FMG ........ relative 1e-12 (same algorithm, different rounding order)
  QoI, rtol refinement ........ relative 1e-10 against the direct band solve
  level-difference sums ....... relative 1e-13 against exactly rounded sums
"""
import ctypes as C
import math

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


def _ctx(name, **over):
    w = synth.workload(name)
    w.update(over)
    kw = dict(n0=w["n0"], num_levels=w["num_levels"], s=w["s"], corr_len=w["corr_len"],
              sigma2=w["sigma2"], mu0=w["mu0"], mu1=w["mu1"], mu2=w["mu2"], rtol=w["rtol"],
              max_iters=w["max_iters"], precision=m.MLMC_FP64,
              qoi_mask=m.MLMC_QOI_MEAN | (m.MLMC_QOI_CENTER if "center" in w["qoi"] else 0),
              max_batch=w.get("max_batch", 64))
    if w["sampling"] == "lattice":
        kw["genvec"] = synth.korobov_vector(w["seed"], w["s"])
        kw["shifts"] = synth.shift_table(w["seed"], w["num_levels"], w["num_shifts"], w["s"])
    return w, m.Context(**kw, device=0)


def _oracle_problem(oracle_mod, w, **over):
    p = dict(mu0=w["mu0"], mu1=w["mu1"], mu2=w["mu2"], rtol=w["rtol"], max_iters=w["max_iters"])
    p.update(over)
    return oracle_mod.Problem(w["n0"], w["num_levels"], w["s"], w["corr_len"], w["sigma2"], **p)


def _lattice_y(oracle_mod, w, level, shifts, n_begin, n_end):
    z = synth.korobov_vector(w["seed"], w["s"])
    D = synth.shift_table(w["seed"], w["num_levels"], w["num_shifts"], w["s"])
    xs, ys = [], []
    for r in shifts:
        x, y = oracle_mod.points(z, D[level, r], n_begin, n_end)
        xs.append(x)
        ys.append(y)
    return np.concatenate(xs), np.concatenate(ys)


def _rel(a, b):
    return np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300))


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n_begin,n_end,shifts", [(0, 1024, (0, 4)), (5, 1000, (3, 5)), (1000, 1001, (15, 16))])
def test_points_bit_exact(oracle_mod, n_begin, n_end, shifts):
    dev = _dev()
    w, ctx = _ctx("mlqmc_fp64_s100")
    level = 3
    pts = ctx.lattice(level, n_begin, n_end, *shifts)
    B = ctx.count(pts)
    x = torch.zeros((B, w["s"]), dtype=torch.int64, device=dev)
    y = torch.zeros((B, w["s"]), dtype=torch.float64, device=dev)
    ctx.points_gen(pts, x, y)
    torch.cuda.synchronize()
    xo, yo = _lattice_y(oracle_mod, w, level, range(*shifts), n_begin, n_end)
    assert np.array_equal(x.cpu().numpy().view(np.uint64), xo)
    yg = y.cpu().numpy()
    ulps = np.abs(yg - yo) / np.spacing(np.abs(yo))
    worst = np.unravel_index(np.argmax(ulps), ulps.shape)
    assert ulps.max() <= 4, f"max {ulps.max():.1f} ulp at y={yo[worst]!r} (gpu {yg[worst]!r})"


@pytest.mark.parametrize("name,k,B", [("mlmc_fp64_s10", 2, 37), ("mlqmc_fp64_s100", 4, 70)])
def test_field_matches_direct_sum(oracle_mod, name, k, B):
    dev = _dev()
    w, ctx = _ctx(name)
    P = _oracle_problem(oracle_mod, w)
    if w["sampling"] == "mc":
        yo = synth.mc_normals(w["seed"], k, B, w["s"])
        pts = ctx.explicit(k, torch.tensor(yo, device=dev))
        keep = pts
    else:
        pts = ctx.lattice(k, 0, B // 2, 0, 2)
        _, yo = _lattice_y(oracle_mod, w, k, range(2), 0, B // 2)
        B = ctx.count(pts)
    M = ctx.field_size(k)
    assert M == P.field_size(k)
    z = torch.zeros((B, M), dtype=torch.float64, device=dev)
    ctx.field(pts, z)
    torch.cuda.synchronize()
    zg = z.cpu().numpy()
    for b in range(B):
        zo = P.field(yo[b], k)
        assert np.max(np.abs(zg[b] - zo)) <= 1e-13, b


def _solve(ctx, pts, nlev, z=None, sums=False, info=False):
    dev = torch.device("cuda:0")
    B = ctx.count(pts)
    q = torch.full((B, nlev, ctx.nq), float("nan"), dtype=torch.float64, device=dev)
    s = torch.zeros((pts.shift_end - pts.shift_begin, ctx.nq, nlev, 2), dtype=torch.float64,
                    device=dev) if sums else None
    res = ctx.fmg_solve(pts, z=z, qoi=q, sums=s, want_info=info)
    torch.cuda.synchronize()
    return q.cpu().numpy(), (s.cpu().numpy() if sums else None), res


@pytest.mark.parametrize("name,ks,B", [("mlmc_fp64_s10", (0, 1, 2), 21), ("mlqmc_fp64_s100", (0, 2, 5), 9)])
def test_fmg_fixed_cycles_match_oracle_fmg(oracle_mod, name, ks, B):
    """Same field (the oracle's) on both sides: isolates the multigrid."""
    dev = _dev()
    w, ctx = _ctx(name)
    P = _oracle_problem(oracle_mod, w)
    rng = np.random.default_rng(100)
    for k in ks:
        ys = rng.standard_normal((B, w["s"]))
        zs = np.stack([P.field(y, k) for y in ys])
        pts = ctx.explicit(k, torch.tensor(ys, device=dev))
        qg, _, _ = _solve(ctx, pts, k + 1, z=torch.tensor(zs, device=dev))
        for b in range(B):
            qo = P.sample_from_field(k, zs[b], 0)["qoi"][:, : ctx.nq]
            assert _rel(qg[b], qo) <= 1e-12, (k, b, qg[b], qo)


@pytest.mark.parametrize("mu1,mu2", [(1, 1), (1, 2), (2, 1)])
def test_fmg_one_sweep_cycles_every_pass_kind(oracle_mod, mu1, mu2):
    """V(1,1), V(1,2) and V(2,1) cycles (Section 4: mu1 pre- and mu2
    post-smoothing sweeps): with the large grids 32^2 .. 128^2 forced to each
    pass kind (32x32 tiles, 16x16 tiles, row streaming, and tiles before
    streaming), the QoIs match the oracle's FMG on the same field and are
    bitwise the same for every kind."""
    dev = _dev()
    w, ctx = _ctx("mlqmc_fp64_s100", mu1=mu1, mu2=mu2)
    P = _oracle_problem(oracle_mod, w)
    k, B = 5, 4                                     # finest MG grid 128^2
    ys = np.random.default_rng(7 + 10 * mu1 + mu2).standard_normal((B, w["s"]))
    zs = np.stack([P.field(y, k) for y in ys])
    qo = np.stack([P.sample_from_field(k, zs[b], 0)["qoi"][:, : ctx.nq] for b in range(B)])
    T32, T16, ST = m.MLMC_PASS_TILE32, m.MLMC_PASS_TILE16, m.MLMC_PASS_STREAM
    first = None
    for pre, post in [(T32, T32), (T16, T16), (ST, ST), (T32, ST), (ST, T16)]:
        ctx.set_tuning(dict(e, pre=pre, post=post) for e in ctx.tuning())
        pts = ctx.explicit(k, torch.tensor(ys, device=dev))
        qg, _, _ = _solve(ctx, pts, k + 1, z=torch.tensor(zs, device=dev))
        assert _rel(qg, qo) <= 1e-12, (pre, post)
        if first is None:
            first = qg
        assert np.array_equal(qg, first), (pre, post)


def test_full_path_matches_oracle(oracle_mod):
    """Points, field, FMG and QoI all on the GPU for lattice samples."""
    _dev()
    w, ctx = _ctx("mlqmc_fp64_s100")
    P = _oracle_problem(oracle_mod, w)
    k = 4
    pts = ctx.lattice(k, 3, 35, 6, 8)
    qg, _, _ = _solve(ctx, pts, k + 1)
    _, yo = _lattice_y(oracle_mod, w, k, range(6, 8), 3, 35)
    qo, bad = P.batch(k, yo, 0)
    assert bad == 0
    assert _rel(qg, qo[:, :, : ctx.nq]) <= 1e-11


def test_rtol_refinement_matches_direct_solve(oracle_mod):
    dev = _dev()
    w, ctx = _ctx("mlqmc_fp64_s100", rtol=1e-12, max_iters=40, mu0=1)
    P = _oracle_problem(oracle_mod, w)
    k = 3
    ys = np.random.default_rng(7).standard_normal((6, w["s"]))
    pts = ctx.explicit(k, torch.tensor(ys, device=dev))
    qg, _, info = _solve(ctx, pts, k + 1, info=True)
    assert info["status"] == m.MLMC_OK and info["not_converged"] == 0
    assert 0 < info["max_rel_residual"] <= 1e-12
    for b in range(len(ys)):
        qd = P.sample(k, ys[b], 1)[:, : ctx.nq]
        assert _rel(qg[b], qd) <= 1e-10, b


def test_rtol_not_converged_reports(oracle_mod):
    dev = _dev()
    w, ctx = _ctx("mlqmc_fp64_s100", rtol=1e-15, max_iters=1, mu0=1)
    ys = np.random.default_rng(8).standard_normal((3, w["s"]))
    pts = ctx.explicit(2, torch.tensor(ys, device=dev))
    qg, _, info = _solve(ctx, pts, 3, info=True)
    assert info["status"] == m.MLMC_E_NOCONV
    assert info["not_converged"] == 3 and info["max_iters_used"] == 1
    assert np.all(np.isfinite(qg))


def test_mlmc_estimate_end_to_end(oracle_mod):
    """Plain MLMC, FP64, N(0,1) samples 256/64/16 on 16^2..64^2: per-sample QoI,
    level-difference sums and the estimator against the oracle."""
    from oracle import estimators as est
    dev = _dev()
    w, ctx = _ctx("mlmc_fp64_s10", max_batch=256)
    P = _oracle_problem(oracle_mod, w)
    L1 = w["num_levels"]
    sums_all = np.zeros((L1, 1, 1, L1, 2))
    F_oracle = []
    for k, N in enumerate(w["samples_per_level"]):
        ys = synth.mc_normals(w["seed"], k, N, w["s"])
        pts = ctx.explicit(k, torch.tensor(ys, device=dev))
        qg, sg, _ = _solve(ctx, pts, k + 1, sums=True)
        qo, bad = P.batch(k, ys, 0)
        assert bad == 0
        assert _rel(qg[:, :, 0], qo[:, :, 0]) <= 1e-12
        # sums against exactly rounded sums of the GPU's own QoI
        for l in range(k + 1):
            d = qg[:, l, 0] - (qg[:, l - 1, 0] if l else 0.0)
            assert abs(sg[0, 0, l, 0] - math.fsum(d)) <= 1e-13 * abs(math.fsum(np.abs(d)))
            assert abs(sg[0, 0, l, 1] - math.fsum(d * d)) <= 1e-13 * math.fsum(d * d)
        sums_all[k, 0, 0, : k + 1] = sg[0, 0]
        F_oracle.append(qo[None, :, :, 0])
    for reuse in (False, True):
        got = m.mlmc_estimate(np.array(w["samples_per_level"]), sums_all, 1, 1, reuse)
        want = est.mlmc_estimate(F_oracle, reuse)
        assert abs(got["q_bar"][0] - want["q_bar"]) <= 1e-11 * abs(want["q_bar"])
        assert np.allclose(got["upsilon"][0, :, 0], want["upsilon"][:, 0], rtol=1e-10, atol=1e-15)
        if not reuse:
            assert abs(got["var_q"][0] - want["var_q"]) <= 1e-8 * want["var_q"]


def test_deterministic_alone_vs_in_batch():
    _dev()
    w, ctx = _ctx("mlqmc_fp64_s100")
    k = 3
    pts = ctx.lattice(k, 0, 40, 1, 3)
    q1, _, _ = _solve(ctx, pts, k + 1)
    q2, _, _ = _solve(ctx, pts, k + 1)
    assert np.array_equal(q1, q2)
    for r in (1, 2):
        for n in (0, 17, 39):
            qa, _, _ = _solve(ctx, ctx.lattice(k, n, n + 1, r, r + 1), k + 1)
            assert np.array_equal(qa[0], q1[(r - 1) * 40 + n])


def test_chunked_equals_single_chunk():
    """max_batch = 3 forces several chunks with a ragged tail."""
    _dev()
    w, big = _ctx("mlqmc_fp64_s100", max_batch=64)
    _, small = _ctx("mlqmc_fp64_s100", max_batch=3)
    k = w["num_levels"] - 1 - 2
    pts = big.lattice(k, 0, 23, 0, 1)
    qa, sa, _ = _solve(big, pts, k + 1, sums=True)
    qb, sb, _ = _solve(small, pts, k + 1, sums=True)
    assert np.array_equal(qa, qb)
    assert np.allclose(sa, sb, rtol=1e-14, atol=0)


def test_empty_batch_and_invalid_points():
    dev = _dev()
    w, ctx = _ctx("mlqmc_fp64_s100")
    q, s, _ = _solve(ctx, ctx.lattice(2, 5, 5, 0, 2), 3, sums=True)
    assert q.shape[0] == 0 and np.all(s == 0.0)
    sentinel = torch.full((4, 3, ctx.nq), 7.0, dtype=torch.float64, device=dev)
    for bad in [ctx.lattice(9, 0, 4), ctx.lattice(2, 0, 4, 0, 17), ctx.lattice(2, 0, 4, 3, 3),
                m.mlmc_points(m.MLMC_POINTS_LATTICE, 2, 0, 1, 0, (1 << 32) + 1, None)]:
        with pytest.raises(m.MlmcError) as e:
            ctx.fmg_solve(bad, qoi=sentinel)
        assert e.value.status == m.MLMC_E_INVAL
    torch.cuda.synchronize()
    assert torch.all(sentinel == 7.0)


def test_full_size_bench_workload_sampled(oracle_mod):
    """The benchmark's launch configuration: 2^10 lattice points x 16 shifts on
    4^2..256^2 in one call.  Sampled samples against the oracle; sums against
    exactly rounded sums of the whole QoI table."""
    _dev()
    w, ctx = _ctx("mlqmc_fp64_s100", max_batch=16384)
    P = _oracle_problem(oracle_mod, w)
    k = w["num_levels"] - 1
    npts = 1 << w["lattice_log2n"]
    R = w["num_shifts"]
    pts = ctx.lattice(k, 0, npts, 0, R)
    qg, sg, _ = _solve(ctx, pts, k + 1, sums=True)
    assert np.all(np.isfinite(qg))
    picks = [(r, n) for r in (0, 7, 15) for n in (0, 1, 511, 1023)]
    for r, n in picks:
        _, yo = _lattice_y(oracle_mod, w, k, [r], n, n + 1)
        qo = P.sample(k, yo[0], 0)[:, : ctx.nq]
        assert _rel(qg[r * npts + n], qo) <= 1e-11, (r, n)
    for r in (0, 9, 15):
        for q in range(ctx.nq):
            for l in range(k + 1):
                blk = qg[r * npts:(r + 1) * npts, :, q]
                d = blk[:, l] - (blk[:, l - 1] if l else 0.0)
                assert abs(sg[r, q, l, 0] - math.fsum(d)) <= 1e-13 * math.fsum(np.abs(d))


@pytest.mark.parametrize("B", [512, 2048])
def test_tile_passes_race_free_at_256(oracle_mod, B):
    """256^2 with many samples per launch (512: tile pre and post passes; 2048:
    tile pre, row-streaming post).  Tiles read their neighbours' cells as
    halo, so every pass writes an array the launch does not read; the result
    is bitwise reproducible across calls and matches the oracle."""
    dev = _dev()
    w, ctx = _ctx("mlqmc_fp64_s100", max_batch=B)
    P = _oracle_problem(oracle_mod, w)
    k = w["num_levels"] - 1
    pts = ctx.lattice(k, 0, B, 0, 1)
    q1, _, _ = _solve(ctx, pts, k + 1)
    q2, _, _ = _solve(ctx, pts, k + 1)
    assert np.array_equal(q1, q2)
    _, ys = _lattice_y(oracle_mod, w, k, [0], 0, 4)
    for b in range(4):
        qo = P.sample(k, ys[b], 0)[:, : ctx.nq]
        assert _rel(q1[b], qo) <= 1e-11, b


def _mixed_ctx(**over):
    w = synth.workload("mlqmc_mixed_s400")
    w.update(over)
    ctx = m.Context(w["n0"], w["num_levels"], w["s"], w["corr_len"], w["sigma2"],
                    mu0=w["mu0"], mu1=w["mu1"], mu2=w["mu2"], rtol=w["rtol"],
                    max_iters=w["max_iters"], precision=over.get("precision", m.MLMC_MIXED),
                    qoi_mask=m.MLMC_QOI_MEAN | m.MLMC_QOI_CENTER,
                    max_batch=w.get("max_batch", 16), device=0)
    return w, ctx


@pytest.mark.parametrize("k,B", [(3, 100), (5, 7)])
def test_mixed_field_digit_bound(oracle_mod, k, B):
    """Mixed-precision field (Section 5 product as bf16 digit products on the
    matrix cores).  With 2^(E_r - 1) <= max_j |y_j| < 2^E_r per sample and
    likewise E_m per cell over the basis column, five digits per operand and
    the fifteen products of weight 2^0 .. 2^-32, each mode contributes at most
    1.6 * 2^(E_r + E_m - 38) (digit remainders below 2^-33 of the scale, dropped
    products of weight 2^-40 and below), so |z - z_fp64| <= 2 s 2^(E_r + E_m -
    38).  The digit sums are exact, so the error has no rounding bias: its mean
    over all cells stays below 1e-12 (FP32-accumulated bf16 splits leave a bias
    of a few 1e-8 here).
    Ragged in both the sample and the column tiles (M, B not multiples of 64)."""
    dev = _dev()
    w, ctx = _mixed_ctx(num_levels=k + 1)
    P = _oracle_problem(oracle_mod, w)
    ys = np.random.default_rng(5 + k).standard_normal((B, w["s"]))
    pts = ctx.explicit(k, torch.tensor(ys, device=dev))
    M = ctx.field_size(k)
    z = torch.full((B, M), float("nan"), dtype=torch.float64, device=dev)
    ctx.field(pts, z)
    torch.cuda.synchronize()
    zg = z.cpu().numpy()
    basis = np.stack([P.field(np.eye(w["s"])[j], k) for j in range(w["s"])])   # [s][M]
    zo = ys @ basis
    Er = np.frexp(np.abs(ys).max(axis=1))[1].astype(float)              # per sample
    Em = np.frexp(np.abs(basis).max(axis=0))[1].astype(float)           # per cell
    bound = 2 * w["s"] * np.exp2(Er[:, None] + Em[None, :] - 38)
    err = zg - zo
    ratio = float(np.max(np.abs(err) / bound))
    print(f"\nmax |z - z_fp64| = {np.abs(err).max():.2e} ({ratio:.2e} of the bound), "
          f"mean error {err.mean():.2e}")
    assert ratio <= 1.0
    assert abs(err.mean()) <= 1e-12


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_rough_lattice_workload_every_sample_converges(oracle_mod, precision):
    """The s = 400, lambda = 0.1, sigma^2 = 2 lattice workload up to 128^2
    (stages <= 32^2 in the LDS-resident kernel, 64^2 and 128^2 in the
    grid-wide flexible-CG passes): every sample of a 96-point batch reaches
    rtol within a few dozen preconditioned steps, and sampled QoIs agree with
    the band Cholesky solve on every level."""
    dev = _dev()
    prec = m.MLMC_MIXED if precision == "mixed" else m.MLMC_FP64
    k = 5
    w = synth.workload("mlqmc_mixed_s400")
    w["num_levels"] = k + 1
    ctx = m.Context(w["n0"], w["num_levels"], w["s"], w["corr_len"], w["sigma2"],
                    mu0=w["mu0"], mu1=w["mu1"], mu2=w["mu2"], rtol=w["rtol"],
                    max_iters=w["max_iters"], precision=prec,
                    qoi_mask=m.MLMC_QOI_MEAN | m.MLMC_QOI_CENTER,
                    genvec=synth.korobov_vector(w["seed"], w["s"]),
                    shifts=synth.shift_table(w["seed"], w["num_levels"], w["num_shifts"], w["s"]),
                    max_batch=96, device=0)
    P = _oracle_problem(oracle_mod, w)
    npts = 96
    pts = ctx.lattice(k, 0, npts, 0, 1)
    qg, _, info = _solve(ctx, pts, k + 1, info=True)
    print(f"\n{precision}: max steps {info['max_iters_used']}, "
          f"max relres {info['max_rel_residual']:.2e}")
    assert info["status"] == m.MLMC_OK and info["not_converged"] == 0, info
    assert info["max_iters_used"] <= 40
    assert 0 < info["max_rel_residual"] <= w["rtol"]
    assert np.all(np.isfinite(qg))
    _, ys = _lattice_y(oracle_mod, w, k, [0], 0, npts)
    tol = 1e-8
    for b in range(0, npts, 24):
        qd = P.sample(k, ys[b], 1)
        rel = np.abs(qg[b] - qd) / np.abs(qd)
        assert rel.max() <= tol, (b, rel)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_refinement_high_contrast_matches_direct_solve(oracle_mod, precision):
    """sigma^2 = 2, lambda = 0.1, s = 400: FP64 residual refinement to 1e-10
    with FP64 or FP32 V-cycles, against the oracle's FP64 field and band
    Cholesky solve on every level up to 128^2 (the batched tile path).  The
    mixed path converges to the operator of its FP64 coefficient copy, so its
    error is that of the digit-product field plus the solve tolerance; it is
    reported per level and held to 1e-8 relative."""
    dev = _dev()
    prec = m.MLMC_MIXED if precision == "mixed" else m.MLMC_FP64
    w, ctx = _mixed_ctx(precision=prec)
    P = _oracle_problem(oracle_mod, w)
    k = 5
    ys = np.random.default_rng(31).standard_normal((3, w["s"]))
    pts = ctx.explicit(k, torch.tensor(ys, device=dev))
    qg, _, info = _solve(ctx, pts, k + 1, info=True)
    assert info["status"] == m.MLMC_OK and info["not_converged"] == 0, info
    assert 0 < info["max_rel_residual"] <= w["rtol"]
    errs = np.zeros((k + 1, 2))
    for b in range(len(ys)):
        qd = P.sample(k, ys[b], 1)
        errs = np.maximum(errs, np.abs(qg[b] - qd) / np.abs(qd))
    print(f"\n{precision}: max relative QoI error per level (mean, centre):\n{errs}")
    tol = 1e-9 if precision == "fp64" else 1e-8
    assert errs.max() <= tol, errs


def test_adaptive_driver_on_gpu():
    """Algorithm 1 (Section 3.4) driving the library on the s = 100 lattice
    workload: reaches its tolerance, every call solves exactly the new lattice
    points of all shifts, and estimates at two tolerances agree within their
    error bounds."""
    from paper_1806_05619_amd.driver import GpuSampler, mg_mlqmc
    _dev()
    w, ctx = _ctx("mlqmc_fp64_s100", max_batch=4096)
    res = {}
    for eps in (4e-3, 2e-3):
        r = mg_mlqmc(GpuSampler(ctx), eps, max_level=w["num_levels"] - 1,
                     max_points=1 << w["lattice_log2n"])
        print(f"\neps {eps}: L {r['L']} N {r['N'].tolist()} q {r['q_bar']:.10f} "
              f"sd {math.sqrt(r['var']):.2e} bias {r['bias']:.2e} alpha {r['alpha']:.2f}")
        assert r["converged"], r
        assert r["var"] <= eps * eps / 2 and r["bias"] <= eps / math.sqrt(2)
        res[eps] = r
    a, b = res[4e-3], res[2e-3]
    assert abs(a["q_bar"] - b["q_bar"]) <= 3 * (4e-3 + 2e-3)


@pytest.mark.parametrize("precision", [m.MLMC_FP64, m.MLMC_MIXED])
def test_unattainable_rtol_stops_at_rounding_floor(oracle_mod, precision):
    """rtol below what an FP64 residual can show: every stage, in the
    LDS-resident kernels (<= 32^2) and in the CG passes (64^2, 128^2), stops
    once four steps in a row fail to bring the residual ratio 10% below its
    best value, long before max_iters;
    the samples are reported as not converged and the QoIs are those of the
    direct solve."""
    dev = _dev()
    w = synth.workload("mlqmc_fp64_s100")
    L1 = 6
    ctx = m.Context(w["n0"], L1, w["s"], w["corr_len"], w["sigma2"], mu0=1, mu1=2, mu2=2,
                    rtol=1e-30, max_iters=200, precision=precision,
                    qoi_mask=m.MLMC_QOI_MEAN | m.MLMC_QOI_CENTER,
                    genvec=synth.korobov_vector(w["seed"], w["s"]),
                    shifts=synth.shift_table(w["seed"], L1, w["num_shifts"], w["s"]),
                    max_batch=32, device=0)
    P = _oracle_problem(oracle_mod, dict(w, num_levels=L1), mu0=1, rtol=1e-30, max_iters=200)
    k = L1 - 1
    B = 12
    pts = ctx.lattice(k, 0, B, 2, 3)
    q, _, info = _solve(ctx, pts, k + 1, info=True)
    print(f"\nprecision {precision}: {info}", flush=True)
    assert info["status"] == m.MLMC_E_NOCONV and info["not_converged"] == B
    assert 4 <= info["max_iters_used"] < 60
    assert info["max_rel_residual"] <= 1e-12
    z = synth.korobov_vector(w["seed"], w["s"])
    D = synth.shift_table(w["seed"], L1, w["num_shifts"], w["s"])
    _, ys = oracle_mod.points(z, D[k, 2], 0, 3)
    tol = 1e-11 if precision == m.MLMC_FP64 else 1e-8
    for b in range(3):
        qo = P.sample(k, ys[b], 1)[:, : ctx.nq]
        assert _rel(q[b], qo) <= tol, b


def test_monte_carlo_sampler_and_mlmc_driver():
    """Plain MLMC through the same driver: R replicas of i.i.d. normals stand
    in for the shifts.  The sampler's level sums equal exactly rounded sums of
    the per-sample QoIs of the same explicit points, and MLMC agrees with
    MG-MLQMC within the two error bounds."""
    from paper_1806_05619_amd.driver import GpuMcSampler, GpuSampler, mg_mlqmc
    dev = _dev()
    w, ctx = _ctx("mlqmc_fp64_s100", max_batch=4096)

    def normals(level, r, n0, n1):
        return synth.mc_normals(w["seed"], level, n1, w["s"], replica=r)[n0:n1]

    S = GpuMcSampler(ctx, normals, 3)
    k = 3
    sums = S.sample(k, 5, 42)
    for r in range(3):
        y = torch.tensor(normals(k, r, 5, 42), device=dev)
        q, _, _ = _solve(ctx, ctx.explicit(k, y), k + 1)
        for qi in range(ctx.nq):
            d = np.diff(np.concatenate([np.zeros((37, 1)), q[:, :, qi]], axis=1), axis=1)
            for l in range(k + 1):
                assert abs(sums[r, qi, l, 0] - math.fsum(d[:, l])) <= 1e-13 * math.fsum(np.abs(d[:, l]))
                assert abs(sums[r, qi, l, 1] - math.fsum(d[:, l] ** 2)) <= 1e-13 * math.fsum(d[:, l] ** 2)
    eps = 2e-3
    a = mg_mlqmc(GpuMcSampler(ctx, normals, 16), eps, max_level=w["num_levels"] - 1, reuse=False)
    b = mg_mlqmc(GpuSampler(ctx), eps, max_level=w["num_levels"] - 1, reuse=True)
    print(f"\nMLMC {a['q_bar']:.6f} (L {a['L']}, N {a['N'].tolist()}), "
          f"MG-MLQMC {b['q_bar']:.6f} (L {b['L']}, N {b['N'].tolist()})")
    assert a["converged"] and b["converged"]
    assert abs(a["q_bar"] - b["q_bar"]) <= 3 * eps


def test_uneven_workload_finest_level_sampled(oracle_mod):
    """The finest level of the uneven workload at its own launch
    configuration: 8 lattice points x 16 shifts at 2048^2 in one mixed-path
    call (s = 400, refinement to 1e-10 with the rounding-floor stop).  Two
    samples against the oracle's FMG in FP64 with the same stopping rule."""
    dev = _dev()
    w = synth.workload("uneven_mixed_s400")
    L1, R = w["num_levels"], w["num_shifts"]
    ctx = m.Context(w["n0"], L1, w["s"], w["corr_len"], w["sigma2"], mu0=w["mu0"], mu1=w["mu1"],
                    mu2=w["mu2"], rtol=w["rtol"], max_iters=w["max_iters"],
                    precision=m.MLMC_MIXED, qoi_mask=m.MLMC_QOI_MEAN | m.MLMC_QOI_CENTER,
                    genvec=synth.korobov_vector(w["seed"], w["s"]),
                    shifts=synth.shift_table(w["seed"], L1, R, w["s"]), max_batch=128, device=0)
    k = L1 - 1
    print(f"\nuneven finest level {w['n0'] << k}^2, 128 samples", flush=True)
    q, _, info = _solve(ctx, ctx.lattice(k, 0, 8, 0, R), k + 1, info=True)
    assert np.all(np.isfinite(q))
    assert info["max_rel_residual"] <= 1e-9, info
    P = _oracle_problem(oracle_mod, w)
    _, ys = _lattice_y(oracle_mod, w, k, [0], 0, 2)
    qo, _ = P.batch(k, ys, 0, nthreads=2)
    for b in range(2):
        assert _rel(q[b], qo[b][:, : ctx.nq]) <= 1e-8, b


@pytest.mark.parametrize("precision", [m.MLMC_FP64, m.MLMC_MIXED])
def test_mixed_workload_finest_level_sampled(oracle_mod, precision):
    """The s = 400 workload's finest level (1024^2) at the launch configuration
    of the mixed-vs-FP64 measurement: 64 lattice points of shift 0 in one
    call.  Two samples against the oracle's FP64 FMG with the same stopping
    rule, both precisions."""
    dev = _dev()
    w = synth.workload("mlqmc_mixed_s400")
    L1, R = w["num_levels"], w["num_shifts"]
    ctx = m.Context(w["n0"], L1, w["s"], w["corr_len"], w["sigma2"], mu0=w["mu0"], mu1=w["mu1"],
                    mu2=w["mu2"], rtol=w["rtol"], max_iters=w["max_iters"], precision=precision,
                    qoi_mask=m.MLMC_QOI_MEAN | m.MLMC_QOI_CENTER,
                    genvec=synth.korobov_vector(w["seed"], w["s"]),
                    shifts=synth.shift_table(w["seed"], L1, R, w["s"]), max_batch=64, device=0)
    k = L1 - 1
    print(f"\nmixed workload finest level {w['n0'] << k}^2, 64 samples, precision {precision}",
          flush=True)
    q, _, info = _solve(ctx, ctx.lattice(k, 0, 64, 0, 1), k + 1, info=True)
    assert np.all(np.isfinite(q)) and info["max_rel_residual"] <= 1e-9, info
    P = _oracle_problem(oracle_mod, w)
    _, ys = _lattice_y(oracle_mod, w, k, [0], 0, 2)
    qo, _ = P.batch(k, ys, 0, nthreads=2)
    for b in range(2):
        assert _rel(q[b], qo[b][:, : ctx.nq]) <= 1e-8, b
