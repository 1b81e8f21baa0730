"""GPU tests of the large-grid pass kinds and their autotuner: every kind
(32x32 tiles, 16x16 tiles, row streaming) of the pre and post passes gives
bitwise the QoIs of the default choice, for both V-cycle precisions, and a
measured table installs only kinds that keep those bits."""
import itertools

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1806_05619_amd as m  # noqa: E402

T32, T16, ST = m.MLMC_PASS_TILE32, m.MLMC_PASS_TILE16, m.MLMC_PASS_STREAM


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _ctx(name, precision, max_batch):
    w = synth.workload(name)
    return w, m.Context(n0=w["n0"], num_levels=w["num_levels"], s=w["s"], corr_len=w["corr_len"],
                        sigma2=w["sigma2"], mu0=w["mu0"], mu1=w["mu1"], mu2=w["mu2"],
                        rtol=w["rtol"], max_iters=w["max_iters"], precision=precision,
                        qoi_mask=m.MLMC_QOI_MEAN | m.MLMC_QOI_CENTER,
                        genvec=synth.korobov_vector(w["seed"], w["s"]),
                        shifts=synth.shift_table(w["seed"], w["num_levels"], w["num_shifts"], w["s"]),
                        max_batch=max_batch, device=0)


def _solve(ctx, level, n0, n1, r0, r1):
    pts = ctx.lattice(level, n0, n1, r0, r1)
    q = torch.full((ctx.count(pts), level + 1, ctx.nq), float("nan"), dtype=torch.float64,
                   device="cuda:0")
    ctx.fmg_solve(pts, qoi=q)
    torch.cuda.synchronize()
    return q.cpu().numpy()


def _force(ctx, pre, post):
    ctx.set_tuning(dict(e, pre=pre, post=post) for e in ctx.tuning())


@pytest.mark.parametrize("name,precision,level,sizes", [
    ("mlqmc_fp64_s100", m.MLMC_FP64, 6, ((0, 3, 5, 6), (7, 47, 0, 1))),     # 32^2 .. 256^2
    ("mlqmc_mixed_s400", m.MLMC_FP64, 5, ((0, 2, 1, 3), (9, 29, 4, 5))),    # rtol, FP64 V-cycles
    ("mlqmc_mixed_s400", m.MLMC_MIXED, 5, ((0, 2, 1, 3), (9, 29, 4, 5))),   # FP32 V-cycles
])
def test_every_pass_kind_gives_the_same_bits(name, precision, level, sizes):
    """Every combination of kinds on the 32^2 grid (fixed-cycle mode) and on
    the larger grids gives the QoIs of the default choice, on every level of
    the solve."""
    _dev()
    w, ctx = _ctx(name, precision, max_batch=64)
    fixed = w["rtol"] <= 0
    levels = (level, 3) if fixed else (level,)
    want = {(lv, r): _solve(ctx, lv, *r) for lv in levels for r in sizes}
    small = [T32, T16, ST] if fixed else []
    large = [T32, T16, ST]
    for k32 in small or [None]:
        for pre, post in itertools.product(large, large):
            ent = []
            for e in ctx.tuning():
                if e["n"] == 32 and fixed:
                    ent.append(dict(e, pre=k32, post=k32))
                elif ST not in (pre, post) or 32 <= e["n"] <= 512:
                    ent.append(dict(e, pre=pre, post=post))
            ctx.set_tuning(ent)
            print(f"{name} precision {precision}: 32^2 {k32} pre {pre} post {post}", flush=True)
            for (lv, r), q0 in want.items():
                assert np.array_equal(_solve(ctx, lv, *r), q0), (k32, pre, post, lv, r)


def test_autotune_installs_measured_kinds_and_keeps_results():
    _dev()
    w, ctx = _ctx("mlqmc_fp64_s100", m.MLMC_FP64, max_batch=256)
    before = [_solve(ctx, 6, 0, 5, 2, 3), _solve(ctx, 6, 3, 131, 7, 9)]
    table = ctx.autotune()
    assert [e["n"] for e in table[::m.MLMC_BATCH_CLASSES]] == [32, 64, 128, 256]
    # the workspace holds 256 samples of the 256^2 hierarchy, so a chunk
    # whose finest grid is n holds 256 M(256)/M(n) samples (M: cells of the
    # hierarchy up to n): measured classes 0..4 at 256^2, ..5 at 128^2, ..6
    # at 64^2, ..8 at 32^2 (16399 samples)
    top_class = {256: 4, 128: 5, 64: 6, 32: 8}
    for e in table:
        measured = e["batch_class"] <= top_class[e["n"]]
        assert (e["pre_ms"] > 0 and e["post_ms"] > 0) == measured, e
        assert e["pre"] in (T32, T16, ST) and e["post"] in (T32, T16, ST)
    print("tuned:", [(e["n"], e["batch_class"], e["pre"], e["post"]) for e in table
                     if e["pre_ms"] > 0], flush=True)
    after = [_solve(ctx, 6, 0, 5, 2, 3), _solve(ctx, 6, 3, 131, 7, 9)]
    for a, b in zip(before, after):
        assert np.array_equal(a, b)
    with pytest.raises(m.MlmcError):
        ctx.autotune(level=7)


@pytest.mark.parametrize("precision", [m.MLMC_FP64, m.MLMC_MIXED])
def test_autotune_refinement_contexts(precision):
    """rtol contexts: 64^2 and up are tile grids (32^2 is LDS-resident), and
    every kind is open to both V-cycle precisions (the FP32 ones stream too).
    The tuned table keeps every result bitwise."""
    _dev()
    w, ctx = _ctx("mlqmc_mixed_s400", precision, max_batch=32)
    before = _solve(ctx, 5, 0, 3, 2, 4)
    table = ctx.autotune(5)
    assert [e["n"] for e in table[::m.MLMC_BATCH_CLASSES]][:3] == [64, 128, 256]
    for e in table:
        assert e["pre"] in (T32, T16, ST) and e["post"] in (T32, T16, ST), e
        if e["n"] <= 128 and e["batch_class"] == 0:      # tuned: levels <= 5 reach 128^2
            assert e["pre_ms"] > 0 and e["post_ms"] > 0, e
        if e["n"] > 128:
            assert e["pre_ms"] == 0, e
    assert np.array_equal(_solve(ctx, 5, 0, 3, 2, 4), before)


@pytest.mark.parametrize("L", [8, 9, 10])
@pytest.mark.parametrize("name,precision", [("mlqmc_fp64_s100", m.MLMC_FP64),
                                            ("mlqmc_mixed_s400", m.MLMC_FP64),
                                            ("mlqmc_mixed_s400", m.MLMC_MIXED)])
def test_streaming_large_grids_match_tiles(oracle_mod, name, precision, L):
    """Grids up to 512^2 (L = 8), 1024^2 and 2048^2, whose streaming
    workgroups hold 4, 8 and 16 wavefronts per sample (one barrier per row
    step): streaming, tiles and a mix give the same bits, fixed-cycle and
    refinement mode, FP64 and FP32 V-cycles; up to 1024^2 one sample against
    the oracle's FMG (fixed cycles: the same algorithm, 1e-12; refinement:
    both to rtol 1e-10, 1e-8)."""
    _dev()
    w = synth.workload(name)
    ctx = m.Context(n0=w["n0"], num_levels=L, s=w["s"], corr_len=w["corr_len"], sigma2=w["sigma2"],
                    mu0=w["mu0"], mu1=w["mu1"], mu2=w["mu2"], rtol=w["rtol"],
                    max_iters=w["max_iters"], precision=precision,
                    qoi_mask=m.MLMC_QOI_MEAN | m.MLMC_QOI_CENTER,
                    genvec=synth.korobov_vector(w["seed"], w["s"]),
                    shifts=synth.shift_table(w["seed"], L, w["num_shifts"], w["s"]),
                    max_batch=8, device=0)
    base = [dict(e) for e in ctx.tuning()]
    want = None
    for pre, post in [(T32, T32), (ST, ST), (T16, ST), (ST, T32)]:
        ctx.set_tuning(dict(e, pre=pre, post=post) for e in base)
        print(f"{name} precision {precision}: pre {pre} post {post}", flush=True)
        q = _solve(ctx, L - 1, 0, 3, 1, 2)
        assert np.all(np.isfinite(q))
        if want is None:
            want = q
        assert np.array_equal(q, want), (pre, post)
    if L > 9:
        return
    P = oracle_mod.Problem(w["n0"], L, w["s"], w["corr_len"], w["sigma2"], mu0=w["mu0"],
                           mu1=w["mu1"], mu2=w["mu2"], rtol=w["rtol"], max_iters=w["max_iters"])
    D = synth.shift_table(w["seed"], L, w["num_shifts"], w["s"])
    _, y = oracle_mod.points(synth.korobov_vector(w["seed"], w["s"]), D[L - 1, 1], 0, 1)
    qo = P.sample(L - 1, y[0], 0)
    tol = 1e-12 if w["rtol"] == 0 else 1e-8
    assert np.max(np.abs(want[0] - qo) / np.abs(qo)) <= tol
