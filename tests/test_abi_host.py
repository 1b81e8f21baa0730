"""CPU tests of the C ABI: the library loads and exports every declared
symbol, arguments are validated before any GPU work, and the host-side parts
(KL mode table, FMG schedule, estimator) agree with the oracle.  No compute
runs on a GPU here."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import synth
import paper_1806_05619_amd as m

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "mlmc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mlmc_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = m.lib()
    declared = _declared_symbols()
    assert len(declared) >= 12
    for name in declared:
        assert hasattr(L, name), name
    assert set(declared) == set(m.EXPORTS)


def test_status_strings():
    L = m.lib()
    assert L.mlmc_status_str(0) == b"ok"
    assert L.mlmc_status_str(-1) == b"invalid argument"
    assert L.mlmc_status_str(-4) == b"not converged"


def _cfg(**kw):
    base = dict(n0=4, num_levels=3, s=10, corr_len=0.3, sigma2=1.0, mu0=2, mu1=2, mu2=2,
                rtol=0.0, max_iters=0, precision=0, qoi_mask=1, num_shifts=0, genvec=None,
                shifts=None, max_batch=16)
    base.update(kw)
    return m.mlmc_config(**base)


@pytest.mark.parametrize("bad", [
    dict(n0=3), dict(n0=1), dict(num_levels=0), dict(n0=4, num_levels=12), dict(s=0),
    dict(corr_len=0.0), dict(sigma2=-1.0), dict(mu1=0, mu2=0), dict(mu0=0),
    dict(rtol=1e-8, max_iters=0), dict(rtol=1e-8, max_iters=5, mu1=3),
    dict(rtol=1e-8, max_iters=5, mu2=0), dict(precision=1), dict(precision=7),
    dict(qoi_mask=0), dict(qoi_mask=4), dict(max_batch=0),
    dict(field_kind=2), dict(field_kind=1, nu=0.0), dict(field_kind=1, nu=9.0),
    dict(field_kind=1, nu=1.0, nystrom_q=3), dict(field_kind=1, nu=1.0, nystrom_q=97),
    dict(field_kind=1, nu=1.0, nystrom_q=4, s=17),
])
def test_create_rejects_invalid_config(bad):
    L = m.lib()
    h = C.c_void_p()
    cfg = _cfg(**bad)
    assert L.mlmc_create(C.byref(cfg), 0, C.byref(h)) == m.MLMC_E_INVAL
    assert not h.value
    assert len(L.mlmc_last_error(None)) > 0


def _host_ctx(**kw):
    cfg = dict(n0=4, num_levels=3, s=10, corr_len=0.3, sigma2=1.0)
    cfg.update(kw)
    return m.Context(**cfg, device=-1)


def test_matern_field_needs_a_device():
    # the Nystrom eigensolve runs on the GPU: no host-only Matern context
    with pytest.raises(m.MlmcError):
        _host_ctx(field_kind=m.MLMC_FIELD_MATERN, nu=1.0)


def test_host_only_context_refuses_gpu_calls():
    ctx = _host_ctx()
    pts = m.Context.lattice(0, 0, 4)
    with pytest.raises(m.MlmcError):
        ctx.fmg_solve(pts)
    with pytest.raises(m.MlmcError):
        ctx.field(pts, None)


def test_field_size_and_levels():
    ctx = _host_ctx(n0=16, num_levels=3)
    # multigrid levels 2^2 .. 16^2 below MLMC level 0
    assert ctx.field_size(0) == 4 + 16 + 64 + 256
    assert ctx.field_size(2) == 4 + 16 + 64 + 256 + 1024 + 4096
    assert ctx.field_size(3) == 0
    assert ctx.nq == 1
    assert _host_ctx(qoi_mask=3).nq == 2


@pytest.mark.parametrize("lam,s", [(0.3, 10), (0.3, 100), (0.1, 400), (0.05, 1000)])
def test_mode_table_bit_exact_with_oracle(oracle_mod, lam, s):
    ctx = _host_ctx(s=s, corr_len=lam)
    i, j, t = ctx.kl_modes()
    oi, oj, ot = oracle_mod.kl_modes(lam, s)
    assert np.array_equal(i, oi) and np.array_equal(j, oj)
    assert np.allclose(t, ot, rtol=1e-14, atol=0)


def test_fmg_trace_matches_figure_and_oracle(oracle_mod):
    golden = open(os.path.join(ROOT, "tests", "golden", "fmg_trace_mu0_1_level3.txt")).read().split()
    want = [int(v) for v in golden[0].split(",")]
    circled = [int(v) for v in golden[1].split(",")]
    ctx = _host_ctx(n0=2, num_levels=4, mu0=1)
    lv, mk = ctx.fmg_trace(3)
    assert lv == want
    assert [i + 1 for i, v in enumerate(mk) if v] == circled
    # other cycle counts and hierarchies: identical to the oracle's recursion
    for n0, L, mu0, k in [(4, 5, 2, 4), (16, 3, 2, 2), (2, 3, 3, 2)]:
        ctx = _host_ctx(n0=n0, num_levels=L, mu0=mu0)
        lv, mk = ctx.fmg_trace(k)
        P = oracle_mod.Problem(n0, L, 4, 0.3, 1.0, mu0=mu0)
        G = P.finest_mg_level(k)
        r = P.fmg(G, np.ones(P.field_size(k)), trace_cap=10000)
        assert lv == r["trace"] and mk == r["marks"]


def _F_from_sums(F, nq_index=0):
    """mlmc_estimate's input sums [k][r][q][l][2] built from per-sample F."""
    L1 = len(F)
    R = F[0].shape[0]
    sums = np.zeros((L1, R, 1, L1, 2))
    for k in range(L1):
        for r in range(R):
            for l in range(k + 1):
                d = F[k][r, :, l] - (F[k][r, :, l - 1] if l else 0.0)
                sums[k, r, 0, l, 0] = np.sum(d)
                sums[k, r, 0, l, 1] = np.sum(d * d)
    return sums


@pytest.mark.parametrize("R,reuse", [(5, True), (5, False), (1, False), (1, True)])
def test_estimate_matches_oracle(R, reuse):
    from oracle import estimators as est
    rng = np.random.default_rng(R + 10 * reuse)
    N = [40, 17, 6, 3]
    F = []
    for k in range(4):
        base = rng.standard_normal((R, N[k], 1)) + 3.0
        F.append(base + 0.2 * np.cumsum(rng.standard_normal((R, N[k], k + 1)), axis=2))
    want = est.mlmc_estimate(F, reuse)
    got = m.mlmc_estimate(np.array(N), _F_from_sums(F), R, 1, reuse)
    tol = dict(rtol=1e-12, atol=1e-14)
    assert np.allclose(got["upsilon"][0], want["upsilon"], **tol)
    assert np.allclose(got["q_shift"][0], want["q_shift"], **tol)
    assert np.allclose(got["q_bar"][0], want["q_bar"], **tol)
    assert np.allclose(got["upsilon_bar"][0], want["upsilon_bar"], **tol)
    if R == 1 and reuse:
        assert np.isnan(got["var_q"][0]) and np.all(np.isnan(got["var_level"][0]))
    else:
        assert np.allclose(got["var_level"][0], want["var_level"], rtol=1e-10, atol=1e-16)
        assert np.allclose(got["var_q"][0], want["var_q"], rtol=1e-10, atol=1e-16)


def test_estimate_rejects_bad_input():
    with pytest.raises(m.MlmcError):
        m.mlmc_estimate(np.array([-1, 2]), np.zeros((2, 2, 1, 2, 2)), 2, 1, True)


def _server_cfg(**kw):
    w = synth.workload("mlqmc_fp64_s100")
    z = synth.korobov_vector(w["seed"], w["s"])
    D = synth.shift_table(w["seed"], w["num_levels"], w["num_shifts"], w["s"])
    base = dict(n0=w["n0"], num_levels=w["num_levels"], s=w["s"], corr_len=w["corr_len"],
                sigma2=w["sigma2"], mu0=2, mu1=2, mu2=2, rtol=0.0, max_iters=0, precision=0,
                qoi_mask=1, num_shifts=w["num_shifts"], genvec=z.ctypes.data,
                shifts=D.ctypes.data, max_batch=16)
    base.update(kw)
    return m.mlmc_config(**base), (z, D)


@pytest.mark.parametrize("dev,slots,samples,over", [
    (-1, 1, 16, {}), (0, 0, 16, {}), (0, 2, 0, {}), (0, 1, 16, dict(genvec=None)),
    (0, 1, 16, dict(shifts=None)), (0, 1, 16, dict(n0=3)), (0, 1, 16, dict(mu1=0, mu2=0)),
])
def test_server_create_rejects_invalid_arguments(dev, slots, samples, over):
    """Argument errors are reported before any device work (no GPU here)."""
    L = m.lib()
    cfg, keep = _server_cfg(**over)
    h = C.c_void_p(123)
    assert L.mlmc_server_create(C.byref(cfg), dev, slots, samples, C.byref(h)) == m.MLMC_E_INVAL
    assert not h.value
    assert L.mlmc_server_create(C.byref(cfg), 0, 1, 16, None) == m.MLMC_E_INVAL


def test_server_calls_reject_null_handles():
    L = m.lib()
    req = m.mlmc_request(0, 0, 1, 0, 1, 0, None)
    res = (m.mlmc_result * 4)()
    n = C.c_int32(-1)
    st = m.mlmc_server_stats()
    assert L.mlmc_server_destroy(None) == m.MLMC_OK
    assert L.mlmc_server_submit(None, C.byref(req)) == m.MLMC_E_INVAL
    assert L.mlmc_server_poll(None, res, 4, 0, C.byref(n)) == m.MLMC_E_INVAL
    assert L.mlmc_server_stats_get(None, C.byref(st)) == m.MLMC_E_INVAL


def _default_kind(n, c, fp64):
    """The documented default of grid side n and batch class c."""
    tiles = 4 ** c * max(1, n // 32) ** 2
    lanes = 4 ** c * (n // 2)
    smallest = 1 if c == 0 else 4 ** (c - 1) + 1               # smallest chunk of the class
    spb = 1 if n >= 128 else 64 // (n // 2)
    tile = m.MLMC_PASS_TILE16 if tiles <= 256 else m.MLMC_PASS_TILE32
    has_stream = 32 <= n <= (1024 if fp64 else 2048)
    big = ((tiles >= 65536 or (fp64 and n <= 64 and tiles >= 16384)) and lanes >= 131072
           and smallest // spb >= 256)
    return m.MLMC_PASS_STREAM if has_stream and big else tile


def test_tuning_table_defaults_and_validation():
    """Pass-kind table of a context (host-only: no measurement): one entry per
    tile grid and batch class with the documented defaults; mlmc_tuning_set
    checks every entry before changing any."""
    # refinement contexts: tile grids 64^2 .. 2048^2, FP64 and FP32 V-cycles
    for prec in (m.MLMC_FP64, m.MLMC_MIXED):
        c2 = _host_ctx(n0=4, num_levels=10, rtol=1e-10, max_iters=60, precision=prec)
        t2 = c2.tuning()
        assert sorted({e["n"] for e in t2}) == [64, 128, 256, 512, 1024, 2048]
        for e in t2:
            k = _default_kind(e["n"], e["batch_class"], prec == m.MLMC_FP64)
            assert (e["pre"], e["post"]) == (k, k), (prec, e)
        kinds = {(e["n"], e["batch_class"]): e["pre"] for e in t2}
        assert kinds[(1024, 5)] == m.MLMC_PASS_STREAM              # 257 .. 1024 samples of 1024^2
        assert kinds[(1024, 4)] == m.MLMC_PASS_TILE32              # from 65: fewer workgroups than CUs
        assert kinds[(512, 4)] == m.MLMC_PASS_TILE32               # 256 samples: 65536 lanes
        assert kinds[(2048, 4)] == m.MLMC_PASS_TILE32              # 128 samples of 2048^2
        assert kinds[(2048, 5)] == (m.MLMC_PASS_TILE32 if prec == m.MLMC_FP64
                                    else m.MLMC_PASS_STREAM)
    ctx = _host_ctx(n0=4, num_levels=7)             # tile grids 32^2 .. 256^2
    t = ctx.tuning()
    assert [(e["n"], e["batch_class"]) for e in t] == [
        (n, c) for n in (32, 64, 128, 256) for c in range(m.MLMC_BATCH_CLASSES)]
    for e in t:
        k = _default_kind(e["n"], e["batch_class"], True)
        assert e["pre"] == k and e["pre_ms"] == 0.0, e
        assert e["post"] == k, e
    kinds = {(e["n"], e["batch_class"]): (e["pre"], e["post"]) for e in t}
    assert kinds[(256, 1)] == (m.MLMC_PASS_TILE16,) * 2            # 4 samples: 256 tiles
    assert kinds[(256, 7)] == (m.MLMC_PASS_STREAM,) * 2            # 16384 samples
    assert kinds[(32, 7)] == (m.MLMC_PASS_STREAM,) * 2             # 16384 samples of 32^2
    assert kinds[(32, 6)] == (m.MLMC_PASS_TILE32,) * 2
    assert kinds[(64, 6)] == (m.MLMC_PASS_STREAM,) * 2             # 4096 samples of 64^2
    with pytest.raises(m.MlmcError):
        ctx.autotune()                              # host-only: no device to measure on
    L = m.lib()
    assert L.mlmc_autotune(None, 0, None) == m.MLMC_E_INVAL
    cnt = C.c_int32(-1)
    assert L.mlmc_tuning_get(None, None, 0, C.byref(cnt)) == m.MLMC_E_INVAL
    T16, ST, T32 = m.MLMC_PASS_TILE16, m.MLMC_PASS_STREAM, m.MLMC_PASS_TILE32
    for bad in [dict(n=16, batch_class=0, pre=T32, post=T32),      # LDS-resident grid
                dict(n=48, batch_class=0, pre=T32, post=T32),
                dict(n=512, batch_class=0, pre=T32, post=T32),     # beyond the finest level
                dict(n=64, batch_class=10, pre=T32, post=T32),
                dict(n=64, batch_class=-1, pre=T32, post=T32),
                dict(n=64, batch_class=0, pre=T32, post=3)]:
        with pytest.raises(m.MlmcError):
            ctx.set_tuning([dict(n=128, batch_class=2, pre=T16, post=T16), bad])
        assert ctx.tuning() == t                    # nothing changed
    ctx.set_tuning([dict(n=128, batch_class=2, pre=T16, post=ST), dict(n=32, batch_class=9, pre=T16, post=T16)])
    t2 = {(e["n"], e["batch_class"]): (e["pre"], e["post"]) for e in ctx.tuning()}
    assert t2[(128, 2)] == (T16, ST) and t2[(32, 9)] == (T16, T16)
    assert sum(t2[k] != (e["pre"], e["post"]) for e in t for k in [(e["n"], e["batch_class"])]) == 2
    # mixed precision: the FP32 V-cycles' defaults and an installed choice;
    # rtol mode keeps 32^2 LDS-resident
    mx = _host_ctx(n0=4, num_levels=7, precision=1, rtol=1e-10, max_iters=50)
    tm = mx.tuning()
    assert [e["n"] for e in tm[::m.MLMC_BATCH_CLASSES]] == [64, 128, 256]
    assert all(e["pre"] == e["post"] == _default_kind(e["n"], e["batch_class"], False) for e in tm)
    mx.set_tuning([dict(n=256, batch_class=7, pre=T32, post=ST)])
    assert {(e["n"], e["batch_class"]): (e["pre"], e["post"]) for e in mx.tuning()}[(256, 7)] == (T32, ST)
    with pytest.raises(m.MlmcError):                 # no streaming pass above 2048^2
        _host_ctx(n0=4, num_levels=11).set_tuning([dict(n=4096, batch_class=0, pre=ST, post=T32)])
    with pytest.raises(m.MlmcError):                 # rtol mode: 32^2 is LDS-resident
        mx.set_tuning([dict(n=32, batch_class=0, pre=T32, post=T32)])
    assert _host_ctx(n0=4, num_levels=3).tuning() == []          # all grids LDS-resident


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
