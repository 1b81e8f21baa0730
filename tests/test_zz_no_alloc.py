"""mlmc_field_static, the field entry point that allocates nothing (its
staging lives in the library's static device scratch): through the C ABI it
returns bitwise the z of mlmc_field on the same context, FP64 and mixed, for
lattice and explicit points, on two calls in a row (the second smaller, so
stale scratch contents would show), and it refuses a set that does not fit
its scratch."""
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


def _ctx(precision):
    w = synth.workload("mlqmc_mixed_s400")
    L = 5
    return w, m.Context(w["n0"], L, w["s"], w["corr_len"], w["sigma2"], mu0=w["mu0"], mu1=w["mu1"],
                        mu2=w["mu2"], rtol=w["rtol"], max_iters=w["max_iters"],
                        precision=precision, qoi_mask=m.MLMC_QOI_MEAN | m.MLMC_QOI_CENTER,
                        genvec=synth.korobov_vector(w["seed"], w["s"]),
                        shifts=synth.shift_table(w["seed"], L, w["num_shifts"], w["s"]),
                        max_batch=64, device=0)


def _both(ctx, pts, level):
    dev = torch.device("cuda:0")
    B = ctx.count(pts)
    M = ctx.field_size(level)
    z1 = torch.full((B, M), float("nan"), dtype=torch.float64, device=dev)
    z2 = torch.full((B, M), float("nan"), dtype=torch.float64, device=dev)
    ctx.field(pts, z1)
    ctx.field_static(pts, z2)
    torch.cuda.synchronize()
    return z1.cpu().numpy(), z2.cpu().numpy()


@pytest.mark.parametrize("precision", [m.MLMC_FP64, m.MLMC_MIXED])
def test_field_static_equals_field(precision):
    dev = _dev()
    w, ctx = _ctx(precision)
    # lattice points: 120 samples at 64^2, then 7 at 16^2
    for level, n0, n1, r0, r1 in [(4, 0, 40, 0, 3), (2, 5, 12, 1, 2)]:
        print(f"precision {precision}: lattice level {level} points {n0}..{n1} shifts {r0}..{r1}",
              flush=True)
        z1, z2 = _both(ctx, ctx.lattice(level, n0, n1, r0, r1), level)
        assert np.all(np.isfinite(z1))
        assert np.array_equal(z1, z2), (level, n0, n1)
    # explicit points: 90 then 3 samples
    rng = np.random.default_rng(17)
    for level, B in [(3, 90), (1, 3)]:
        y = torch.tensor(rng.standard_normal((B, w["s"])), device=dev)
        z1, z2 = _both(ctx, ctx.explicit(level, y), level)
        assert np.all(np.isfinite(z1))
        assert np.array_equal(z1, z2), (level, B)


def test_field_static_refuses_oversized_sets():
    dev = _dev()
    w, ctx = _ctx(m.MLMC_MIXED)
    B = 11000                     # 8 s B bytes of lattice staging alone exceed 32 MiB
    z = torch.zeros((1, ctx.field_size(0)), dtype=torch.float64, device=dev)
    with pytest.raises(m.MlmcError) as e:
        ctx.field_static(ctx.lattice(0, 0, B, 0, 1), z)
    assert e.value.status == m.MLMC_E_INVAL and "scratch" in str(e.value)
    # the context is still usable
    z1, z2 = _both(ctx, ctx.lattice(1, 0, 4, 0, 1), 1)
    assert np.array_equal(z1, z2)
