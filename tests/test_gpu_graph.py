"""A fixed-cycle solve (rtol = 0, no info requested) makes no host
synchronisation and allocates nothing, so a caller can capture it into a HIP
graph on its stream and replay it.  Through the C ABI (the binding passes
torch's current stream), a captured solve of 256 lattice samples at 64^2
(points, KL field, FMG with two V(2,2) cycles per stage, the QoI table and the
per-shift level-difference sums) is replayed three times, with eager solves of
other samples on the same context between the replays (they overwrite the
shared workspace) and the outputs reset in between; every replay must give
bitwise the QoIs and sums of the eager solve, for the default pass kinds and
with row streaming forced on every tile grid."""
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


@pytest.mark.parametrize("kinds", ["default", "stream"])
def test_fixed_cycle_solve_replays_from_a_captured_graph(kinds):
    dev = _dev()
    w = synth.workload("mlqmc_fp64_s100")
    L, level = 5, 4                       # MLMC levels 4^2 .. 64^2
    ctx = m.Context(w["n0"], L, w["s"], w["corr_len"], w["sigma2"], mu0=w["mu0"], mu1=w["mu1"],
                    mu2=w["mu2"], rtol=0.0, precision=m.MLMC_FP64,
                    qoi_mask=m.MLMC_QOI_MEAN | m.MLMC_QOI_CENTER,
                    genvec=synth.korobov_vector(w["seed"], w["s"]),
                    shifts=synth.shift_table(w["seed"], L, w["num_shifts"], w["s"]),
                    max_batch=256, device=0)
    try:
        if kinds == "stream":
            ctx.set_tuning(dict(e, pre=m.MLMC_PASS_STREAM, post=m.MLMC_PASS_STREAM)
                           for e in ctx.tuning())
        nq, R = 2, 4
        pts = ctx.lattice(level, 0, 64, 0, R)            # 256 samples
        other = ctx.lattice(level, 64, 128, 0, R)        # the eager work between replays
        B = ctx.count(pts)
        nan = float("nan")
        q_ref = torch.full((B, level + 1, nq), nan, dtype=torch.float64, device=dev)
        s_ref = torch.full((R, nq, level + 1, 2), nan, dtype=torch.float64, device=dev)
        print(f"kinds {kinds}: eager solve of {B} samples at level {level}", flush=True)
        ctx.fmg_solve(pts, qoi=q_ref, sums=s_ref)
        torch.cuda.synchronize()
        q_ref, s_ref = q_ref.cpu().numpy(), s_ref.cpu().numpy()
        assert np.all(np.isfinite(q_ref)) and np.all(np.isfinite(s_ref))

        q_g = torch.full((B, level + 1, nq), nan, dtype=torch.float64, device=dev)
        s_g = torch.full((R, nq, level + 1, 2), nan, dtype=torch.float64, device=dev)
        q_o = torch.empty((ctx.count(other), level + 1, nq), dtype=torch.float64, device=dev)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            ctx.fmg_solve(pts, qoi=q_g, sums=s_g)         # warm-up off the capture
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        print(f"kinds {kinds}: capture", flush=True)
        with torch.cuda.graph(g):
            ctx.fmg_solve(pts, qoi=q_g, sums=s_g)
        torch.cuda.synchronize()
        for rep in range(3):
            q_g.fill_(nan)
            s_g.fill_(nan)
            ctx.fmg_solve(other, qoi=q_o)
            torch.cuda.synchronize()
            print(f"kinds {kinds}: replay {rep}", flush=True)
            g.replay()
            torch.cuda.synchronize()
            assert np.array_equal(q_g.cpu().numpy(), q_ref), rep
            assert np.array_equal(s_g.cpu().numpy(), s_ref), rep
        del g
    finally:
        ctx.close()
