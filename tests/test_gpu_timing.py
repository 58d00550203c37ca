"""Per-kernel event timing (pfc_opts.timing, pfc_kernel_time): the bitmask selects which
launches are timed, single-kernel launches carry their own start/stop events, and timing
never changes a result (bitwise)."""
import numpy as np
import pytest

import pfc_inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pfc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1703_01202_amd as m
    return m


CASES = {   # ILU(0) on the 64^2 noise workload, FP32 LU boxes on a 128^2 crystal grid (adaptive dt)
    "ilu0": (I.small_noise_64(), dict(sub_solver="ilu0")),
    "lu": (I.crystal_growth(128, (2, 8), nsteps=4), dict(sub_solver="lu", dt_max=10.0, eta=5000.0)),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_timing_mask_counts_and_leaves_results_unchanged(pfc, case):
    w, extra = CASES[case]
    kw = dict(precond_fp32=True, dt_min=w.dt_min, dt_max=w.dt_max, newton_rtol=w.newton_rtol,
              newton_atol=w.newton_atol)
    kw.update(extra)
    phi0 = torch.from_numpy(w.initial()).cuda()
    runs = {}
    for name, timing in [("off", 0), ("apply", 1), ("all", True)]:
        s = pfc.Solver(w.shape, w.lengths, w.gamma, w.sub, w.overlap, timing=timing, **kw)
        phi = phi0.clone()
        stats = [s.step(phi) for _ in range(4)]
        runs[name] = (phi.cpu().numpy(), [s.kernel_time(k) for k in range(4)], stats)
        s.close()
    ref = runs["off"][0]
    for name in ("apply", "all"):
        assert np.array_equal(runs[name][0], ref), name
    off, apply_only, every = runs["off"][1], runs["apply"][1], runs["all"][1]
    assert all(c == 0 and ms == 0.0 for c, ms in off)
    gmres = sum(st["gmres_its"] for st in runs["apply"][2])
    assert apply_only[0][0] >= gmres > 0 and apply_only[0][1] > 0.0   # one apply per Arnoldi step at least
    assert apply_only[1] == (0, 0.0) and apply_only[2] == (0, 0.0) and apply_only[3] == (0, 0.0)
    assert every[0][0] == apply_only[0][0]
    for k in range(4):
        assert every[k][0] > 0 and every[k][1] > 0.0, k
