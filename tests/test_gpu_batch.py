"""Batched ragged instances (include/pfc_batch.h): stepping many independent grids of uneven
size from several host threads gives, instance by instance, exactly what stepping each one
alone gives (same kernels, same reduction orders, only other streams)."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pfc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1703_01202_amd as m
    return m


def _instances():
    from pfc_inputs import noise_ic
    out = []
    for i, (n, gamma, mean) in enumerate([(64, 0.25, -0.30), (96, 0.15, -0.25), (128, 0.35, -0.28),
                                          (64, 0.30, -0.32), (160, 0.20, -0.22)]):
        L = n * math.pi / 2
        inst = dict(shape=(n, n), lengths=(L, L), gamma=gamma, sub=(n // 32, n // 32), overlap=2,
                    dt_min=1e-2, dt_max=10.0, eta=5000.0, precond_fp32=True, guess="extrap")
        out.append((inst, noise_ic((n, n), mean, 0.05, 3000 + i)))
    return out


def test_batch_matches_instances_stepped_alone(pfc):
    insts = _instances()
    batch = pfc.Batch([i for i, _ in insts], workers=3)
    phis = [torch.from_numpy(p0).cuda() for _, p0 in insts]
    batch_stats = [batch.step(phis) for _ in range(4)]
    for k, (inst, p0) in enumerate(insts):
        kw = dict(inst)
        shape, lengths, gamma, sub, ov = (kw.pop(x) for x in ("shape", "lengths", "gamma", "sub", "overlap"))
        s = pfc.Solver(shape, lengths, gamma, sub, ov, **kw)
        phi = torch.from_numpy(p0).cuda()
        for step in range(4):
            st = s.step(phi)
            assert st["newton_its"] == batch_stats[step][k]["newton_its"]
            assert st["dt"] == batch_stats[step][k]["dt"]
        assert torch.equal(phi, phis[k]), k
        s.close()
    batch.close()


def test_batch_rejects_a_bad_instance_and_bad_fields(pfc):
    insts = _instances()
    bad = dict(insts[0][0])
    bad["sub"] = (3, 3)                                # 3 does not divide 64
    with pytest.raises(pfc.PfcError):
        pfc.Batch([insts[1][0], bad], workers=2)
    batch = pfc.Batch([insts[0][0]], workers=1)
    with pytest.raises(ValueError):
        batch.step([torch.zeros((8, 8), dtype=torch.float64, device="cuda")])
    batch.close()


def test_autotune_times_candidates_and_skips_rejected_ones():
    """The autotuner runs every candidate on the library, reports the ones the library rejects
    (an overlap wider than the grid allows) with their error, leaves phi0 untouched, and returns
    the fastest of the candidates that ran."""
    from paper_1703_01202_amd.autotune import autotune
    import pfc_inputs as I

    w = I.small_noise_64()
    phi0 = torch.from_numpy(w.initial()).cuda()
    keep = phi0.clone()
    kw = dict(sub_solver="ilu0", precond_fp32=False, dt_min=w.dt_min, dt_max=w.dt_max, guess="previous")
    cands = [((4, 4), 2, 0), ((4, 4), 40, 0), ((2, 2), 2, 5)]
    best, table = autotune(w.shape, w.lengths, w.gamma, phi0, kw, cands, steps=3, warmup=1)
    assert torch.equal(phi0, keep)
    assert len(table) == 3 and "error" in table[1] and "steps_per_s" not in table[1]
    ran = [r for r in table if "steps_per_s" in r]
    assert len(ran) == 2 and best is max(ran, key=lambda r: r["steps_per_s"])
    assert all(r["newton_its"] > 0 for r in ran)
    assert np.isfinite(best["steps_per_s"])


def test_benchmark_batch_instances_reach_the_oracle_root(pfc):
    """The benchmark's 64-instance batch configuration (FP32 exact LU on boxes of 64 x 16 owned
    cells with overlap 4, extrapolated guess, lagged factors), run as a ragged batch of sampled
    instances: every 128^2 instance and the first 192^2 one of the set, with the first 256^2
    one beside them unchecked.  One step from the initial states, Newton to 1e-10; each
    checked instance's solution is the oracle's Newton root (direct solves) for the same
    state and step to rel 1e-9."""
    import pfc_inputs as I
    from oracle import scheme as S
    ws = I.batch_instances(64)
    small = [w for w in ws if w.shape == (128, 128)]
    pick = small + [next(w for w in ws if w.shape == (192, 192)), next(w for w in ws if w.shape == (256, 256))]
    insts = [dict(shape=w.shape, lengths=w.lengths, gamma=w.gamma, sub=(w.shape[0] // 64, w.shape[1] // 16),
                  overlap=4, dt_min=w.dt_min, dt_max=w.dt_max, eta=w.eta, newton_rtol=0.0, newton_atol=1e-10,
                  lin_rtol=w.lin_rtol, lin_atol=w.lin_atol, sub_solver="lu", precond_fp32=True, guess="extrap",
                  precond_lag=20) for w in pick]
    batch = pfc.Batch(insts, workers=4)
    phi0 = [w.initial() for w in pick]
    phis = [torch.from_numpy(p).cuda() for p in phi0]
    st = batch.step(phis)
    for k, w in enumerate(pick[:-1]):
        h = S.spacing(w.shape, w.lengths)
        ref = S.newton_solve(phi0[k], st[k]["dt"], w.gamma, h)
        assert ref.converged
        got = phis[k].cpu().numpy()
        assert S.rel_l2(got, ref.Phi) <= 1e-9, (k, w.shape, S.rel_l2(got, ref.Phi))
    batch.close()
