"""HIP-graph replay of the Arnoldi steps (pfc_opts.use_graph): every time step is checked
against the same solver launching its kernels one by one.  The graphs are replayed many
times per step (every Newton iteration) between eager work and synchronisations, and they
are recaptured whenever dt changes (the adaptive case)."""
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


CASES = {
    "ilu_fixed_dt": (I.small_noise_64(), dict(), 8),
    "ilu_adaptive_dt": (I.small_noise_64(), dict(dt_max=10.0, eta=50.0), 8),
    "lu_fp32_lagged": (I.crystal_growth(128, (2, 8)), dict(sub_solver="lu", precond_fp32=True, precond_lag=5,
                                                           guess="extrap", eta=5000.0, dt_max=10.0), 6),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_graph_replay_matches_eager_launches(pfc, case):
    w, extra, nsteps = CASES[case]
    stream = torch.cuda.Stream()                       # graphs need a non-default stream
    with torch.cuda.stream(stream):
        kw = dict(dt_min=w.dt_min, dt_max=w.dt_max, newton_rtol=w.newton_rtol, newton_atol=w.newton_atol)
        kw.update(extra)
        eager = pfc.Solver(w.shape, w.lengths, w.gamma, w.sub, w.overlap, stream=stream.cuda_stream, **kw)
        graph = pfc.Solver(w.shape, w.lengths, w.gamma, w.sub, w.overlap, stream=stream.cuda_stream,
                           use_graph=True, **kw)
        phi_e = torch.from_numpy(w.initial()).cuda()
        phi_g = phi_e.clone()
        dts = set()
        for n in range(nsteps):
            se = eager.step(phi_e)
            sg = graph.step(phi_g)
            assert torch.equal(phi_e, phi_g), (case, n)
            assert (se["newton_its"], se["gmres_its"], se["dt"]) == (sg["newton_its"], sg["gmres_its"], sg["dt"])
            dts.add(se["dt"])
        if case == "ilu_adaptive_dt":
            assert len(dts) > 2                          # the graphs were recaptured
        assert graph.kernel_time(4)[0] > 0                 # the graph path did run
        assert eager.kernel_time(4)[0] == 0
        eager.close()
        graph.close()
    stream.synchronize()


def test_graph_option_needs_a_stream(pfc):
    w = I.small_noise_64()
    with pytest.raises(pfc.PfcError):
        pfc.Solver(w.shape, w.lengths, w.gamma, w.sub, w.overlap, stream=0, use_graph=True)
