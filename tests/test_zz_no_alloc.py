"""pfc_residual_noalloc (no context, no allocation, fixed device scratch) against
pfc_residual: bitwise the same F and norm, on two calls in a row, the second on a smaller
grid (the fixed partial-sum array keeps the first call's contents and must not leak them)."""
import ctypes

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


def _noalloc(pfc, shape, L, gamma, Phi, phi, dt, F, want_norm=True, mobility=0):
    from paper_1703_01202_amd import _lib
    lib = _lib.load()
    g, m, _ = pfc._structs(lib, shape, L, gamma, (2,) * len(shape), 1)
    m.mobility = mobility
    nrm = ctypes.c_double(-1.0)
    st = lib.pfc_residual_noalloc(ctypes.byref(g), ctypes.byref(m), ctypes.c_void_p(Phi.data_ptr()),
                                  ctypes.c_void_p(phi.data_ptr()), float(dt), None, ctypes.c_void_p(F.data_ptr()),
                                  ctypes.byref(nrm) if want_norm else None,
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, nrm.value


CASES = [((1024, 1024), (400.0, 400.0), (16, 16), 4, 0.01),     # the crystal benchmark's grid
         ((200, 120), (78.125, 46.875), (2, 2), 4, 1.0)]         # smaller and ragged against the tiles


def test_noalloc_residual_matches_pfc_residual(pfc):
    for shape, L, sub, ov, dt in CASES:
        n = shape[-1]
        phi = I.hex_crystallites_ic(n=n, L=L[-1], seed=1) if shape[0] == shape[1] else \
            I.noise_ic(shape, -0.285, 0.3, 4)
        Phi = phi + 0.01 * np.random.default_rng(5).standard_normal(shape)
        P, p = torch.from_numpy(Phi).cuda(), torch.from_numpy(phi).cuda()
        s = pfc.Solver(shape, L, 0.25, sub, ov)
        ref, ref_n = s.residual(P, p, dt)
        s.close()
        F = torch.full(shape, np.nan, dtype=torch.float64, device="cuda")
        st, nrm = _noalloc(pfc, shape, L, 0.25, P, p, dt, F)
        assert st == 0
        assert torch.equal(F, ref)
        assert nrm == ref_n
        F2 = torch.empty_like(F)
        st, _ = _noalloc(pfc, shape, L, 0.25, P, p, dt, F2, want_norm=False)
        torch.cuda.synchronize()
        assert st == 0 and torch.equal(F2, ref)


def test_noalloc_residual_rejects_what_it_does_not_build(pfc):
    shape, L = (64, 64), (40.0, 40.0)
    P = torch.zeros(shape, dtype=torch.float64, device="cuda")
    F = torch.empty_like(P)
    assert _noalloc(pfc, shape, L, 0.25, P, P, 0.0, F)[0] == -1            # dt
    assert _noalloc(pfc, shape, L, 0.25, P, P, 0.1, F, mobility=1)[0] == -1
    assert _noalloc(pfc, shape, L, 0.25, P, P, 0.1, P)[0] == -1            # F aliases an input
    s3 = (16, 16, 16)
    P3 = torch.zeros(s3, dtype=torch.float64, device="cuda")
    assert _noalloc(pfc, s3, (16.0,) * 3, 0.56, P3, P3, 0.1, torch.empty_like(P3))[0] == -8
