"""Pins of the oracle's Krylov-Schwarz reference routines (CPU only)."""
import numpy as np
import pytest

from oracle import scheme as S
from oracle import schwarz as W


def _state(shape, seed=0):
    g = np.random.default_rng(seed)
    phi = -0.285 + 0.05 * g.uniform(-1, 1, shape)
    Phi = phi + 0.01 * g.standard_normal(shape)
    return Phi, phi


def test_decomposition_partitions_grid():
    shape = (30, 22)
    doms = W.decompose(shape, (3, 4), 2)
    cover = np.zeros(shape, int)
    for d in doms:
        idx = d.ext_global_indices()
        own = d.owned_mask_local()
        cover.ravel()[idx[own]] += 1
        assert idx.size == np.prod(d.ext_n)
        assert len(np.unique(idx)) == idx.size
    assert (cover == 1).all()
    with pytest.raises(ValueError):
        W.decompose((16, 16), (1, 4), 1)
    with pytest.raises(ValueError):
        W.decompose((16, 16), (2, 2), 3)        # 8 + 6 > 16 - 3


@pytest.mark.parametrize("shape,sub,ov", [((16, 14), (2, 2), 2), ((12, 12, 12), (2, 2, 2), 1)])
def test_subdomain_matrix_equals_zero_ring_problem(shape, sub, ov):
    # Eq. (25) (restriction of the global Jacobian) and Eq. (26) (subdomain problem
    # with phi = 0 on the three-layer ring) give the same matrix.
    h = tuple(0.6 + 0.1 * a for a in range(len(shape)))
    Phi, phi = _state(shape, 1)
    dt, g = 0.7, 0.25
    J = S.jacobian_csr(Phi, phi, dt, g, h)
    for d in W.decompose(shape, sub, ov)[:3]:
        A1 = W.subdomain_matrix(J, d).toarray()
        A2 = W.subdomain_matrix_zero_ring(Phi, phi, dt, g, h, d)
        np.testing.assert_allclose(A1, A2, atol=1e-12 * np.abs(A1).max())
        # structural pattern = stencil couplings inside the box
        pat = W.subdomain_pattern(d.ext_n)
        for i in range(0, A1.shape[0], 7):
            assert sorted(np.nonzero(A1[i])[0].tolist()) == pat[i]


def test_ilu0_defining_property():
    shape, h = (16, 16), (np.pi / 2, np.pi / 2)
    Phi, phi = _state(shape, 2)
    J = S.jacobian_csr(Phi, phi, 0.1, 0.25, h)
    d = W.decompose(shape, (2, 2), 2)[3]
    A = W.subdomain_matrix(J, d).toarray()
    pat = W.subdomain_pattern(d.ext_n)
    rows = W.ilu0(A, pat)
    L, U = W.ilu0_dense_factors(rows)
    LU = L @ U
    for i, p in enumerate(pat):
        np.testing.assert_allclose(LU[i, p], A[i, p], atol=1e-12 * np.abs(A).max())
        # no entry outside the pattern
        outside = np.setdiff1d(np.arange(A.shape[0]), p)
        assert np.all(L[i, outside[outside < i]] == 0) and np.all(U[i, outside[outside > i]] == 0)
    b = np.random.default_rng(3).standard_normal(A.shape[0])
    np.testing.assert_allclose(W.ilu0_solve(rows, b), np.linalg.solve(LU, b), rtol=1e-10, atol=1e-12)


def test_ilu0_is_exact_when_pattern_is_full():
    # in a 2x3 box every pair of cells is within |dx|+|dy| <= 3, so the pattern is
    # full, no fill is dropped and ILU(0) is the exact LU factorisation.
    rng = np.random.default_rng(4)
    ext = (2, 3)
    pat = W.subdomain_pattern(ext)
    assert all(len(p) == 6 for p in pat)
    A = rng.standard_normal((6, 6)) + 8 * np.eye(6)
    rows = W.ilu0(A, pat)
    b = rng.standard_normal(6)
    np.testing.assert_allclose(W.ilu0_solve(rows, b), np.linalg.solve(A, b), rtol=1e-12)


def test_ilu0_tridiagonal_no_fill_is_exact():
    n = 12
    rng = np.random.default_rng(5)
    A = np.diag(4 + rng.uniform(size=n)) + np.diag(rng.uniform(size=n - 1), 1) + np.diag(rng.uniform(size=n - 1), -1)
    pat = [[j for j in (i - 1, i, i + 1) if 0 <= j < n] for i in range(n)]
    rows = W.ilu0(A, pat)
    b = rng.standard_normal(n)
    np.testing.assert_allclose(W.ilu0_solve(rows, b), np.linalg.solve(A, b), rtol=1e-12)


def test_schwarz_overlap0_is_block_jacobi_and_variants_agree():
    shape, h = (16, 16), (0.8, 0.8)
    Phi, phi = _state(shape, 6)
    J = S.jacobian_csr(Phi, phi, 0.5, 0.25, h)
    doms = W.decompose(shape, (2, 2), 0)
    sol = W.schwarz_setup(J, doms, "lu")
    r = np.random.default_rng(7).standard_normal(shape)
    Jd = J.toarray()
    expect = np.zeros(r.size)
    for d in doms:
        idx = d.ext_global_indices()
        expect[idx] = np.linalg.solve(Jd[np.ix_(idx, idx)], r.ravel()[idx])
    for var in ("left", "right", "as"):
        np.testing.assert_allclose(W.schwarz_apply(r, doms, sol, var).ravel(), expect, rtol=1e-10, atol=1e-12)


def test_left_ras_matches_dense_definition():
    # Eq. (23) written with dense solves of the zero-ring subdomain problems (Eq. (26))
    shape, h = (20, 18), (0.9, 0.9)
    Phi, phi = _state(shape, 8)
    dt, g = 1.0, 0.25
    J = S.jacobian_csr(Phi, phi, dt, g, h)
    doms = W.decompose(shape, (2, 3), 2)
    sol = W.schwarz_setup(J, doms, "lu")
    r = np.random.default_rng(9).standard_normal(shape)
    z = W.schwarz_apply(r, doms, sol, "left").ravel()
    expect = np.zeros(r.size)
    for d in doms:
        A = W.subdomain_matrix_zero_ring(Phi, phi, dt, g, h, d)
        idx = d.ext_global_indices()
        y = np.linalg.solve(A, r.ravel()[idx])
        own = d.owned_mask_local()
        expect[idx[own]] = y[own]
    np.testing.assert_allclose(z, expect, rtol=1e-10, atol=1e-12)
    # AS adds the overlapped parts: its owned part differs, its total is the sum of all extensions
    z_as = W.schwarz_apply(r, doms, sol, "as").ravel()
    tot = 0.0
    for d in doms:
        A = W.subdomain_matrix_zero_ring(Phi, phi, dt, g, h, d)
        tot += np.linalg.solve(A, r.ravel()[d.ext_global_indices()]).sum()
    assert abs(z_as.sum() - tot) < 1e-9 * np.abs(z_as).sum()


def test_fgmres_identity_full_restart_is_direct_solve():
    rng = np.random.default_rng(10)
    n = 40
    A = np.eye(n) * 3 + rng.standard_normal((n, n)) / np.sqrt(n)
    b = rng.standard_normal(n)
    res = W.fgmres(lambda x: A @ x, lambda v: v, b, 1e-14, 0.0, restart=n, maxit=n)
    np.testing.assert_allclose(res.x, np.linalg.solve(A, b), rtol=1e-10)
    # monitored residual is non-increasing and is the true residual at the end
    assert all(b2 <= b1 * (1 + 1e-12) for b1, b2 in zip(res.res_history, res.res_history[1:]))


def test_arnoldi_relation_and_orthonormality():
    rng = np.random.default_rng(11)
    n, m = 60, 12
    A = np.eye(n) + rng.standard_normal((n, n)) / np.sqrt(n)
    P = np.diag(1 + rng.uniform(size=n))
    V, Z, H = W.arnoldi_mgs(lambda x: A @ x, lambda v: P @ v, rng.standard_normal(n), m)
    np.testing.assert_allclose(A @ Z.T, V.T @ H, atol=1e-12)
    np.testing.assert_allclose(V @ V.T, np.eye(m + 1), atol=1e-12)


def test_fgmres_stopping_rule_with_ras():
    # the linear test of Sec. 4: ||J S + F|| <= max(xi_r ||F||, xi_a) at exit
    shape, h = (24, 24), (np.pi / 2, np.pi / 2)
    Phi, phi = _state(shape, 12)
    J = S.jacobian_csr(Phi, phi, 0.1, 0.25, h)
    doms = W.decompose(shape, (2, 2), 2)
    sol = W.schwarz_setup(J, doms, "ilu0")
    F = S.residual(Phi, phi, 0.1, 0.25, h).ravel()
    res = W.fgmres(lambda x: J @ x, lambda r: W.schwarz_apply(r, doms, sol, "left"), -F, 1e-3, 1e-11)
    true = np.linalg.norm(J @ res.x + F)
    assert true <= 1.0001 * max(1e-3 * np.linalg.norm(F), 1e-11)
    assert res.iterations <= 5      # ILU(0)-RAS is an excellent preconditioner at h = pi/2


def test_inexact_nks_reproduces_the_newton_count_of_table1_test_a():
    """The paper's printed Newton count pins the oracle's inexact Newton-Krylov-Schwarz step.

    Test A of the parameter study (Sec. 5, Table 1): 256 x 256 mesh on [0, 128]^2,
    gamma 0.025, phi = 0.07 + U(-0.07, 0.07), fixed dt = 0.01, first 10 steps, the listed
    tolerances, classical AS with delta = 1 (3 mesh layers) and LU subdomain solves on 24
    subdomains: 30 Newton iterations in all (every subdomain solver gives 30) and 3.87 GMRES
    iterations per Newton step.  The Newton count follows from the stop tests of Eqs. (20)
    and (21) (each inexact step gains about xi_r), so it is reproduced exactly; the GMRES
    count depends on the paper's random field and core layout, which are not given, and
    is checked to 20%."""
    import json
    import os

    import pfc_inputs as I

    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "test_a_newton_counts.json")))
    st = g["setup"]
    shape = tuple(st["mesh"])
    h = S.spacing(shape, tuple(st["domain"]))
    phi = I.noise_ic(shape, st["phi_mean"], st["phi_noise"], 0)
    newton = gmres = 0
    for _ in range(st["steps"]):
        r = W.nks_step(phi, st["dt"], st["gamma"], h, (4, 6), 3, kind="lu", variant="as", eps_r=st["eps_r"],
                       eps_a=st["eps_a"], xi_r=st["xi_r"], xi_a=st["xi_a"])
        assert r.res_norms[-1] <= max(st["eps_r"] * r.res_norms[0], st["eps_a"])
        phi = r.Phi
        newton += r.newton
        gmres += r.gmres
    ref = g["table1_classical_as_delta1"]
    assert newton == ref["total_newton"]["LU"]
    assert abs(gmres / newton - ref["gmres_per_newton"]["LU"]) <= 0.2 * ref["gmres_per_newton"]["LU"]


def test_nks_step_stops_where_eq20_says():
    """nks_step's stop test is Eq. (20) against ||F(phi^n)||: with eps_r = 0 it runs to eps_a,
    and a looser eps_r takes no more iterations (a dropped or misplaced reference fails here)."""
    shape = (32, 32)
    h = S.spacing(shape, (16.0, 16.0))
    phi = -0.285 + 0.05 * np.random.default_rng(3).uniform(-1, 1, shape)
    tight = W.nks_step(phi, 0.1, 0.25, h, (2, 2), 3, eps_r=0.0, eps_a=1e-9)
    loose = W.nks_step(phi, 0.1, 0.25, h, (2, 2), 3, eps_r=1e-4, eps_a=0.0)
    assert tight.res_norms[-1] <= 1e-9 < tight.res_norms[-2]
    assert loose.res_norms[-1] <= 1e-4 * loose.res_norms[0] < loose.res_norms[-2]
    assert loose.newton <= tight.newton
    F = S.residual(tight.Phi, phi, 0.1, 0.25, h)
    assert np.linalg.norm(F) == pytest.approx(tight.res_norms[-1], rel=1e-12)


@pytest.mark.parametrize("dt,stable", [(0.1, True), (0.5, False)])
def test_natural_order_ilu0_on_test_d_mesh_size(dt, stable):
    """Why test D's 256^3 grid runs at dt = 0.1: on its mesh size (h = 80 pi / 256) the
    natural-order ILU(0) of a 3-D subdomain matrix (Eqs. (25)-(26), liquid phi = -0.35,
    gamma = 0.35, box of 4^3 cells extended by 3 layers) keeps every pivot positive at the
    dt = 0.1 of the paper's test-D tuning runs, and loses that at its production dt_min = 0.5:
    negative pivots, and a preconditioned operator whose spectrum leaves any bounded region."""
    import math

    n_own, ov = 4, 3
    hv = 80 * math.pi / 256
    shape = (4 * n_own,) * 3
    h = S.spacing(shape, (hv * shape[0],) * 3)
    phi = np.full(shape, -0.35)
    dom = W.decompose(shape, (4, 4, 4), ov)[0]
    A = W.subdomain_matrix_zero_ring(phi, phi, dt, 0.35, h, dom)
    rows = W.ilu0(A, W.subdomain_pattern(dom.ext_n))
    piv = np.array([r[i] for i, r in enumerate(rows)])
    L, U = W.ilu0_dense_factors(rows)
    ev = np.linalg.eigvals(np.linalg.solve(U, np.linalg.solve(L, A)))
    if stable:
        assert piv.min() > 0
        assert 0 < ev.real.min() and abs(ev).max() < 10
    else:
        assert piv.min() < 0
        assert abs(ev).max() > 1e6


# ---------------------------------------------------------------------------
# ILU(k) (Sec. 4 subdomain solvers; Table 1's ILU(1) and ILU(2) columns)
# ---------------------------------------------------------------------------

def _fill_path_levels(pattern):
    """Level of every entry by the fill-path theorem (Hysom and Pothen): (i, j) has level L
    when the shortest path from i to j in the graph of A whose inner vertices are all numbered
    below min(i, j) has L + 1 edges.  Brute force, one search per pair."""
    n = len(pattern)
    adj = [set(p) - {i} for i, p in enumerate(pattern)]
    lev = {}
    for i in range(n):
        for j in range(n):
            if i == j:
                lev[(i, j)] = 0
                continue
            m = min(i, j)
            dist = {i: 0}
            frontier = [i]
            found = None
            while frontier and found is None:
                nxt = []
                for u in frontier:
                    for v in adj[u]:
                        if v == j:
                            found = dist[u] + 1
                            break
                        if v < m and v not in dist:
                            dist[v] = dist[u] + 1
                            nxt.append(v)
                    if found is not None:
                        break
                frontier = nxt
            if found is not None:
                lev[(i, j)] = found - 1
    return lev


@pytest.mark.parametrize("ext", [(8, 8), (9, 7)])
def test_iluk_levels_follow_the_fill_path_theorem(ext):
    pat = W.subdomain_pattern(ext)
    ref = _fill_path_levels(pat)
    for k in (0, 1, 2, 3):
        rows = W.iluk_levels(pat, k)
        got = {(i, j): v for i, r in enumerate(rows) for j, v in r.items()}
        want = {key: v for key, v in ref.items() if v <= k}
        assert got == want, k


def test_iluk_defining_property_and_nesting():
    shape, h = (20, 20), (0.5, 0.5)
    Phi, phi = _state(shape, 4)
    J = S.jacobian_csr(Phi, phi, 0.01, 0.25, h)
    d = W.decompose(shape, (2, 2), 2)[1]
    A = W.subdomain_matrix(J, d).toarray()
    pat = W.subdomain_pattern(d.ext_n)
    prev = None
    for k in (0, 1, 2):
        pk = W.iluk_pattern(pat, k)
        if prev is not None:
            assert all(set(a) < set(b) or set(a) == set(b) for a, b in zip(prev, pk))
            assert sum(map(len, pk)) > sum(map(len, prev))
        prev = pk
        L, U = W.ilu0_dense_factors(W.iluk(A, pat, k))
        LU = L @ U
        mask = np.zeros_like(A, dtype=bool)
        for i, cols in enumerate(pk):
            mask[i, cols] = True
        np.testing.assert_allclose(LU[mask], A[mask], atol=1e-11 * np.abs(A).max())
        if k == 0:
            assert W.iluk(A, pat, 0) == W.ilu0(A, pat)


def test_iluk_with_enough_levels_is_the_exact_lu():
    """With enough levels the pattern is the whole band profile of the box matrix (no entry
    of the exact LU factors is dropped) and ILU(k) is the exact factorisation."""
    shape, h = (16, 16), (0.5, 0.5)
    Phi, phi = _state(shape, 5)
    J = S.jacobian_csr(Phi, phi, 0.1, 0.25, h)
    d = W.decompose(shape, (2, 2), 1)[0]
    A = W.subdomain_matrix(J, d).toarray()
    pat = W.subdomain_pattern(d.ext_n)
    n = A.shape[0]
    k = 0
    while sum(map(len, W.iluk_pattern(pat, k))) != sum(map(len, W.iluk_pattern(pat, k + 1))):
        k += 1
    rows = W.iluk(A, pat, k)
    L, U = W.ilu0_dense_factors(rows)
    np.testing.assert_allclose(L @ U, A, atol=1e-12 * np.abs(A).max())
    b = np.random.default_rng(6).standard_normal(n)
    np.testing.assert_allclose(W.ilu0_solve(rows, b), np.linalg.solve(A, b), rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("dt,own,ov,stable_levels", [(0.01, 16, 4, (1, 2)), (1.0, 32, 3, ())])
def test_natural_order_iluk_on_test_b_mesh_size(dt, own, ov, stable_levels):
    """Why the 1024^2 crystal workload (test B's mesh, h = 400/1024) uses exact subdomain LU:
    natural-order ILU(k) of its subdomain matrices (Eqs. (25)-(26), at the benchmark's crystal
    state) is stable only at the benchmark's dt_min = 0.01 on boxes 24 cells wide, and only
    with fill (k = 1, 2: positive pivots, preconditioned spectrum near 1); ILU(0) has negative
    pivots there.  At test B's dt = 1 on a box 38 cells wide, ILU(0), ILU(1) and ILU(2) all
    have negative pivots and preconditioned spectra beyond 1e4 in modulus."""
    import pfc_inputs as I
    n = 8 * own
    L = 400.0 * n / 1024
    phi = I.hex_crystallites_ic(n=n, L=L, seed=1)
    h = S.spacing((n, n), (L, L))
    doms = W.decompose((n, n), (8, 8), ov)
    dom = max(doms, key=lambda d: np.var(phi.ravel()[d.ext_global_indices()]))   # a box on a crystallite
    A = W.subdomain_matrix_zero_ring(phi, phi, dt, 0.25, h, dom)
    pat = W.subdomain_pattern(dom.ext_n)
    for k in (0, 1, 2):
        rows = W.iluk(A, pat, k)
        piv = np.array([r[i] for i, r in enumerate(rows)])
        Lf, Uf = W.ilu0_dense_factors(rows)
        ev = np.linalg.eigvals(np.linalg.solve(Uf, np.linalg.solve(Lf, A)))
        if k in stable_levels:
            assert piv.min() > 0, k
            assert 0.5 < ev.real.min() and abs(ev).max() < 2, (k, ev.real.min(), abs(ev).max())
        else:
            assert piv.min() < 0, k
            assert abs(ev).max() > 1e4, (k, abs(ev).max())


@pytest.mark.slow
def test_natural_order_iluk_on_test_d_mesh_size():
    """Why test D's production steps (dt 0.5..10) run with ILU(2): on its mesh size, for the same
    3-D subdomain matrix as the ILU(0) pin above, ILU(2) keeps positive pivots and a
    preconditioned spectrum near 1 up to dt = 10, while ILU(1) loses them at dt = 10."""
    import math

    n_own, ov = 4, 3
    hv = 80 * math.pi / 256
    shape = (4 * n_own,) * 3
    h = S.spacing(shape, (hv * shape[0],) * 3)
    phi = np.full(shape, -0.35)
    dom = W.decompose(shape, (4, 4, 4), ov)[0]
    A = W.subdomain_matrix_zero_ring(phi, phi, 10.0, 0.35, h, dom)
    pat = W.subdomain_pattern(dom.ext_n)
    for k, stable in ((1, False), (2, True)):
        rows = W.iluk(A, pat, k)
        piv = np.array([r[i] for i, r in enumerate(rows)])
        L, U = W.ilu0_dense_factors(rows)
        ev = np.linalg.eigvals(np.linalg.solve(U, np.linalg.solve(L, A)))
        if stable:
            assert piv.min() > 0 and 0.5 < ev.real.min() and abs(ev).max() < 2, k
        else:
            assert piv.min() < 0 and abs(ev).max() > 10, k
