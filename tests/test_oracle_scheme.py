"""Pins of the FP64 oracle's scheme (CPU only).

Each test checks the oracle against something other than itself: a Fourier
closed form, an exact identity the paper proves (DVD summation, energy law,
summation by parts, mass conservation), complex-step differentiation, a direct
sparse solve, or a manufactured solution with known convergence order.
"""
import math
import os

import numpy as np
import pytest

from oracle import scheme as S
import pfc_inputs as I


def _rand_pair(shape, seed=0, mean=-0.285, amp=0.3):
    g = np.random.default_rng(seed)
    phi = mean + amp * g.uniform(-1, 1, shape)
    Phi = phi + 0.1 * g.standard_normal(shape)
    return Phi, phi


@pytest.mark.parametrize("shape,lengths", [((12, 10), (7.0, 5.0)), ((6, 8, 10), (4.0, 5.0, 6.0))])
def test_laplacian_fourier_symbol(shape, lengths):
    # Delta_d exp(i k.x) = -sum_a (4/h_a^2) sin^2(pi k_a / N_a) exp(i k.x)
    h = S.spacing(shape, lengths)
    ks = [2, 3, 1][: len(shape)]
    idx = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    theta = sum(2 * np.pi * k * i / n for k, i, n in zip(ks, idx, shape))
    u = np.cos(theta)
    sym = sum(4.0 / h[a] ** 2 * math.sin(math.pi * ks[a] / shape[a]) ** 2 for a in range(len(shape)))
    np.testing.assert_allclose(S.lap(u, h), -sym * u, atol=1e-12 * sym)
    L = S.laplacian_matrix(shape, h)
    np.testing.assert_allclose((L @ u.ravel()).reshape(shape), -sym * u, atol=1e-12 * sym)


def test_laplacian_bruteforce_matrix():
    shape, h = (5, 7), (0.7, 0.3)
    n = 35
    D = np.zeros((n, n))
    for j in range(5):
        for i in range(7):
            p = j * 7 + i
            D[p, p] += -2 / h[0] ** 2 - 2 / h[1] ** 2
            D[p, ((j + 1) % 5) * 7 + i] += 1 / h[0] ** 2
            D[p, ((j - 1) % 5) * 7 + i] += 1 / h[0] ** 2
            D[p, j * 7 + (i + 1) % 7] += 1 / h[1] ** 2
            D[p, j * 7 + (i - 1) % 7] += 1 / h[1] ** 2
    np.testing.assert_allclose(S.laplacian_matrix(shape, h).toarray(), D, atol=1e-12)
    u = np.random.default_rng(1).standard_normal(shape)
    np.testing.assert_allclose(S.lap(u, h).ravel(), D @ u.ravel(), atol=1e-11)


def test_energy_constant_state():
    # gradient and curvature terms vanish: G_d = (1-gamma)/2 c^2 + c^4/4
    c, g = -0.37, 0.25
    phi = np.full((8, 9), c)
    h = (0.5, 0.25)
    G = S.local_energy(phi, g, h)
    np.testing.assert_allclose(G, 0.5 * (1 - g) * c * c + 0.25 * c ** 4, rtol=1e-14)
    assert abs(S.free_energy(phi, g, h) - G.sum() * 0.125) < 1e-12


def test_energy_single_mode_closed_form():
    # phi = a sin(k x): mean sin^2 = 1/2, mean sin^4 = 3/8, Delta_d phi = -lam phi,
    # mean (D^+ phi)^2 = mean (D^- phi)^2 = lam a^2 / 2 with lam = (4/h^2) sin^2(k h/2).
    n, L, g, a, m = 32, 20.0, 0.3, 0.7, 3
    h = L / n
    x = (np.arange(n) + 0.5) * h
    k = 2 * np.pi * m / L
    phi = np.tile(a * np.sin(k * x), (6, 1))       # axes (y, x); 6 rows in y
    hh = (1.0, h)
    lam = 4 / h ** 2 * math.sin(k * h / 2) ** 2
    mean_G = (1 - g) * a * a / 4 + 3 * a ** 4 / 32 + lam * lam * a * a / 4 - lam * a * a / 2
    assert abs(S.free_energy(phi, g, hh) - mean_G * 6 * L) < 1e-11 * abs(mean_G * 6 * L) + 1e-12


@pytest.mark.parametrize("shape", [(16, 12), (6, 7, 8)])
def test_dvd_summation_identity(shape):
    # Eq. (10): sum (G_d(Phi) - G_d(phi)) = sum mu_d (Phi - phi)
    h = tuple(0.4 + 0.1 * a for a in range(len(shape)))
    Phi, phi = _rand_pair(shape, 3)
    g = 0.25
    lhs = np.sum(S.local_energy(Phi, g, h) - S.local_energy(phi, g, h))
    rhs = np.sum(S.dvd_derivative(Phi, phi, g, h) * (Phi - phi))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, np.sum(np.abs(S.local_energy(Phi, g, h))))


@pytest.mark.parametrize("shape", [(16, 12), (6, 7, 8)])
def test_energy_law_identity(shape):
    # Eqs. (14)-(15) for any Phi (not only the root):
    # F_d(Phi) - F_d(phi) = -dt vol sum_a sum (D^+_a mu)^2 + dt vol sum mu F(Phi)
    h = tuple(0.5 + 0.05 * a for a in range(len(shape)))
    Phi, phi = _rand_pair(shape, 4)
    g, dt = 0.35, 0.7
    mu = S.dvd_derivative(Phi, phi, g, h)
    F = S.residual(Phi, phi, dt, g, h)
    vol = float(np.prod(h))
    dissip = sum(np.sum(S.d_plus(mu, h, a) ** 2) for a in range(len(shape)))
    lhs = S.free_energy(Phi, g, h) - S.free_energy(phi, g, h)
    rhs = -dt * vol * dissip + dt * vol * np.sum(mu * F)
    assert abs(lhs - rhs) <= 1e-10 * (abs(lhs) + dt * vol * dissip)


def test_summation_by_parts_variable_mobility():
    # Eq. (14): sum g (D M D) g = -sum M/2 [(D^+ g)^2 + (D^- g)^2], per axis, edge M = node mean
    shape, h = (10, 14), (0.6, 0.45)
    g = np.random.default_rng(5).standard_normal(shape)
    M = 1.0 + 0.5 * np.random.default_rng(6).uniform(size=shape)
    lhs = np.sum(g * S.div_mobility_grad(g, M, h))
    rhs = -sum(np.sum(M / 2 * (S.d_plus(g, h, a) ** 2 + S.d_minus(g, h, a) ** 2)) for a in range(2))
    assert abs(lhs - rhs) <= 1e-11 * abs(rhs)
    np.testing.assert_allclose(S.div_mobility_grad(g, np.ones(shape), h), S.lap(g, h), atol=1e-12)


@pytest.mark.parametrize("mob", [None, S.mobility_one_minus_sq])
def test_mass_identity(mob):
    # the flux divergence sums to zero, so sum F(Phi) = sum (Phi - phi)/dt exactly
    shape, h = (12, 12), (0.5, 0.5)
    Phi, phi = _rand_pair(shape, 7)
    dt = 0.3
    F = S.residual(Phi, phi, dt, 0.25, h, mobility=mob)
    assert abs(F.sum() - (Phi - phi).sum() / dt) <= 1e-10 * np.abs(F).sum()


def test_residual_constant_states():
    shape, h = (8, 8), (0.5, 0.5)
    Phi, phi = np.full(shape, 0.3), np.full(shape, -0.1)
    np.testing.assert_allclose(S.residual(Phi, phi, 0.2, 0.25, h), (0.3 + 0.1) / 0.2, rtol=1e-14)


def test_residual_single_mode_closed_form():
    # Phi = phi = a sin(theta), theta = k x: u = phi, q = a^3 sin^3 = a^3 (3 sin - sin 3theta)/4,
    # F = -Delta_d mu = lam1 [(1-g) - 2 lam1 + lam1^2 + 3a^2/4] a sin(theta) - lam3 a^3/4 sin(3 theta)
    n, L, g, a, m = 48, 30.0, 0.25, 0.4, 2
    h = L / n
    x = (np.arange(n) + 0.5) * h
    k = 2 * np.pi * m / L
    th = k * x
    phi = np.tile(a * np.sin(th), (5, 1))
    lam1 = 4 / h ** 2 * math.sin(k * h / 2) ** 2
    lam3 = 4 / h ** 2 * math.sin(3 * k * h / 2) ** 2
    expect = (lam1 * ((1 - g) - 2 * lam1 + lam1 ** 2 + 0.75 * a * a) * a * np.sin(th)
              - lam3 * a ** 3 / 4 * np.sin(3 * th))
    F = S.residual(phi, phi, 0.1, g, (1.0, h))
    np.testing.assert_allclose(F, np.tile(expect, (5, 1)), atol=1e-12 * np.abs(expect).max())


@pytest.mark.parametrize("shape", [(10, 9), (7, 8, 9)])
def test_jacobian_complex_step(shape):
    # F is a polynomial in Phi, so Im F(Phi + i e v) / e is J v to rounding
    h = tuple(0.7 + 0.1 * a for a in range(len(shape)))
    Phi, phi = _rand_pair(shape, 8)
    v = np.random.default_rng(9).standard_normal(shape)
    dt, g, e = 0.4, 0.3, 1e-30
    cs = np.imag(S.residual(Phi + 1j * e * v, phi, dt, g, h)) / e
    J = S.jacobian_csr(Phi, phi, dt, g, h)
    scale = np.abs(cs).max()
    np.testing.assert_allclose((J @ v.ravel()).reshape(shape), cs, atol=1e-13 * scale)
    np.testing.assert_allclose(S.jv(Phi, phi, dt, g, h, v), cs, atol=1e-13 * scale)
    # row nonzero count of the composite stencil: 25 (2-D) / 63 (3-D)
    assert J.getrow(0).nnz == (25 if len(shape) == 2 else 63)


def test_jacobian_symbol_uniform_state():
    shape, lengths = (16, 12), (9.0, 7.0)
    h = S.spacing(shape, lengths)
    c0, dt, g = -0.3, 2.0, 0.25
    Phi = np.full(shape, c0)
    cbar = float(S.jacobian_coef(Phi, Phi)[0, 0])
    sym = S.jacobian_symbol(shape, h, dt, g, cbar)
    for ky, kx in [(0, 0), (3, 2), (8, 6), (5, 1)]:
        jj, ii = np.meshgrid(np.arange(16), np.arange(12), indexing="ij")
        u = np.cos(2 * np.pi * (ky * jj / 16 + kx * ii / 12))
        Ju = S.jv(Phi, Phi, dt, g, h, u)
        np.testing.assert_allclose(Ju, sym[ky, kx] * u, atol=1e-11 * max(1, abs(sym[ky, kx])))


def test_newton_converges_quadratically_to_floor():
    w = I.small_noise_64()
    phi = w.initial()
    h = S.spacing(w.shape, w.lengths)
    res = S.newton_solve(phi, 0.1, w.gamma, h)
    assert res.res_norms[-1] < 1e-12
    r = res.res_norms
    # quadratic phase: r_{k+1} <= C r_k^2 once r_k < 1e-2
    for a, b in zip(r[1:-1], r[2:]):
        if 1e-9 < a < 1e-2:
            assert b <= 50 * a * a + 1e-13


def test_fft_gmres_newton_matches_direct():
    w = I.crystal_growth(64, (2, 2))
    phi = w.initial()
    h = S.spacing(w.shape, w.lengths)
    for dt in (0.5, 10.0):
        a = S.newton_solve(phi, dt, w.gamma, h, linear="direct").Phi
        b = S.newton_solve(phi, dt, w.gamma, h, linear="fftgmres").Phi
        assert S.rel_l2(b, a) < 1e-12


def test_adaptive_dt_special_cases():
    assert S.adaptive_dt(5.0, 5.0, 0.3, 0.01, 10.0, 4e5) == 10.0          # F' = 0
    assert S.adaptive_dt(5.0, 4.0, 1.0, 0.01, 10.0, 0.0) == 10.0          # eta = 0
    # eta |F'|^2 = 3  ->  dt_max / 2
    assert abs(S.adaptive_dt(1.0 + math.sqrt(3.0) * 0.5, 1.0, 0.5, 0.01, 10.0, 1.0) - 5.0) < 1e-12
    assert S.adaptive_dt(100.0, 0.0, 0.01, 0.02, 10.0, 5000.0) == 0.02    # floor


def test_energy_monotone_and_mass_conserved_small_run():
    w = I.small_noise_64()
    phi = w.initial()
    h = S.spacing(w.shape, w.lengths)
    tr = S.run(phi, 3, w.gamma, h, 0.1, 0.1)
    assert all(b <= a + 1e-10 for a, b in zip(tr.energies, tr.energies[1:]))
    assert max(abs(m - tr.masses[0]) for m in tr.masses) <= 1e-12 * abs(tr.masses[0])


# ---------------------------------------------------------------------------
# Manufactured solution: second order in space and time (Sec. 5, accuracy study)
# ---------------------------------------------------------------------------

def _mms(L, n, g, pbar=-0.2, a=0.3):
    k = 2 * np.pi / L
    h = L / n
    x = (np.arange(n) + 0.5) * h
    X, Y = np.meshgrid(x, x, indexing="xy")
    K = 2 * k * k

    def exact(t):
        return pbar + a * math.exp(-t) * np.sin(k * X) * np.cos(k * Y)

    def source(t):
        psi = a * math.exp(-t) * np.sin(k * X) * np.cos(k * Y)
        phi = pbar + psi
        gx = a * math.exp(-t) * k * np.cos(k * X) * np.cos(k * Y)
        gy = -a * math.exp(-t) * k * np.sin(k * X) * np.sin(k * Y)
        lin = -K * ((1 - g) - 2 * K + K * K) * psi          # Delta[(1-g) psi + 2 Delta psi + Delta^2 psi]
        cub = 3 * phi ** 2 * (-K * psi) + 6 * phi * (gx * gx + gy * gy)   # Delta(phi^3)
        return -psi - (lin + cub)

    return exact, source, (h, h)


def _mms_solve(L, n, g, T, nsteps):
    exact, source, h = _mms(L, n, g)
    dt = T / nsteps
    phi = exact(0.0)
    for s in range(nsteps):
        src = 0.5 * (source(s * dt) + source((s + 1) * dt))
        phi = S.newton_solve(phi, dt, g, h, src=src, linear="direct").Phi
    return phi, exact(T)


def test_mms_truncation_error_second_order():
    # consistency: residual of the exact solution is O(h^2 + dt^2)
    L, g = 8 * np.pi, 0.25
    errs_h = []
    for n in (32, 64, 128):
        exact, source, h = _mms(L, n, g)
        dt = 1e-4
        tau = S.residual(exact(dt), exact(0.0), dt, g, h, src=0.5 * (source(0) + source(dt)))
        errs_h.append(np.abs(tau).max())
    rates = [math.log2(a / b) for a, b in zip(errs_h, errs_h[1:])]
    assert all(1.9 < r < 2.1 for r in rates), rates
    errs_t = []
    exact, source, h = _mms(L, 64, g)
    for dt in (0.2, 0.1, 0.05):
        tau = S.residual(exact(1 + dt), exact(1.0), dt, g, h, src=0.5 * (source(1) + source(1 + dt)))
        tau0 = S.residual(exact(1 + 1e-6), exact(1.0), 1e-6, g, h,
                          src=0.5 * (source(1) + source(1 + 1e-6)))
        errs_t.append(np.abs(tau - tau0).max())
    rates = [math.log2(a / b) for a, b in zip(errs_t, errs_t[1:])]
    assert all(1.9 < r < 2.1 for r in rates), rates


def test_mms_solution_converges_second_order_in_space():
    L, g, T = 8 * np.pi, 0.25, 0.2
    errs = []
    for n in (12, 24, 48):
        num, ex = _mms_solve(L, n, g, T, 40)
        errs.append(S.rel_l2(num, ex))
    rates = [math.log2(a / b) for a, b in zip(errs, errs[1:])]
    assert all(1.8 < r < 2.2 for r in rates), (errs, rates)


def test_solution_self_convergence_second_order_in_time():
    L, g, T, n = 8 * np.pi, 0.25, 1.0, 16
    ref, _ = _mms_solve(L, n, g, T, 256)
    errs = [S.rel_l2(_mms_solve(L, n, g, T, m)[0], ref) for m in (8, 16, 32)]
    rates = [math.log2(a / b) for a, b in zip(errs, errs[1:])]
    assert all(1.8 < r < 2.3 for r in rates), (errs, rates)


def test_fft_gmres_newton_matches_direct_128():
    """The oracle's solver above 256^2 (FFT-preconditioned GMRES to 1e-14) gives the root of
    the exact sparse direct Newton at 128^2 on the crystal mesh size, small and large dt."""
    w = I.crystal_growth(128, (2, 2))
    phi = w.initial()
    h = S.spacing(w.shape, w.lengths)
    for dt in (0.01, 10.0):
        a = S.newton_solve(phi, dt, w.gamma, h, linear="direct")
        b = S.newton_solve(phi, dt, w.gamma, h, linear="fftgmres")
        assert a.converged and b.converged
        assert S.rel_l2(b.Phi, a.Phi) < 1e-12


@pytest.mark.slow
@pytest.mark.skipif(not os.environ.get("PFC_SLOW_TESTS"),
                    reason="3 minutes of SuperLU at 256^2; set PFC_SLOW_TESTS=1 (the 128^2 case runs by default)")
def test_fft_gmres_newton_matches_direct_256():
    w = I.crystal_growth(256, (2, 2))
    phi = w.initial()
    h = S.spacing(w.shape, w.lengths)
    a = S.newton_solve(phi, 1.0, w.gamma, h, linear="direct")
    b = S.newton_solve(phi, 1.0, w.gamma, h, linear="fftgmres")
    assert S.rel_l2(b.Phi, a.Phi) < 1e-12


def test_fft_gmres_refuses_an_unconverged_solve():
    """A system with no solution (the Jacobian with its first row zeroed, a right-hand side
    that is not zero there) raises instead of returning an inexact direction."""
    w = I.crystal_growth(64, (2, 2))
    phi = w.initial()
    h = S.spacing(w.shape, w.lengths)
    J = S.jacobian_csr(phi, phi, 10.0, w.gamma, h)
    rhs = np.random.default_rng(0).standard_normal(phi.size)
    bad = J.tolil()
    bad[0, :] = 0.0
    with pytest.raises(RuntimeError):
        S._solve_fft_gmres(bad.tocsr(), rhs, w.shape, h, 10.0, w.gamma, float(np.mean(S.jacobian_coef(phi, phi))))
    x = S._solve_fft_gmres(J, rhs, w.shape, h, 10.0, w.gamma, float(np.mean(S.jacobian_coef(phi, phi))))
    floor = np.finfo(np.float64).eps * np.linalg.norm(abs(J) @ np.abs(x))     # rounding level of J x
    assert np.linalg.norm(J @ x - rhs) <= max(1e-12 * np.linalg.norm(rhs), floor)


def test_run_dt_history_three_steps():
    """Eq. (16) in the time loop: dt_0 = dt_min; dt_1 from F^1, F^0 and dt_0; dt_2 from F^2, F^1
    and dt_1 (the energies of the states the loop accepted).  A constant state keeps its
    energy, so every later step takes dt_max; eta = 0 does the same for any state."""
    w = I.small_noise_64()
    h = S.spacing(w.shape, w.lengths)
    phi0 = w.initial()
    tr = S.run(phi0, 3, w.gamma, h, 0.05, 2.0, eta=0.01)
    E, d = tr.energies, tr.dts
    assert d[0] == 0.05
    fp1 = abs(E[1] - E[0]) / d[0]
    fp2 = abs(E[2] - E[1]) / d[1]
    assert d[1] == pytest.approx(max(0.05, 2.0 / math.sqrt(1.0 + 0.01 * fp1 * fp1)), rel=1e-15)
    assert d[2] == pytest.approx(max(0.05, 2.0 / math.sqrt(1.0 + 0.01 * fp2 * fp2)), rel=1e-15)
    assert 0.05 < d[1] < 2.0 and 0.05 < d[2] < 2.0          # the formula's interior branch ran
    flat = S.run(np.full(w.shape, -0.285), 3, w.gamma, h, 0.05, 2.0, eta=40.0)
    assert flat.dts == [0.05, 2.0, 2.0]
    free = S.run(phi0, 2, w.gamma, h, 0.05, 2.0, eta=0.0)
    assert free.dts == [0.05, 2.0]


# ---------------------------------------------------------------------------
# Variable mobility M = 1 - phi^2 and Neumann-type boundary conditions (Sec. 2; Sec. 3,
# Eq. (12) with M_d at the averaged state; Sec. 5, test B's four variants)
# ---------------------------------------------------------------------------

VARIANTS = [("periodic", None), ("periodic", S.mobility_one_minus_sq), ("neumann", None),
            ("neumann", S.mobility_one_minus_sq)]


def _pair(shape, seed, amp=0.3):
    g = np.random.default_rng(seed)
    phi = -0.2 + amp * g.uniform(-1, 1, shape)
    return phi + 0.1 * g.standard_normal(shape), phi


def _mirror_ext(u):
    """Even reflection across every upper face: a periodic field on twice the grid whose
    wrap reproduces the Neumann mirror ghosts of ``u``."""
    for a in range(u.ndim):
        u = np.concatenate([u, np.flip(u, axis=a)], axis=a)
    return u


@pytest.mark.parametrize("bc,mob", VARIANTS)
def test_jacobian_complex_step_all_variants(bc, mob):
    shape, h, gam, dt = (9, 11), (0.7, 0.9), 0.3, 0.37
    Phi, phi = _pair(shape, 11)
    v = np.random.default_rng(12).standard_normal(shape)
    cs = S.residual(Phi + 1e-30j * v, phi, dt, gam, h, mobility=mob, bc=bc).imag / 1e-30
    scale = np.abs(cs).max()
    assert np.abs(S.jv(Phi, phi, dt, gam, h, v, mobility=mob, bc=bc) - cs).max() <= 1e-14 * scale
    J = S.jacobian_csr(Phi, phi, dt, gam, h, mobility=mob, bc=bc)
    assert np.abs(J @ v.ravel() - cs.ravel()).max() <= 1e-14 * scale


@pytest.mark.parametrize("mob", [None, S.mobility_one_minus_sq])
def test_neumann_equals_periodic_on_the_mirror_extended_grid(mob):
    """The Neumann mirror ghosts are what a periodic grid of twice the size gives for the even
    reflection of the field, so every Neumann quantity is the periodic one restricted."""
    shape, h, gam, dt = (7, 10), (0.8, 0.6), 0.25, 0.5
    Phi, phi = _pair(shape, 13)
    F = S.residual(Phi, phi, dt, gam, h, mobility=mob, bc="neumann")
    Fe = S.residual(_mirror_ext(Phi), _mirror_ext(phi), dt, gam, h, mobility=mob)
    np.testing.assert_allclose(F, Fe[:7, :10], rtol=0, atol=1e-12 * np.abs(F).max())
    v = np.random.default_rng(14).standard_normal(shape)
    Jv = S.jv(Phi, phi, dt, gam, h, v, mobility=mob, bc="neumann")
    Jve = S.jv(_mirror_ext(Phi), _mirror_ext(phi), dt, gam, h, _mirror_ext(v), mobility=mob)
    np.testing.assert_allclose(Jv, Jve[:7, :10], rtol=0, atol=1e-12 * np.abs(Jv).max())
    E = S.free_energy(phi, gam, h, "neumann")
    assert abs(4.0 * E - S.free_energy(_mirror_ext(phi), gam, h)) <= 1e-12 * abs(E)


def test_neumann_laplacian_spectrum_is_the_cosine_symbol():
    """Under the mirror ghosts Delta_d is diagonalised by the cosines cos(pi k (i + 1/2) / n),
    eigenvalue -(4/h^2) sin^2(pi k / (2n)) per axis."""
    shape, h = (6, 9), (0.7, 1.3)
    L = S.laplacian_matrix(shape, h, "neumann").toarray()
    lam = [(4.0 / h[a] ** 2) * np.sin(np.pi * np.arange(shape[a]) / (2 * shape[a])) ** 2 for a in range(2)]
    expect = np.sort(-(lam[0][:, None] + lam[1][None, :]).ravel())
    np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(L)), expect, atol=1e-12 * np.abs(expect).max())


@pytest.mark.parametrize("bc,mob", VARIANTS)
def test_dvd_energy_law_and_mass_all_variants(bc, mob):
    """For any Phi (not only the root): the DVD identity vol sum(G(Phi) - G(phi)) =
    vol sum mu (Phi - phi) (Eq. (10)); with it and summation by parts the energy law
    F(Phi) - F(phi) = dt vol [sum mu F(Phi) - sum_faces M_e (D^+ mu)^2] (Eqs. (14)-(15), here with
    the mobility on the faces and no flux through Neumann faces); and sum F = sum (Phi - phi)/dt."""
    shape, h, gam, dt = (10, 12), (0.7, 0.9), 0.3, 0.41
    Phi, phi = _pair(shape, 15)
    vol = h[0] * h[1]
    mu = S.dvd_derivative(Phi, phi, gam, h, bc)
    dE = S.free_energy(Phi, gam, h, bc) - S.free_energy(phi, gam, h, bc)
    assert abs(dE - vol * np.sum(mu * (Phi - phi))) <= 1e-12 * abs(dE)
    F = S.residual(Phi, phi, dt, gam, h, mobility=mob, bc=bc)
    m = np.ones(shape) if mob is None else mob(0.5 * (Phi + phi))
    diss = 0.0
    for a in range(2):
        n = shape[a]
        dmu = np.diff(mu, axis=a) if bc == "neumann" else np.roll(mu, -1, axis=a) - mu
        me = 0.5 * (np.take(m, range(n - 1), axis=a) + np.take(m, range(1, n), axis=a)) if bc == "neumann" \
            else 0.5 * (m + np.roll(m, -1, axis=a))
        diss += np.sum(me * dmu ** 2) / h[a] ** 2
    rhs = dt * vol * (np.sum(mu * F) - diss)
    assert abs(dE - rhs) <= 1e-11 * max(abs(dE), 1.0)
    assert abs(np.sum(F) - np.sum(Phi - phi) / dt) <= 1e-12 * np.abs(Phi - phi).sum() / dt


@pytest.mark.parametrize("bc,mob", VARIANTS)
def test_newton_root_and_short_run_all_variants(bc, mob):
    """Newton with the exact Jacobian converges quadratically to the rounding floor for all
    four variants of test B (Sec. 5); over a short run the energy does not increase and the
    mass is kept."""
    shape = (16, 16)
    L = (16 * 400.0 / 1024,) * 2
    h = S.spacing(shape, L)
    phi = I.noise_ic(shape, -0.285, 0.1, 3)
    res = S.newton_solve(phi, 0.1, 0.25, h, mobility=mob, bc=bc)
    assert res.converged and res.res_norms[-1] < 1e-9
    tr = S.run(phi, 3, 0.25, h, 0.1, 0.1, mobility=mob, bc=bc)
    assert all(b <= a + 1e-12 * abs(a) for a, b in zip(tr.energies, tr.energies[1:]))
    assert max(abs(m - tr.masses[0]) for m in tr.masses) <= 1e-12 * abs(tr.masses[0])
