"""FP64 oracle of the discrete PFC scheme and of its per-step nonlinear solve.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Arrays are numpy float64 with C order; axis order is (z, y, x) in 3-D and (y, x)
in 2-D, so x is the fastest index.  ``h`` is the tuple of mesh sizes per array
axis.  The mesh is cell centred (Sec. 3: cell centres at (i - 1/2) * dx,
1 <= i <= Nx).  Boundary conditions (Sec. 2): ``bc="periodic"`` (every shift wraps
around) or ``bc="neumann"``, the Neumann-type conditions read as zero normal
differences: the ghost cell beyond a boundary face mirrors the cell inside it
(u_0 = u_1, u_(N+1) = u_N), applied to every field a difference operator acts on.

Everything here follows the paper's definitions one to one; the only library
primitives used are ``numpy.roll`` (periodic index shift), ``scipy.sparse``
assembly, a sparse LU (SuperLU) and, for grids too large for a direct solve,
scipy's GMRES with an FFT preconditioner.  Whatever solver is used, the result
is the root of the discrete system to the floating-point floor, which is the
definition of the step.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.fft
import scipy.sparse as sp
import scipy.sparse.linalg as spla


# ---------------------------------------------------------------------------
# Grid and difference operators (Sec. 3: D^+, D^-, D^<2>, Delta_d)
# ---------------------------------------------------------------------------

def spacing(shape, lengths):
    """Mesh sizes h_a = L_a / N_a per array axis (Sec. 3, uniform mesh)."""
    return tuple(float(L) / int(n) for n, L in zip(shape, lengths))


BCS = ("periodic", "neumann")


def _nbr(u, axis, s, bc="periodic"):
    """u at index i+s (s = +1 or -1) along ``axis``: periodic wrap, or the mirror ghost of the
    Neumann-type conditions (the cell itself where i+s leaves the grid)."""
    if bc == "periodic":
        return np.roll(u, -s, axis=axis)
    if bc != "neumann" or s not in (1, -1):
        raise ValueError(f"bad boundary condition {bc!r} or shift {s}")
    n = u.shape[axis]
    idx = np.clip(np.arange(n) + s, 0, n - 1)
    return np.take(u, idx, axis=axis)


def d_plus(u, h, axis, bc="periodic"):
    """Forward difference D^+ along ``axis`` (Sec. 3)."""
    return (_nbr(u, axis, 1, bc) - u) / h[axis]


def d_minus(u, h, axis, bc="periodic"):
    """Backward difference D^- along ``axis`` (Sec. 3)."""
    return (u - _nbr(u, axis, -1, bc)) / h[axis]


def second_diff(u, h, axis, bc="periodic"):
    """Three-point second difference D^<2> along ``axis`` (Sec. 3)."""
    return (_nbr(u, axis, 1, bc) - 2.0 * u + _nbr(u, axis, -1, bc)) / h[axis] ** 2


def lap(u, h, bc="periodic"):
    """Discrete Laplacian Delta_d = sum over axes of D^<2> (Sec. 3)."""
    out = np.zeros_like(u)
    for a in range(u.ndim):
        out = out + second_diff(u, h, a, bc)
    return out


def div_mobility_grad(g, m_node, h, bc="periodic"):
    """Discrete nabla_d . M nabla_d g (Sec. 3).

    D_a M D_a g at i = [M_{i+1/2} (g_{i+1} - g_i) - M_{i-1/2} (g_i - g_{i-1})] / h_a^2,
    with the edge mobility the mean of the two node values.  With M = 1 this is
    ``lap``.  Under the Neumann-type conditions the mirror ghost makes the boundary face's
    difference, hence its flux, zero.
    """
    out = np.zeros_like(g)
    for a in range(g.ndim):
        m_e = 0.5 * (m_node + _nbr(m_node, a, 1, bc))      # M at i+1/2
        flux = m_e * (_nbr(g, a, 1, bc) - g)                # M_{i+1/2}(g_{i+1}-g_i)
        prev = _nbr(flux, a, -1, "periodic")                # flux at i-1/2 ...
        if bc == "neumann":                                 # ... zero at the first face
            sl = [slice(None)] * g.ndim
            sl[a] = 0
            prev[tuple(sl)] = 0.0
        out = out + (flux - prev) / h[a] ** 2
    return out


# ---------------------------------------------------------------------------
# Discrete energy and mass (Sec. 3, Eqs. (7)-(8); mass conservation)
# ---------------------------------------------------------------------------

def local_energy(phi, gamma, h, bc="periodic"):
    """Discrete local energy G_d of Eq. (7), cell by cell."""
    g = 0.5 * (1.0 - gamma) * phi ** 2 + 0.25 * phi ** 4 + 0.5 * lap(phi, h, bc) ** 2
    for a in range(phi.ndim):
        g = g - 0.5 * (d_plus(phi, h, a, bc) ** 2 + d_minus(phi, h, a, bc) ** 2)
    return g


def cell_volume(h):
    return float(np.prod(h))


def free_energy(phi, gamma, h, bc="periodic"):
    """Discrete free energy F_d of Eq. (8): sum of G_d times the cell volume."""
    return float(np.sum(local_energy(phi, gamma, h, bc)) * cell_volume(h))


def mass(phi, h):
    """Discrete mass sum(phi) * cell volume (conserved by the scheme, Sec. 3)."""
    return float(np.sum(phi) * cell_volume(h))


# ---------------------------------------------------------------------------
# Discrete variational derivative and the semi-implicit scheme (Eqs. (11)-(12))
# ---------------------------------------------------------------------------

def dvd_derivative(Phi, phi, gamma, h, bc="periodic"):
    """Discrete variational derivative mu_d of Eq. (11).

    mu_d = [(1 - gamma) + 2 Delta_d + Delta_d^2] ((Phi + phi)/2)
           + (Phi^3 + Phi^2 phi + Phi phi^2 + phi^3) / 4,
    where Phi is the new level phi^(n+1) and phi the old level phi^(n).
    """
    u = 0.5 * (Phi + phi)
    lu = lap(u, h, bc)
    linear = (1.0 - gamma) * u + 2.0 * lu + lap(lu, h, bc)
    cubic = (Phi ** 3 + Phi ** 2 * phi + Phi * phi ** 2 + phi ** 3) / 4.0
    return linear + cubic


def mobility_one_minus_sq(u):
    """Variable mobility M(u) = 1 - u^2 (Sec. 5, test B variants)."""
    return 1.0 - u * u


mobility_one_minus_sq.derivative = lambda u: -2.0 * u      # M'(u)


def residual(Phi, phi, dt, gamma, h, mobility=None, src=None, bc="periodic"):
    """Residual of the semi-implicit scheme, Eq. (12), as the system of Eq. (17).

    F(Phi) = (Phi - phi)/dt - nabla_d . M_d nabla_d mu_d(Phi, phi)  [- src]

    with M_d = M((Phi + phi)/2) (Eq. (12)); ``mobility=None`` means M = 1.
    ``src`` is an optional already time-averaged source term (used only by the
    manufactured-solution tests).
    """
    mu = dvd_derivative(Phi, phi, gamma, h, bc)
    if mobility is None:
        flux_div = lap(mu, h, bc)
    else:
        flux_div = div_mobility_grad(mu, mobility(0.5 * (Phi + phi)), h, bc)
    F = (Phi - phi) / dt - flux_div
    if src is not None:
        F = F - src
    return F


def jacobian_coef(Phi, phi):
    """c = d/dPhi of the cubic part of Eq. (11): (3 Phi^2 + 2 Phi phi + phi^2)/4."""
    return (3.0 * Phi ** 2 + 2.0 * Phi * phi + phi ** 2) / 4.0


def jv(Phi, phi, dt, gamma, h, v, mobility=None, bc="periodic"):
    """Matrix-free Jacobian action J v, J = dF/dPhi (Sec. 4, Eq. (19)).

    M = 1: J v = v/dt - Delta_d[ (1-gamma)/2 v + Delta_d v + 1/2 Delta_d^2 v + c v ].
    Variable M (evaluated at u = (Phi + phi)/2): with w the bracket above,
    J v = v/dt - nabla_d . M nabla_d w - nabla_d . (M'(u) v / 2) nabla_d mu_d,
    the second term from the mobility's dependence on Phi (the edge values are means of the
    node values, so their derivative is the mean of the node derivatives).
    """
    c = jacobian_coef(Phi, phi)
    lv = lap(v, h, bc)
    inner = 0.5 * (1.0 - gamma) * v + lv + 0.5 * lap(lv, h, bc) + c * v
    if mobility is None:
        return v / dt - lap(inner, h, bc)
    u = 0.5 * (Phi + phi)
    mu = dvd_derivative(Phi, phi, gamma, h, bc)
    return (v / dt - div_mobility_grad(inner, mobility(u), h, bc)
            - div_mobility_grad(mu, 0.5 * mobility.derivative(u) * v, h, bc))


# ---------------------------------------------------------------------------
# Assembled operators
# ---------------------------------------------------------------------------

def shift_matrix(n, s, bc="periodic"):
    """1-D matrix of u -> u_(i+s), s = +-1: periodic wrap or the Neumann mirror ghost."""
    i = np.arange(n)
    j = (i + s) % n if bc == "periodic" else np.clip(i + s, 0, n - 1)
    return sp.coo_matrix((np.ones(n), (i, j)), shape=(n, n)).tocsr()


def periodic_second_diff_matrix(n, bc="periodic"):
    """1-D second-difference matrix (unscaled), duplicates summed (``bc`` as ``_nbr``)."""
    return (shift_matrix(n, 1, bc) + shift_matrix(n, -1, bc) - 2.0 * sp.identity(n, format="csr")).tocsr()


def _axis_op(shape, a, op):
    """The 1-D operator ``op`` acting along array axis ``a`` of the C-order flattening."""
    out = None
    for b in range(len(shape)):
        blk = op if a == b else sp.identity(shape[b], format="csr")
        out = blk if out is None else sp.kron(out, blk, format="csr")
    return out


def laplacian_matrix(shape, h, bc="periodic"):
    """Delta_d as a sparse matrix on the C-order flattening of ``shape``."""
    mats = None
    for a in range(len(shape)):
        term = _axis_op(shape, a, periodic_second_diff_matrix(shape[a], bc) / h[a] ** 2)
        mats = term if mats is None else mats + term
    return mats.tocsr()


def _face_ops(n, bc):
    """1-D face operators of nabla_d . M nabla_d: the difference g_(i+1) - g_i at face i+1/2,
    the face mean (m_i + m_(i+1))/2, and the divergence f_(i+1/2) - f_(i-1/2).  Under the
    Neumann-type conditions the last face's difference is zero and the divergence takes no
    flux through the first face (the mirror ghost)."""
    I = sp.identity(n, format="csr")
    Sp = shift_matrix(n, 1, bc)
    D = (Sp - I).tocsr()
    E = (0.5 * (Sp + I)).tocsr()
    if bc == "periodic":
        B = (I - shift_matrix(n, -1, bc)).tocsr()
    else:
        i = np.arange(n)
        B = sp.coo_matrix((np.concatenate([np.ones(n), -np.ones(n - 1)]),
                           (np.concatenate([i, i[1:]]), np.concatenate([i, i[:-1]]))), shape=(n, n)).tocsr()
    return D, E, B


def jacobian_csr(Phi, phi, dt, gamma, h, mobility=None, bc="periodic"):
    """Exact Jacobian of ``residual`` as a CSR matrix (Sec. 4, Eq. (19); with a variable
    mobility the terms of ``jv``)."""
    n = Phi.size
    L = laplacian_matrix(Phi.shape, h, bc)
    I = sp.identity(n, format="csr")
    c = sp.diags(jacobian_coef(Phi, phi).ravel())
    inner = 0.5 * (1.0 - gamma) * I + L + 0.5 * (L @ L) + c
    if mobility is None:
        return (I / dt - L @ inner).tocsr()
    u = 0.5 * (Phi + phi)
    m = mobility(u).ravel()
    dm = sp.diags(0.5 * mobility.derivative(u).ravel())
    mu = dvd_derivative(Phi, phi, gamma, h, bc).ravel()
    J = I / dt
    for a in range(Phi.ndim):
        D1, E1, B1 = _face_ops(Phi.shape[a], bc)
        D, E, B = (_axis_op(Phi.shape, a, op) for op in (D1, E1, B1))
        B = B / h[a] ** 2
        J = J - B @ sp.diags(E @ m) @ D @ inner - B @ sp.diags(D @ mu) @ E @ dm
    return J.tocsr()


def jacobian_symbol(shape, h, dt, gamma, cbar):
    """Fourier symbol of the Jacobian at a uniform coefficient c = cbar.

    Delta_d has symbol -kappa, kappa = sum_a (4/h_a^2) sin^2(pi k_a / N_a); hence
    J has symbol 1/dt + kappa [ (1-gamma)/2 - kappa + kappa^2/2 + cbar ].
    Returned on the real-FFT half spectrum.
    """
    kap = 0.0
    nd = len(shape)
    for a in range(nd):
        n = shape[a]
        k = np.arange(n // 2 + 1) if a == nd - 1 else np.arange(n)
        lam = (4.0 / h[a] ** 2) * np.sin(np.pi * k / n) ** 2
        sh = [1] * nd
        sh[a] = lam.size
        kap = kap + lam.reshape(sh)
    return 1.0 / dt + kap * (0.5 * (1.0 - gamma) - kap + 0.5 * kap ** 2 + cbar)


# ---------------------------------------------------------------------------
# Newton's method with an exact inner solve (Sec. 4, Eqs. (17)-(20))
# ---------------------------------------------------------------------------

ARMIJO = 1e-4          # sufficient-decrease constant of the backtracking line search
LAMBDA_MIN = 2.0 ** -10


@dataclass
class NewtonResult:
    Phi: np.ndarray
    iterations: int
    res_norms: list = field(default_factory=list)
    converged: bool = True


def _solve_direct(J, rhs):
    return spla.splu(J.tocsc()).solve(rhs)


def _solve_fft_gmres(J, rhs, shape, h, dt, gamma, cbar, workers=-1):
    """GMRES to 1e-14 on J x = rhs, preconditioned by the uniform-c symbol inverse."""
    sym = jacobian_symbol(shape, h, dt, gamma, cbar)
    tiny = 1e-3 / dt
    sym = np.where(np.abs(sym) < tiny, np.copysign(tiny, sym), sym)

    def prec(r):
        R = scipy.fft.rfftn(r.reshape(shape), workers=workers)
        return scipy.fft.irfftn(R / sym, s=shape, workers=workers).ravel()

    n = rhs.size
    A = spla.LinearOperator((n, n), matvec=lambda x: J @ x, dtype=np.float64)
    M = spla.LinearOperator((n, n), matvec=prec, dtype=np.float64)
    x, info = spla.gmres(A, rhs, M=M, rtol=1e-14, atol=0.0, restart=60, maxiter=40)
    # the direction must be the exact one to rounding: the true residual must reach 1e-12 of
    # the right-hand side, or the rounding level of the product J x itself (eps || |J| |x| ||,
    # which binds at large dt) when that level is below 1e-8 of the right-hand side, whatever
    # GMRES reports; an unconverged solve is never returned
    bn = float(np.linalg.norm(rhs))
    res = float(np.linalg.norm(rhs - J @ x))
    floor = np.finfo(np.float64).eps * float(np.linalg.norm(abs(J) @ np.abs(x)))
    floor = floor if floor <= 1e-8 * bn else 0.0
    if info < 0 or not np.isfinite(res) or res > max(1e-12 * bn, floor):
        raise RuntimeError(f"FFT-preconditioned GMRES did not converge (info {info}, residual {res:.3e} "
                           f"of {bn:.3e}, rounding level {floor:.3e})")
    return x


def newton_solve(phi_n, dt, gamma, h, guess=None, src=None, linear="auto",
                 maxit=30, step_floor=1e-14, mobility=None, bc="periodic"):
    """Root of F(Phi) = 0 by Newton's method with backtracking (Eqs. (18)-(19)).

    The initial iterate is the previous solution phi_n (Sec. 4) unless ``guess``
    is given.  Each direction solves J S = -F exactly (SuperLU), or, for grids
    above 256^2 cells, by GMRES to 1e-14 with an FFT preconditioner.  The step
    length halves from 1 while ||F(Phi + lam S)|| > (1 - 1e-4 lam) ||F(Phi)||.
    The oracle iterates to the floating-point floor: it stops when the Newton
    step is below 1e-14 max(1, |Phi|_inf) or when no decrease is possible.
    """
    Phi = (phi_n if guess is None else guess).astype(np.float64).copy()
    shape = Phi.shape
    general = mobility is not None or bc != "periodic"
    if linear == "auto":
        linear = "direct" if Phi.size <= 256 * 256 or general else "fftgmres"
    if general and linear != "direct":
        raise ValueError("the FFT preconditioner is built for periodic grids with M = 1")
    F = residual(Phi, phi_n, dt, gamma, h, src=src, mobility=mobility, bc=bc)
    norms = [float(np.linalg.norm(F))]
    it = 0
    for it in range(1, maxit + 1):
        J = jacobian_csr(Phi, phi_n, dt, gamma, h, mobility=mobility, bc=bc)
        if linear == "direct":
            S = -_solve_direct(J, F.ravel())
        else:
            cbar = float(np.mean(jacobian_coef(Phi, phi_n)))
            S = -_solve_fft_gmres(J, F.ravel(), shape, h, dt, gamma, cbar)
        S = S.reshape(shape)
        if np.max(np.abs(S)) <= step_floor * max(1.0, float(np.max(np.abs(Phi)))):
            Phi = Phi + S
            F = residual(Phi, phi_n, dt, gamma, h, src=src, mobility=mobility, bc=bc)
            norms.append(float(np.linalg.norm(F)))
            break
        fn = norms[-1]
        lam = 1.0
        accepted = False
        while True:
            trial = Phi + lam * S
            Ft = residual(trial, phi_n, dt, gamma, h, src=src, mobility=mobility, bc=bc)
            ftn = float(np.linalg.norm(Ft))
            if ftn <= (1.0 - ARMIJO * lam) * fn:
                accepted = True
                break
            if lam <= LAMBDA_MIN:
                break
            lam *= 0.5
        if not accepted:
            break                       # rounding floor reached
        Phi, F = trial, Ft
        norms.append(ftn)
    return NewtonResult(Phi=Phi, iterations=it, res_norms=norms,
                        converged=norms[-1] <= 1e-9 * max(1.0, norms[0]) or norms[-1] < 1e-11)


# ---------------------------------------------------------------------------
# Adaptive time step (Sec. 3, Eq. (16)) and the time loop
# ---------------------------------------------------------------------------

def adaptive_dt(F_n, F_nm1, dt_nm1, dt_min, dt_max, eta):
    """dt_n = max(dt_min, dt_max / sqrt(1 + eta |F'|^2)), |F'| = |F^n - F^(n-1)| / dt_(n-1)."""
    fprime = abs(F_n - F_nm1) / dt_nm1
    return max(dt_min, dt_max / math.sqrt(1.0 + eta * fprime * fprime))


@dataclass
class Trajectory:
    phis: list
    dts: list
    energies: list
    masses: list
    newton_its: list


def run(phi0, nsteps, gamma, h, dt_min, dt_max, eta=0.0, linear="auto", keep_all=True, mobility=None,
        bc="periodic"):
    """Advance ``nsteps`` steps; dt_0 = dt_min, then Eq. (16) from the energy history."""
    phi = phi0.astype(np.float64).copy()
    phis = [phi.copy()]
    energies = [free_energy(phi, gamma, h, bc)]
    masses = [mass(phi, h)]
    dts, its = [], []
    for n in range(nsteps):
        if n == 0 or dt_min == dt_max:
            dt = dt_min
        else:
            dt = adaptive_dt(energies[n], energies[n - 1], dts[n - 1], dt_min, dt_max, eta)
        res = newton_solve(phi, dt, gamma, h, linear=linear, mobility=mobility, bc=bc)
        phi = res.Phi
        dts.append(dt)
        its.append(res.iterations)
        energies.append(free_energy(phi, gamma, h, bc))
        masses.append(mass(phi, h))
        if keep_all:
            phis.append(phi.copy())
        else:
            phis = [phi.copy()]
    return Trajectory(phis=phis, dts=dts, energies=energies, masses=masses, newton_its=its)


def rel_l2(a, b):
    """Relative l2 error of Sec. 5, Eq. (27): ||a - b|| / ||b||."""
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
