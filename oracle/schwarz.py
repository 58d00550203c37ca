"""FP64 reference routines for the Krylov-Schwarz part of the solve (Sec. 4).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

These pieces are approximations (a preconditioner, an incomplete factorisation,
a Krylov iteration), so the oracle takes their steps in the paper's order and
notation rather than a closed form:

* the overlapping decomposition: non-overlapping boxes Omega_k, each extended by
  ``overlap`` mesh layers on every side with periodic wrap (Sec. 4; the paper's
  overlap parameter delta counts 3 layers, so its delta corresponds to
  ``overlap = 3 * delta``);
* the subdomain matrix A_k = R_k J R_k^T (Eq. (25)), which equals the
  discretisation of the subdomain problem with phi = 0 on the three-layer ring
  around the extended box (Eq. (26));
* classical AS (Eq. (22)), left-RAS (Eq. (23)) and right-RAS (Eq. (24));
* subdomain solves by sparse LU or by ILU(0), written as the textbook IKJ loop
  (Saad, Iterative Methods for Sparse Linear Systems, Alg. 10.4) on the
  structural stencil pattern;
* right-preconditioned flexible GMRES with modified Gram-Schmidt and Givens
  rotations (Saad and Schultz), stopped by the linear test of Sec. 4.

Pure-Python loops (ILU(0)) are meant for small subdomains.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


# ---------------------------------------------------------------------------
# Decomposition
# ---------------------------------------------------------------------------

@dataclass
class Subdomain:
    owned_lo: tuple     # first owned index per axis
    owned_n: tuple      # owned extent per axis
    overlap: int
    shape: tuple        # global grid shape

    @property
    def ext_n(self):
        return tuple(n + 2 * self.overlap for n in self.owned_n)

    def ext_axis_indices(self, a):
        lo = self.owned_lo[a] - self.overlap
        return (lo + np.arange(self.ext_n[a])) % self.shape[a]

    def ext_global_indices(self):
        """Global flat indices of the extended box, in the box's natural order."""
        axes = [self.ext_axis_indices(a) for a in range(len(self.shape))]
        grids = np.meshgrid(*axes, indexing="ij")
        return np.ravel_multi_index(tuple(g.ravel() for g in grids), self.shape)

    def owned_mask_local(self):
        """Boolean mask over the extended box that marks Omega_k itself."""
        m = np.zeros(self.ext_n, dtype=bool)
        sl = tuple(slice(self.overlap, self.overlap + n) for n in self.owned_n)
        m[sl] = True
        return m.ravel()


def decompose(shape, sub, overlap):
    """Split each axis into ``sub[a]`` boxes starting at floor(k N / sub), extend by ``overlap``.

    Requirements (as the library's): at least 2 boxes per axis and an extended box
    no wider than N - 3 (so no cell of the box meets the box again through the
    periodic wrap within the stencil radius 3).
    """
    nd = len(shape)
    sub = tuple(sub)
    for a in range(nd):
        if sub[a] < 2:
            raise ValueError("need at least two subdomains per axis")
    starts = [[(k * shape[a]) // sub[a] for k in range(sub[a] + 1)] for a in range(nd)]
    out = []
    for idx in itertools.product(*[range(s) for s in sub]):
        lo = tuple(starts[a][idx[a]] for a in range(nd))
        n = tuple(starts[a][idx[a] + 1] - starts[a][idx[a]] for a in range(nd))
        d = Subdomain(lo, n, overlap, tuple(shape))
        for a in range(nd):
            if d.ext_n[a] > shape[a] - 3:
                raise ValueError("extended subdomain too wide for the periodic grid")
        out.append(d)
    return out


def stencil_offsets(nd, radius=3):
    """Offsets (per array axis) of the composite stencil: sum of |o_a| <= 3."""
    rng = range(-radius, radius + 1)
    return [o for o in itertools.product(*([rng] * nd)) if sum(abs(x) for x in o) <= radius]


def subdomain_pattern(ext_n):
    """Structural nonzero pattern of A_k: stencil couplings inside the box."""
    nd = len(ext_n)
    offs = stencil_offsets(nd)
    size = int(np.prod(ext_n))
    rows = []
    for p in range(size):
        coord = np.unravel_index(p, ext_n)
        cols = []
        for o in offs:
            q = tuple(coord[a] + o[a] for a in range(nd))
            if all(0 <= q[a] < ext_n[a] for a in range(nd)):
                cols.append(int(np.ravel_multi_index(q, ext_n)))
        rows.append(sorted(cols))
    return rows


def subdomain_matrix(J, dom):
    """A_k = R_k^delta J (R_k^delta)^T (Eq. (25)) as CSR."""
    idx = dom.ext_global_indices()
    return J[idx][:, idx].tocsr()


def subdomain_matrix_zero_ring(Phi, phi, dt, gamma, h, dom):
    """A_k built from the subdomain problem with phi = 0 on the 3-layer ring (Eq. (26)).

    Column j is the Jacobian action (Eq. (19) with the global coefficient c) on the
    j-th unit vector of the box, evaluated on the box padded by three zero layers
    and without any periodic wrap.
    """
    from .scheme import jacobian_coef
    ext = dom.ext_n
    nd = len(ext)
    pad = 3
    idx = dom.ext_global_indices()
    c_box = jacobian_coef(Phi, phi).ravel()[idx].reshape(ext)
    c_pad = np.pad(c_box, pad)

    def lap_local(u):
        out = np.zeros_like(u)
        for a in range(nd):
            up = np.zeros_like(u)
            dn = np.zeros_like(u)
            sl_hi = [slice(None)] * nd
            sl_lo = [slice(None)] * nd
            sl_hi[a] = slice(1, None)
            sl_lo[a] = slice(None, -1)
            up[tuple(sl_lo)] = u[tuple(sl_hi)]
            dn[tuple(sl_hi)] = u[tuple(sl_lo)]
            out += (up - 2.0 * u + dn) / h[a] ** 2
        return out

    size = int(np.prod(ext))
    A = np.zeros((size, size))
    inner = tuple(slice(pad, pad + n) for n in ext)
    for j in range(size):
        e = np.zeros(size)
        e[j] = 1.0
        v = np.pad(e.reshape(ext), pad)
        lv = lap_local(v)
        w = 0.5 * (1.0 - gamma) * v + lv + 0.5 * lap_local(lv) + c_pad * v
        jv = v / dt - lap_local(w)
        A[:, j] = jv[inner].ravel()
    return A


# ---------------------------------------------------------------------------
# ILU(0), textbook IKJ form
# ---------------------------------------------------------------------------

def ilu0(A, pattern):
    """ILU(0) of A on ``pattern`` (list of sorted column lists per row).

    IKJ variant: for i = 1..n-1, for k < i in the pattern of row i (increasing):
    a_ik <- a_ik / a_kk, then a_ij <- a_ij - a_ik a_kj for every j > k in the
    pattern of row i (a_kj is zero where (k, j) is outside the pattern).
    Returns the factored rows as dicts {col: value}: strictly lower part is L
    (unit diagonal implied), the rest is U.
    """
    A = sp.csr_matrix(A) if not isinstance(A, np.ndarray) else A
    n = len(pattern)
    rows = []
    for i in range(n):
        if isinstance(A, np.ndarray):
            rows.append({j: float(A[i, j]) for j in pattern[i]})
        else:
            r = A.getrow(i)
            d = dict(zip(r.indices.tolist(), r.data.tolist()))
            rows.append({j: float(d.get(j, 0.0)) for j in pattern[i]})
    for i in range(1, n):
        ri = rows[i]
        for k in pattern[i]:
            if k >= i:
                break
            ri[k] = ri[k] / rows[k][k]
            aik = ri[k]
            rk = rows[k]
            for j in pattern[i]:
                if j > k and j in rk:
                    ri[j] = ri[j] - aik * rk[j]
    return rows


# ---------------------------------------------------------------------------
# ILU(k): level-of-fill pattern (Saad, Iterative Methods for Sparse Linear Systems,
# Sec. 10.3.3), numeric factorisation by the same IKJ loop on that pattern
# ---------------------------------------------------------------------------

def iluk_levels(pattern, k):
    """Level of fill of every kept entry of ILU(k) for a matrix with structural ``pattern``.

    Entries of the matrix have level 0.  Eliminating row i in the IKJ order, each
    k' < i of row i whose level is at most k updates every j > k' of row k' and gives
    (i, j) the level min(lev(i, j), lev(i, k') + lev(k', j) + 1); entries whose level
    exceeds k are dropped when row i is done.  Returns one dict {col: level} per row.
    """
    n = len(pattern)
    rows = [dict.fromkeys(p, 0) for p in pattern]
    for i in range(n):
        rows[i][i] = 0
    for i in range(1, n):
        ri = rows[i]
        done = set()
        while True:                  # lower entries in increasing column order, fill included
            cand = [c for c in ri if c < i and c not in done and ri[c] <= k]
            if not cand:
                break
            kk = min(cand)
            done.add(kk)
            lik = ri[kk]
            for j, lkj in rows[kk].items():
                if j > kk:
                    lev = lik + lkj + 1
                    if lev <= k and lev < ri.get(j, k + 1):
                        ri[j] = lev
        rows[i] = {c: v for c, v in ri.items() if v <= k}
    return rows


def iluk_pattern(pattern, k):
    """Sorted column lists of the ILU(k) pattern (ILU(0): the matrix's own pattern)."""
    return [sorted(r) for r in iluk_levels(pattern, k)]


def iluk(A, pattern, k):
    """ILU(k) of A: the IKJ loop of ``ilu0`` on the level-k pattern."""
    return ilu0(A, iluk_pattern(pattern, k))


def ilu0_solve(rows, b):
    """Solve (L U) x = b with the factors of ``ilu0`` (forward, then backward)."""
    n = len(rows)
    y = np.array(b, dtype=np.float64).copy()
    for i in range(n):
        s = y[i]
        for j, v in rows[i].items():
            if j < i:
                s -= v * y[j]
        y[i] = s
    x = y.copy()
    for i in range(n - 1, -1, -1):
        s = x[i]
        for j, v in rows[i].items():
            if j > i:
                s -= v * x[j]
        x[i] = s / rows[i][i]
    return x


def ilu0_dense_factors(rows):
    """Dense L (unit lower) and U from ``ilu0`` rows (small sizes only)."""
    n = len(rows)
    L = np.eye(n)
    U = np.zeros((n, n))
    for i, r in enumerate(rows):
        for j, v in r.items():
            if j < i:
                L[i, j] = v
            else:
                U[i, j] = v
    return L, U


# ---------------------------------------------------------------------------
# Schwarz preconditioners (Eqs. (22)-(24))
# ---------------------------------------------------------------------------

class SubdomainSolver:
    """inv(A_k) by sparse LU ('lu'), ILU(0) ('ilu0') or ILU(k) ('ilu1', 'ilu2', ...)."""

    def __init__(self, A, kind, ext_n):
        self.kind = kind
        if kind == "lu":
            self.lu = spla.splu(sp.csc_matrix(A))
        elif kind == "ilu0":
            self.rows = ilu0(A, subdomain_pattern(ext_n))
        elif kind.startswith("ilu") and kind[3:].isdigit():
            self.rows = iluk(A, subdomain_pattern(ext_n), int(kind[3:]))
        else:
            raise ValueError(kind)

    def solve(self, b):
        if self.kind == "lu":
            return self.lu.solve(b)
        return ilu0_solve(self.rows, b)


def schwarz_setup(J, doms, kind="ilu0"):
    return [SubdomainSolver(subdomain_matrix(J, d), kind, d.ext_n) for d in doms]


def schwarz_apply(r, doms, solvers, variant="left"):
    """z = H^{-1} r for classical AS ('as'), left-RAS ('left') or right-RAS ('right').

    AS:        z = sum_k (R_k^d)^T inv(A_k) R_k^d r      (Eq. (22))
    left-RAS:  z = sum_k (R_k^0)^T inv(A_k) R_k^d r      (Eq. (23))
    right-RAS: z = sum_k (R_k^d)^T inv(A_k) R_k^0 r      (Eq. (24))
    """
    rf = np.asarray(r, dtype=np.float64).ravel()
    z = np.zeros_like(rf)
    for d, s in zip(doms, solvers):
        idx = d.ext_global_indices()
        own = d.owned_mask_local()
        rk = rf[idx].copy()
        if variant == "right":
            rk[~own] = 0.0
        yk = s.solve(rk)
        if variant == "left":
            z[idx[own]] = yk[own]
        else:
            np.add.at(z, idx, yk)
    return z.reshape(np.shape(r))


# ---------------------------------------------------------------------------
# Right-preconditioned flexible GMRES (Sec. 4, Eq. (21))
# ---------------------------------------------------------------------------

@dataclass
class GmresResult:
    x: np.ndarray
    iterations: int
    res_history: list
    V: np.ndarray
    H: np.ndarray


def fgmres(matvec, precond, b, rtol, atol, restart=30, maxit=300):
    """Solve A x = b, x0 = 0, right preconditioning, stop at ||r|| <= max(rtol ||b||, atol).

    Arnoldi with modified Gram-Schmidt on z_j = precond(v_j), w = A z_j; the
    least-squares problem is updated by Givens rotations, so the monitored value
    is the true residual norm of the unpreconditioned system in exact arithmetic.
    The update is x = sum_j y_j z_j (flexible form).  Returns the last cycle's
    basis for the Arnoldi-relation test.
    """
    b = np.asarray(b, dtype=np.float64).ravel()
    n = b.size
    x = np.zeros(n)
    bnorm = float(np.linalg.norm(b))
    target = max(rtol * bnorm, atol)
    hist = [bnorm]
    total = 0
    r = b.copy()
    V = H = None
    while True:
        beta = float(np.linalg.norm(r))
        if beta <= target or total >= maxit:
            break
        m = restart
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        j_done = 0
        for j in range(m):
            Z[j] = np.asarray(precond(V[j]), dtype=np.float64).ravel()
            w = np.asarray(matvec(Z[j]), dtype=np.float64).ravel()
            for i in range(j + 1):
                H[i, j] = float(np.dot(w, V[i]))
                w = w - H[i, j] * V[i]
            H[j + 1, j] = float(np.linalg.norm(w))
            if H[j + 1, j] > 0.0:
                V[j + 1] = w / H[j + 1, j]
            # apply previous rotations to column j, then form the new one
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            total += 1
            j_done = j + 1
            hist.append(abs(g[j + 1]))
            if abs(g[j + 1]) <= target or total >= maxit:
                break
        y = np.linalg.solve(np.triu(H[:j_done, :j_done]), g[:j_done])
        x = x + Z[:j_done].T @ y
        r = b - np.asarray(matvec(x), dtype=np.float64).ravel()
        if abs(g[j_done]) <= target or total >= maxit:
            break
    return GmresResult(x=x, iterations=total, res_history=hist, V=V, H=H)


def arnoldi_mgs(matvec, precond, b, m):
    """Plain Arnoldi (no rotations) for the relation A Z_m = V_{m+1} Hbar_m."""
    b = np.asarray(b, dtype=np.float64).ravel()
    n = b.size
    V = np.zeros((m + 1, n))
    Z = np.zeros((m, n))
    H = np.zeros((m + 1, m))
    V[0] = b / np.linalg.norm(b)
    for j in range(m):
        Z[j] = np.asarray(precond(V[j]), dtype=np.float64).ravel()
        w = np.asarray(matvec(Z[j]), dtype=np.float64).ravel()
        for i in range(j + 1):
            H[i, j] = float(np.dot(w, V[i]))
            w = w - H[i, j] * V[i]
        H[j + 1, j] = float(np.linalg.norm(w))
        V[j + 1] = w / H[j + 1, j]
    return V, Z, H


# ---------------------------------------------------------------------------
# The paper's inexact Newton-Krylov-Schwarz step (Sec. 4, Eqs. (17)-(24))
# ---------------------------------------------------------------------------

@dataclass
class NksResult:
    Phi: np.ndarray
    newton: int            # Newton iterations taken
    gmres: int             # FGMRES iterations over all of them
    res_norms: list        # ||F|| at Phi_0, Phi_1, ...


def nks_step(phi_n, dt, gamma, h, sub, overlap, kind="lu", variant="left", eps_r=1e-8, eps_a=1e-10,
             xi_r=1e-3, xi_a=1e-11, restart=30, maxit=300, newton_maxit=30):
    """One time step phi^n -> phi^(n+1) by the inexact Newton iteration of Sec. 4.

    Phi_0 = phi^n (Eq. (17)).  While ||F(Phi_m)|| > max(eps_r ||F(Phi_0)||, eps_a)
    (Eq. (20)), the correction solves J(Phi_m) S = -F(Phi_m) by right-preconditioned
    FGMRES from S = 0, stopped at max(xi_r ||F(Phi_m)||, xi_a) (Eq. (21)), with the
    Schwarz operator ``variant`` (classical AS 'as', left-RAS 'left', right-RAS 'right';
    Eqs. (22)-(24)).  The subdomain solvers are built from the Jacobian at Phi_0 and kept
    for the whole step (the reuse strategy of Table 1).  Phi_(m+1) = Phi_m + lam S with lam
    halved from 1 until ||F|| falls by the Armijo factor (Eq. (18)).  The defaults are the
    tolerances the paper lists for its experiments (Sec. 5).
    """
    from .scheme import ARMIJO, LAMBDA_MIN, jacobian_csr, residual

    Phi = np.asarray(phi_n, dtype=np.float64).copy()
    shape = Phi.shape
    doms = decompose(shape, sub, overlap)
    F = residual(Phi, phi_n, dt, gamma, h)
    norms = [float(np.linalg.norm(F))]
    target = max(eps_r * norms[0], eps_a)
    solvers = schwarz_setup(jacobian_csr(Phi, phi_n, dt, gamma, h), doms, kind)
    newton = gmres = 0
    while norms[-1] > target and newton < newton_maxit:
        J = jacobian_csr(Phi, phi_n, dt, gamma, h)
        res = fgmres(lambda v: J @ v, lambda r: schwarz_apply(r, doms, solvers, variant), -F.ravel(),
                     xi_r, xi_a, restart=restart, maxit=maxit)
        gmres += res.iterations
        S = res.x.reshape(shape)
        fn, lam = norms[-1], 1.0
        while True:
            trial = Phi + lam * S
            Ft = residual(trial, phi_n, dt, gamma, h)
            ftn = float(np.linalg.norm(Ft))
            if ftn <= (1.0 - ARMIJO * lam) * fn:
                break
            if lam <= LAMBDA_MIN:
                raise RuntimeError("line search failed")
            lam *= 0.5
        Phi, F = trial, Ft
        norms.append(ftn)
        newton += 1
    return NksResult(Phi=Phi, newton=newton, gmres=gmres, res_norms=norms)
