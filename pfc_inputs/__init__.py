"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module only builds initial fields and workload descriptions; it holds none
of the scheme's arithmetic, and it imports neither ``oracle`` nor the HIP
package.  Every random draw is seeded (numpy PCG64).

Initial conditions follow the paper's experiments (Sec. 5):
* ``noise_ic``          uniform noise about a mean density (test A, and the
                        small / 3-D / batched workloads);
* ``hex_crystallites_ic``  hexagonal crystallites in a liquid (test B, Eqs. (29)-(30));
* ``smooth_ic``         the smooth sine product used for the accuracy study (Eq. (28));
* ``bcc_spheres_ic``    BCC crystallite spheres in 3-D (test D, Eqs. (32)-(34));
* ``crack_ic``          the notched, stretched hexagonal lattice of the crack test (test C),
                        on the periodic system ``crack_lengths`` gives.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def cell_centres(n, L):
    """Cell-centred coordinates (i + 1/2) * L / n, i = 0..n-1 (Sec. 3)."""
    return (np.arange(n) + 0.5) * (L / n)


def crack_periods(nx=4096, ny=1024):
    """Lattice periods of test C's periodic system: the most whole periods (2 pi / q_x along x,
    2 pi sqrt(3) / q_y along y) that fit in 4096 pi/3 x 1024 pi/3, scaled with the mesh:
    591 x 76 at 4096 x 1024."""
    qx = math.sqrt(3) / 2
    qy = 0.9 * qx
    px, py = 2 * math.pi / qx, 2 * math.pi * math.sqrt(3) / qy
    return math.floor(4096 * math.pi / 3 * nx / 4096 / px), math.floor(1024 * math.pi / 3 * ny / 1024 / py)


def crack_lengths(nx=4096, ny=1024):
    """(L_y, L_x) of test C's domain: the periodic system itself (crack_periods periods)."""
    qx = math.sqrt(3) / 2
    qy = 0.9 * qx
    mx, my = crack_periods(nx, ny)
    return my * 2 * math.pi * math.sqrt(3) / qy, mx * 2 * math.pi / qx


def crack_ic(nx=4096, ny=1024, notch=(40, 20), liquid=0.79):
    """Stretched hexagonal lattice with a liquid notch (test C, Sec. 5).

    The domain is the periodic system of whole lattice periods that fits in 4096 pi/3 x
    1024 pi/3 (crack_lengths; 591 x 76 periods at the full size, scaled with nx, ny), on an
    nx x ny mesh; lattice 0.49 + cos(q_y y / sqrt 3) cos(q_x x) - 0.5 cos(2 q_y y / sqrt 3) with
    q_x = sqrt(3)/2, q_y = 0.9 q_x over all of it; a notch of notch[0] x notch[1] cells at the
    centre holds the coexisting liquid.  Array axes are (y, x)."""
    Ly, Lx = crack_lengths(nx, ny)
    qx = math.sqrt(3) / 2
    qy = 0.9 * qx
    x, y = cell_centres(nx, Lx), cell_centres(ny, Ly)
    X, Y = np.meshgrid(x, y, indexing="xy")
    phi = 0.49 + np.cos(qy * Y / math.sqrt(3)) * np.cos(qx * X) - 0.5 * np.cos(2 * qy * Y / math.sqrt(3))
    cx, cy = nx // 2, ny // 2
    phi[cy - notch[1] // 2: cy + notch[1] // 2, cx - notch[0] // 2: cx + notch[0] // 2] = liquid
    return phi


def noise_ic(shape, mean, amp, seed):
    """phi = mean + sigma, sigma ~ U(-amp, amp) i.i.d. per cell (seeded)."""
    return mean + rng(seed).uniform(-amp, amp, size=tuple(shape))


def smooth_ic(n, L=32.0):
    """0.5 sin(2 pi x / 32) sin(2 pi y / 32) on [0, L]^2 (Sec. 5, Eq. (28))."""
    x = cell_centres(n, L)
    X, Y = np.meshgrid(x, x, indexing="xy")        # array axes (y, x)
    return 0.5 * np.sin(2 * np.pi * X / 32.0) * np.sin(2 * np.pi * Y / 32.0)


def _periodic_delta(a, b, L):
    d = a - b
    return d - L * np.round(d / L)


def hex_crystallites_ic(n=1024, L=400.0, phibar=-0.285, amp=0.446, q=0.66,
                        radius_cells=10, angles=(-math.pi / 4, 0.0, math.pi / 4),
                        seed=1, min_sep_cells=40, sign=-1.0):
    """Liquid of density ``phibar`` with hexagonal crystallites in disks (test B).

    Inside each disk the density is phibar + sign * amp * [cos(q y~/sqrt3) cos(q x~)
    - cos(2 q y~/sqrt3)/2] (Eq. (29) with q_x = q_y = q), where (x~, y~) are the
    coordinates relative to the disk centre rotated by the crystallite's angle
    (Eq. (30)).  The energy is even in phi, so ``sign=-1`` with a negative mean is
    the mirror image of the paper's positive-mean set-up.  Centres are drawn
    uniformly (seeded) with a minimum periodic separation.
    """
    h = L / n
    x = cell_centres(n, L)
    X, Y = np.meshgrid(x, x, indexing="xy")
    phi = np.full((n, n), phibar, dtype=np.float64)
    g = rng(seed)
    centres = []
    tries = 0
    while len(centres) < len(angles):
        c = g.uniform(0.0, L, size=2)
        tries += 1
        ok = all(math.hypot(_periodic_delta(c[0], o[0], L), _periodic_delta(c[1], o[1], L))
                 >= min_sep_cells * h for o in centres)
        if ok or tries > 10000:
            centres.append(c)
    R = radius_cells * h
    for (cx, cy), w in zip(centres, angles):
        dx = _periodic_delta(X, cx, L)
        dy = _periodic_delta(Y, cy, L)
        inside = dx * dx + dy * dy <= R * R
        xt = math.cos(w) * dx - math.sin(w) * dy
        yt = math.sin(w) * dx + math.cos(w) * dy
        lattice = (np.cos(q * yt / math.sqrt(3.0)) * np.cos(q * xt)
                   - 0.5 * np.cos(2.0 * q * yt / math.sqrt(3.0)))
        phi = np.where(inside, phibar + sign * amp * lattice, phi)
    return phi


def bcc_spheres_ic(n=128, L=40 * math.pi, phibar=-0.35, amp=1.0, q=1 / math.sqrt(2),
                   d0=None, angles=(0.0, -math.pi / 8, math.pi / 8)):
    """Three BCC crystallite spheres in a liquid (test D, Eqs. (32)-(34)).

    Spheres of radius d0 (default L/16, i.e. 5 pi at L = 80 pi) centred at
    (L/2, 3L/4, L/2), (L/4, L/4, L/2), (3L/4, L/4, L/2); each is rotated about z
    by its angle; the envelope is (1 - (r/d0)^2)^2 inside the sphere.
    Array axes are (z, y, x).
    """
    if d0 is None:
        d0 = L / 16.0
    c = cell_centres(n, L)
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    phi = np.full((n, n, n), phibar, dtype=np.float64)
    centres = [(L / 2, 3 * L / 4, L / 2), (L / 4, L / 4, L / 2), (3 * L / 4, L / 4, L / 2)]
    for (x0, y0, z0), w in zip(centres, angles):
        dx, dy, dz = X - x0, Y - y0, Z - z0
        r = np.sqrt(dx * dx + dy * dy + dz * dz)
        rho = np.where(r <= d0, (1.0 - (r / d0) ** 2) ** 2, 0.0)
        xt = math.cos(w) * dx - math.sin(w) * dy
        yt = math.sin(w) * dx + math.cos(w) * dy
        zt = dz
        bcc = (np.cos(q * xt) * np.cos(q * yt) + np.cos(q * xt) * np.cos(q * zt)
               + np.cos(q * yt) * np.cos(q * zt))
        phi = phi + amp * rho * bcc
    return phi


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    shape: tuple            # array shape, (ny, nx) or (nz, ny, nx)
    lengths: tuple          # domain lengths per array axis
    gamma: float
    dt_min: float
    dt_max: float
    eta: float
    nsteps: int
    sub: tuple              # subdomains per array axis
    overlap: int            # overlap in mesh layers
    newton_rtol: float = 1e-8
    newton_atol: float = 1e-10
    lin_rtol: float = 1e-3
    lin_atol: float = 1e-11
    ic: dict = field(default_factory=dict)
    mobility: str = "1"             # "1" or "1-phi^2"
    boundary: str = "periodic"      # "periodic" or "neumann"

    def initial(self):
        kind = self.ic["kind"]
        if kind == "noise":
            return noise_ic(self.shape, self.ic["mean"], self.ic["amp"], self.ic["seed"])
        if kind == "hex":
            return hex_crystallites_ic(n=self.shape[-1], L=self.lengths[-1],
                                       phibar=self.ic["mean"], seed=self.ic["seed"])
        if kind == "bcc":
            return bcc_spheres_ic(n=self.shape[-1], L=self.lengths[-1])
        if kind == "smooth":
            return smooth_ic(self.shape[-1], self.lengths[-1])
        if kind == "crack":
            return crack_ic(nx=self.shape[-1], ny=self.shape[-2])
        raise ValueError(kind)


def small_noise_64():
    """64^2 on [0, 32 pi]^2, gamma 0.25, mean -0.285 + U(+-0.05), 10 steps of 0.1, 4x4 subdomains, overlap 2."""
    L = 32 * math.pi
    return Workload("pfc2d_64_noise", (64, 64), (L, L), 0.25, 0.1, 0.1, 0.0, 10, (4, 4), 2,
                    newton_rtol=0.0, newton_atol=1e-10,
                    ic=dict(kind="noise", mean=-0.285, amp=0.05, seed=0))


def crystal_growth_1024():
    """1024^2 on [0, 400]^2, gamma 0.25, mean -0.285, 3 hex crystallites, 200 adaptive steps."""
    return Workload("pfc2d_1024_crystal", (1024, 1024), (400.0, 400.0), 0.25, 1e-2, 10.0, 5000.0,
                    200, (16, 16), 4, ic=dict(kind="hex", mean=-0.285, seed=1))


def crystal_growth(n, sub, overlap=4, nsteps=200, seed=1):
    """Test-B physics at mesh size 400/1024 on an n^2 grid."""
    L = 400.0 * n / 1024.0
    return Workload(f"pfc2d_{n}_crystal", (n, n), (L, L), 0.25, 1e-2, 10.0, 5000.0, nsteps,
                    tuple(sub), overlap, ic=dict(kind="hex", mean=-0.285, seed=seed))


def test_b_variants(n=1024, nsteps=200):
    """Test B's four variants (Sec. 5): the crystal-growth field on an n^2 grid of mesh size
    400/1024 with (a) periodic boundaries, M = 1; (b) Neumann-type boundaries, M = 1;
    (c) periodic, M = 1 - phi^2; (d) Neumann-type, M = 1 - phi^2."""
    out = []
    for tag, mob, bc in (("a", "1", "periodic"), ("b", "1", "neumann"), ("c", "1-phi^2", "periodic"),
                         ("d", "1-phi^2", "neumann")):
        w = crystal_growth(n, (16, 64), overlap=4, nsteps=nsteps)
        w.name = f"pfc2d_{n}_crystal_{tag}"
        w.mobility, w.boundary = mob, bc
        out.append(w)
    return out


def crack_4096x1024():
    """Test C: 4096 x 1024 mesh on the periodic system of 591 x 76 lattice periods (about
    4096 pi/3 x 1024 pi/3), gamma 1, the notched lattice, adaptive dt 1..5 (eta 100), 16 x 64
    boxes (64 x 64 owned), overlap 3 (delta = 1)."""
    return Workload("pfc2d_crack_4096x1024", (1024, 4096), crack_lengths(4096, 1024), 1.0, 1.0, 5.0,
                    100.0, 200, (16, 64), 3, ic=dict(kind="crack"))


def noise_3d_128():
    """128^3 on [0, 40 pi]^3, gamma 0.56, mean -0.2 + U(+-0.1), 50 adaptive steps, 8^3 subdomains, overlap 2."""
    L = 40 * math.pi
    return Workload("pfc3d_128_noise", (128, 128, 128), (L, L, L), 0.56, 0.1, 10.0, 500.0, 50,
                    (8, 8, 8), 2, ic=dict(kind="noise", mean=-0.2, amp=0.1, seed=2))


def bcc_growth_3d_256(dt_min=0.1, dt_max=0.1):
    """Test D's grid: 256^3 on [0, 80 pi]^3, gamma 0.35, three BCC crystallite spheres (mean -0.35,
    radius 5 pi), 16^3 subdomains (16^3 owned cells), overlap 3 (delta = 1), eta 500.  The paper
    runs dt 0.5..10 here; the default is the dt = 0.1 of its test-D tuning runs, the range where
    natural-order ILU(0) on this mesh size stays stable (it breaks down from dt ~ 0.3 on)."""
    L = 80 * math.pi
    return Workload("pfc3d_bcc_256", (256, 256, 256), (L, L, L), 0.35, dt_min, dt_max, 500.0, 50,
                    (16, 16, 16), 3, ic=dict(kind="bcc"))


def batch_instances(count=64, seed=3):
    """Ragged batch: side ~ U{128,192,256,384,512}, gamma ~ U[0.1,0.4], mean ~ U[-0.35,-0.2]."""
    g = rng(seed)
    sides = g.choice([128, 192, 256, 384, 512], size=count)
    gammas = g.uniform(0.1, 0.4, size=count)
    means = g.uniform(-0.35, -0.2, size=count)
    out = []
    for i in range(count):
        n = int(sides[i])
        L = n * math.pi / 2
        out.append(Workload(f"inst{i}", (n, n), (L, L), float(gammas[i]), 1e-2, 10.0, 5000.0, 1,
                            (max(2, n // 64), max(2, n // 64)), 4,
                            ic=dict(kind="noise", mean=float(means[i]), amp=0.05, seed=3000 + i)))
    return out
