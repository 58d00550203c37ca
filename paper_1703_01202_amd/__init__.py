"""MI355X (gfx950) Newton-Krylov-Schwarz solver for the energy-stable PFC scheme.

Python face of ``libpfc.so``: the ``Solver`` methods map one to one onto the C entry
points of ``include/pfc.h`` (``pfc_residual``, ``pfc_jv``, ``pfc_ras_setup``,
``pfc_ras_apply``, ``pfc_energy``, ``pfc_gmres``, ``pfc_newton``, ``pfc_step``).
Fields are torch float64 tensors on the GPU with the array layout (ny, nx) or
(nz, ny, nx); every computation runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes

from . import _lib
from ._lib import PfcError, PfcStepStats

__all__ = ["Solver", "GuessNet", "Batch", "PfcError", "PfcStepStats", "load"]

load = _lib.load


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _structs(lib, shape, lengths, gamma, sub, overlap, sub_solver="ilu0", precond_fp32=False, dt_min=0.1,
             dt_max=None, eta=0.0, newton_rtol=1e-8, newton_atol=1e-10, lin_rtol=1e-3, lin_atol=1e-11,
             gmres_restart=30, gmres_maxit=300, newton_maxit=50, guess="previous", mass_project=True,
             max_retries=4, timing=False, precond_lag=0, newton_rel_ref=True, use_graph=False, ras_kind="left",
             mobility="1", boundary="periodic"):
    """pfc_grid, pfc_model and pfc_opts for a grid given in array-axis order."""
    shape = tuple(int(s) for s in shape)
    dim = len(shape)
    if dim not in (2, 3):
        raise ValueError("shape must be 2-D or 3-D")
    g = _lib.PfcGrid()
    g.dim = dim
    rev = list(reversed(shape))
    revL = list(reversed([float(x) for x in lengths]))
    revS = list(reversed([int(x) for x in sub]))
    for a in range(3):
        g.n[a] = rev[a] if a < dim else 1
        g.L[a] = revL[a] if a < dim else 1.0
    m = _lib.PfcModel()
    m.gamma = float(gamma)
    m.mobility = _lib.MOBILITY[mobility]
    m.boundary = _lib.BOUNDARY[boundary]
    o = _lib.PfcOpts()
    lib.pfc_default_opts(ctypes.byref(o))
    o.newton_rtol, o.newton_atol = newton_rtol, newton_atol
    o.lin_rtol, o.lin_atol = lin_rtol, lin_atol
    o.newton_maxit, o.gmres_restart, o.gmres_maxit = newton_maxit, gmres_restart, gmres_maxit
    for a in range(3):
        o.sub[a] = revS[a] if a < dim else 1
    o.overlap = int(overlap)
    o.sub_solver, level = _lib.sub_solver_code(sub_solver)
    if o.sub_solver == _lib.SUB_SOLVERS["iluk"]:
        o.ilu_level = level
    o.ras_kind = _lib.RAS_KINDS[ras_kind]
    o.precond_fp32 = int(bool(precond_fp32))
    o.mass_project = int(bool(mass_project))
    o.guess = _lib.GUESS[guess]
    o.dt_min = float(dt_min)
    o.dt_max = float(dt_max if dt_max is not None else dt_min)
    o.eta = float(eta)
    o.max_retries = int(max_retries)
    o.timing = 0xF if timing is True else int(timing)   # True: every kind; else the C bitmask
    o.precond_lag = int(precond_lag)
    o.newton_rel_ref = int(bool(newton_rel_ref))
    o.use_graph = int(bool(use_graph))
    return g, m, o


class Solver:
    """One PFC grid with its solver workspace (a ``pfc_ctx``).

    ``shape`` and ``lengths`` follow the array axes, (ny, nx) or (nz, ny, nx);
    ``sub`` (subdomains per axis) too.  ``overlap`` is in mesh layers.
    """

    def __init__(self, shape, lengths, gamma, sub, overlap, stream=None, **options):
        """Options (keywords, defaults as in pfc_default_opts unless given): sub_solver
        ("ilu0" | "lu" | "ilu1" .. "ilu4" | "iluk0"), precond_fp32, dt_min (0.1), dt_max (= dt_min), eta, newton_rtol,
        newton_atol, lin_rtol, lin_atol, gmres_restart, gmres_maxit, newton_maxit, guess
        ("previous" | "extrap" | "learned"), mass_project, max_retries, timing (True, or the
        bitmask of pfc_opts.timing), precond_lag,
        newton_rel_ref, use_graph (needs ``stream``: a non-default stream handle), ras_kind
        ("left" | "as" | "right": left-RAS, classical AS, right-RAS), mobility ("1" | "1-phi^2"),
        boundary ("periodic" | "neumann")."""
        import torch
        self._torch = torch
        self.lib = _lib.load()
        self.shape = tuple(int(s) for s in shape)
        g, m, o = _structs(self.lib, self.shape, lengths, gamma, sub, overlap, **options)
        self.opts = o
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.stream = stream
        ctx = ctypes.c_void_p()
        st = self.lib.pfc_create(ctypes.byref(g), ctypes.byref(m), ctypes.byref(o), ctypes.c_void_p(stream),
                                 ctypes.byref(ctx))
        if st != _lib.PFC_OK:
            raise PfcError(st, "pfc_create failed (see stderr)")
        self.ctx = ctx

    # -- helpers ---------------------------------------------------------------
    def _check(self, status):
        if status != _lib.PFC_OK:
            raise PfcError(status, self.lib.pfc_last_error(self.ctx).decode())

    def _field(self, t, name):
        torch = self._torch
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
                and t.is_contiguous() and tuple(t.shape) == self.shape):
            raise ValueError(f"{name} must be a contiguous float64 CUDA tensor of shape {self.shape}")
        return _ptr(t)

    def _empty(self):
        return self._torch.empty(self.shape, dtype=self._torch.float64, device="cuda")

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.pfc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- C entry points -------------------------------------------------------
    def residual(self, Phi, phi, dt, src=None, out=None, want_norm=True):
        F = out if out is not None else self._empty()
        nrm = ctypes.c_double(0.0)
        self._check(self.lib.pfc_residual(self.ctx, self._field(Phi, "Phi"), self._field(phi, "phi"), float(dt),
                                          self._field(src, "src") if src is not None else None,
                                          self._field(F, "F"), ctypes.byref(nrm) if want_norm else None))
        return F, nrm.value

    def jv(self, Phi, phi, dt, v, out=None):
        J = out if out is not None else self._empty()
        self._check(self.lib.pfc_jv(self.ctx, self._field(Phi, "Phi"), self._field(phi, "phi"), float(dt),
                                    self._field(v, "v"), self._field(J, "Jv")))
        return J

    def ras_setup(self, Phi, phi, dt):
        self._check(self.lib.pfc_ras_setup(self.ctx, self._field(Phi, "Phi"), self._field(phi, "phi"), float(dt)))

    def ras_apply(self, r, out=None):
        z = out if out is not None else self._empty()
        self._check(self.lib.pfc_ras_apply(self.ctx, self._field(r, "r"), self._field(z, "z")))
        return z

    def energy(self, phi):
        e, m = ctypes.c_double(0.0), ctypes.c_double(0.0)
        self._check(self.lib.pfc_energy(self.ctx, self._field(phi, "phi"), ctypes.byref(e), ctypes.byref(m)))
        return e.value, m.value

    def gmres(self, Phi, phi, dt, b, rtol, atol):
        x = self._empty()
        its, res = ctypes.c_int(0), ctypes.c_double(0.0)
        self._check(self.lib.pfc_gmres(self.ctx, self._field(Phi, "Phi"), self._field(phi, "phi"), float(dt),
                                       self._field(b, "b"), self._field(x, "x"), float(rtol), float(atol),
                                       ctypes.byref(its), ctypes.byref(res)))
        return x, its.value, res.value

    def newton(self, phi, dt, Phi0=None):
        Phi = (Phi0 if Phi0 is not None else phi).clone()
        st = PfcStepStats()
        self._check(self.lib.pfc_newton(self.ctx, self._field(phi, "phi"), float(dt), self._field(Phi, "Phi"),
                                        ctypes.byref(st)))
        return Phi, st.as_dict()

    def step(self, phi):
        st = PfcStepStats()
        self._check(self.lib.pfc_step(self.ctx, self._field(phi, "phi"), ctypes.byref(st)))
        return st.as_dict()

    def guess(self, kind, phi, phi_prev=None, dt=0.0, dt_prev=0.0, out=None):
        """Newton initial guess of ``kind`` ("previous" | "extrap" | "learned") from explicit
        history (pfc_guess)."""
        X = out if out is not None else self._empty()
        self._check(self.lib.pfc_guess(self.ctx, _lib.GUESS[kind], self._field(phi, "phi"),
                                       self._field(phi_prev, "phi_prev") if phi_prev is not None else None,
                                       float(dt), float(dt_prev), self._field(X, "X")))
        return X

    def reset(self):
        self._check(self.lib.pfc_reset(self.ctx))

    def checkpoint_save(self, phi, path):
        self._check(self.lib.pfc_checkpoint_save(self.ctx, self._field(phi, "phi"), str(path).encode()))

    def checkpoint_load(self, phi, path):
        self._check(self.lib.pfc_checkpoint_load(self.ctx, self._field(phi, "phi"), str(path).encode()))

    def attach_net(self, net, scales, dt_range):
        """Use ``net`` (a GuessNet) for ``guess="learned"``; scales = (s_a, s_b, s_o, s_c, beta,
        gamma), dt_range = (dt_ref, dt_lo, dt_hi) (include/pfc_net.h)."""
        sc, dr = _net_args(scales, dt_range)
        self._check(self.lib.pfc_attach_net(self.ctx, net.handle if net is not None else None, sc, dr))
        self._net = net          # the context keeps the pointer: keep the object alive

    def kernel_time(self, which):
        cnt, ms = ctypes.c_long(0), ctypes.c_double(0.0)
        self._check(self.lib.pfc_kernel_time(self.ctx, int(which), ctypes.byref(cnt), ctypes.byref(ms)))
        return cnt.value, ms.value


def _net_args(scales, dt_range):
    if len(scales) != 6 or len(dt_range) != 3:
        raise ValueError("scales = (s_a, s_b, s_o, s_c, beta, gamma), dt_range = (dt_ref, dt_lo, dt_hi)")
    sc = (ctypes.c_double * 6)(*[float(v) for v in scales])
    dr = (ctypes.c_double * 3)(*[float(v) for v in dt_range])
    return sc, dr


class GuessNet:
    """The learned-guess network of ``include/pfc_net.h`` (a ``pfc_net`` handle).

    Inputs are float32 CUDA tensors of shape (2, ny, nx), outputs (ny, nx); parameters
    are a float32 numpy vector of ``GuessNet.NPARAM`` numbers (layout in the header).
    """
    NPARAM = _lib.NET_NPARAM

    def __init__(self, params=None, stream=None):
        import torch
        self._torch = torch
        self.lib = _lib.load()
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        h = ctypes.c_void_p()
        st = self.lib.pfc_net_create(ctypes.c_void_p(stream), ctypes.byref(h))
        if st != _lib.PFC_OK:
            raise PfcError(st, "pfc_net_create failed")
        self.handle = h
        if params is not None:
            self.set_params(params)

    def _check(self, status):
        if status != _lib.PFC_OK:
            raise PfcError(status, self.lib.pfc_net_last_error(self.handle).decode())

    def _plane(self, t, shape, name):
        torch = self._torch
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
                and tuple(t.shape) == tuple(shape)):
            raise ValueError(f"{name} must be a contiguous float32 CUDA tensor of shape {tuple(shape)}")
        return _ptr(t)

    def set_params(self, params):
        import numpy as np
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32).ravel())
        if p.size != self.NPARAM:
            raise ValueError(f"expected {self.NPARAM} parameters, got {p.size}")
        self._check(self.lib.pfc_net_set_params(self.handle, p.ctypes.data_as(_lib.c_float_p)))

    def get_params(self):
        import numpy as np
        p = np.empty(self.NPARAM, dtype=np.float32)
        self._check(self.lib.pfc_net_get_params(self.handle, p.ctypes.data_as(_lib.c_float_p)))
        return p

    def forward(self, x, cond=0.0, out=None):
        """y = network(x; c = cond)."""
        ny, nx = x.shape[1:]
        y = out if out is not None else self._torch.empty((ny, nx), dtype=self._torch.float32, device="cuda")
        self._check(self.lib.pfc_net_forward(self.handle, self._plane(x, (2, ny, nx), "x"), float(cond), ny, nx,
                                             self._plane(y, (ny, nx), "y")))
        return y

    def gradient(self, x, t, cond=0.0, scale=1.0, accumulate=False, want_loss=True):
        ny, nx = x.shape[1:]
        loss = ctypes.c_double(0.0)
        self._check(self.lib.pfc_net_gradient(self.handle, self._plane(x, (2, ny, nx), "x"), float(cond),
                                              self._plane(t, (ny, nx), "t"), ny, nx, float(scale),
                                              int(bool(accumulate)), ctypes.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def get_gradient(self):
        import numpy as np
        g = np.empty(self.NPARAM, dtype=np.float32)
        self._check(self.lib.pfc_net_get_gradient(self.handle, g.ctypes.data_as(_lib.c_float_p)))
        return g

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self._check(self.lib.pfc_net_adam(self.handle, float(lr), float(beta1), float(beta2), float(eps)))

    def close(self):
        if getattr(self, "handle", None):
            self.lib.pfc_net_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Independent instances of uneven size stepped together (``include/pfc_batch.h``).

    ``instances`` is a list of dicts with the ``Solver`` arguments (shape, lengths, gamma,
    sub, overlap and option keywords); ``workers`` host threads drive them.
    """

    def __init__(self, instances, workers=8):
        self.lib = _lib.load()
        n = len(instances)
        G = (_lib.PfcGrid * n)()
        M = (_lib.PfcModel * n)()
        O = (_lib.PfcOpts * n)()
        self.shapes = []
        for i, inst in enumerate(instances):
            kw = dict(inst)
            shape, lengths, gamma = kw.pop("shape"), kw.pop("lengths"), kw.pop("gamma")
            sub, overlap = kw.pop("sub"), kw.pop("overlap")
            G[i], M[i], O[i] = _structs(self.lib, shape, lengths, gamma, sub, overlap, **kw)
            self.shapes.append(tuple(int(x) for x in shape))
        h = ctypes.c_void_p()
        st = self.lib.pfc_batch_create(n, G, M, O, int(workers), ctypes.byref(h))
        if st != _lib.PFC_OK:
            raise PfcError(st, "pfc_batch_create failed (see stderr)")
        self.handle = h
        self.count = n

    def _check(self, status):
        if status != _lib.PFC_OK:
            raise PfcError(status, self.lib.pfc_batch_last_error(self.handle).decode())

    def step(self, phis):
        """Advance every instance one step; phis: list of float64 CUDA tensors (in/out)."""
        import torch
        if len(phis) != self.count:
            raise ValueError("one field per instance")
        for t, shp in zip(phis, self.shapes):
            if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
                    and tuple(t.shape) == shp):
                raise ValueError(f"fields must be contiguous float64 CUDA tensors of shapes {self.shapes}")
        torch.cuda.current_stream().synchronize()          # the batch runs on its own streams
        ptrs = (ctypes.c_void_p * self.count)(*[t.data_ptr() for t in phis])
        st = (PfcStepStats * self.count)()
        codes = (ctypes.c_int * self.count)()
        self._check(self.lib.pfc_batch_step(self.handle, ptrs, st, codes))
        return [s.as_dict() for s in st]

    def reset(self):
        self._check(self.lib.pfc_batch_reset(self.handle))

    def attach_net(self, net, scales, dt_range):
        sc, dr = _net_args(scales, dt_range)
        self._check(self.lib.pfc_batch_attach_net(self.handle, net.handle if net is not None else None, sc, dr))
        self._net = net

    def close(self):
        if getattr(self, "handle", None):
            self.lib.pfc_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
