"""Autotuner for the Schwarz decomposition and factor reuse of one workload, and the paper's
preconditioner study (Table 2) run on this library.

Candidates are (subdomains per axis, overlap, precond_lag) triples.  Each candidate runs
``warmup`` untimed steps, is reset, and then times the first ``steps`` steps of the run
from the initial condition on the library's own solver.  The fastest candidate in time
steps per second is returned, with the whole table.  Candidates the library rejects (box
too wide for a solver, LDS limits) are reported and skipped.  Every step runs in libpfc;
this module only orchestrates and times.
"""
from __future__ import annotations

import itertools
import time

from . import PfcError, Solver


def box_candidates(shape, widths=(24, 28, 32, 40), heights=(64, 32), overlaps=(4, 6, 8)):
    """(sub, overlap) pairs whose boxes have the given extended width (x) and owned height (y)."""
    ny, nx = shape
    out = []
    for wx, hy, ov in itertools.product(widths, heights, overlaps):
        own_x = wx - 2 * ov
        if own_x <= 0 or nx % own_x or ny % hy:
            continue
        out.append(((ny // hy, nx // own_x), ov))
    return out


def autotune(shape, lengths, gamma, phi0, solver_kwargs, candidates, steps=30, warmup=2, net=None,
             net_meta=None, log=None):
    """Time every candidate (sub, overlap, precond_lag) and return (best, table).

    ``phi0`` is a float64 CUDA tensor (not modified); ``solver_kwargs`` the other Solver
    options; ``net``/``net_meta`` the learned-guess network and its scales/dt when the
    options ask for guess="learned"."""
    import torch

    table = []
    for sub, overlap, lag in candidates:
        row = {"sub": list(sub), "overlap": overlap, "precond_lag": lag}
        try:
            s = Solver(shape, lengths, gamma, sub, overlap, precond_lag=lag, **solver_kwargs)
        except (PfcError, ValueError) as e:
            row["error"] = str(e)
            table.append(row)
            continue
        try:
            if net is not None:
                s.attach_net(net, net_meta["scales"], net_meta["dt_range"])
            phi = phi0.clone()
            for _ in range(warmup):
                s.step(phi)
            s.reset()
            phi.copy_(phi0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            newton = gmres = 0
            for _ in range(steps):
                st = s.step(phi)
                newton += st["newton_its"]
                gmres += st["gmres_its"]
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            row.update(steps_per_s=steps / el, newton_its=newton, gmres_its=gmres)
        except PfcError as e:
            row["error"] = str(e)
        finally:
            s.close()
        table.append(row)
        if log:
            log(f"autotune {row}")
    ok = [r for r in table if "steps_per_s" in r]
    if not ok:
        raise RuntimeError("no autotune candidate ran")
    best = max(ok, key=lambda r: r["steps_per_s"])
    return best, table


def table2_study(shape=(256, 256), lengths=(128.0, 128.0), gamma=0.025, phi0=None, sub=(4, 4), steps=10, dt=0.01,
                 deltas=(("as", 0), ("as", 1), ("as", 2), ("left", 1), ("left", 2), ("right", 1), ("right", 2)),
                 sub_solver="ilu0", log=None):
    """The preconditioner study of the paper's Table 2 on this library: for each (Schwarz variant,
    delta) the first ``steps`` fixed steps of ``dt`` from ``phi0`` (default: test A's field) with
    the tolerances of Sec. 5 and subdomain solves ``sub_solver`` (ILU(0), factored once per step).
    delta counts 3 mesh layers.  Returns rows with the Newton iterations, GMRES iterations per
    Newton step and seconds, for comparison with the printed table."""
    import torch

    if phi0 is None:
        import pfc_inputs as I
        phi0 = torch.from_numpy(I.noise_ic(shape, 0.07, 0.07, 0)).cuda()
    rows = []
    for kind, delta in deltas:
        row = {"ras_kind": kind, "delta": delta, "overlap": 3 * delta}
        try:
            s = Solver(shape, lengths, gamma, sub, 3 * delta, sub_solver=sub_solver, precond_fp32=False,
                       guess="previous", dt_min=dt, dt_max=dt, newton_rtol=1e-8, newton_atol=1e-10,
                       lin_rtol=1e-3, lin_atol=1e-11, mass_project=False, ras_kind=kind)
        except (PfcError, ValueError) as e:
            row["error"] = str(e)
            rows.append(row)
            continue
        try:
            phi = phi0.clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            newton = gmres = 0
            for _ in range(steps):
                st = s.step(phi)
                newton += st["newton_its"]
                gmres += st["gmres_its"]
            torch.cuda.synchronize()
            row.update(newton=newton, gmres_per_newton=gmres / max(newton, 1), seconds=time.perf_counter() - t0)
        except PfcError as e:
            row["error"] = str(e)
        finally:
            s.close()
        rows.append(row)
        if log:
            log(f"table2 {row}")
    return rows


def table1_study(shape=(256, 256), lengths=(128.0, 128.0), gamma=0.025, phi0=None, sub=(4, 4), steps=10, dt=0.01,
                 solvers=("ilu0", "ilu1", "ilu2", "lu"), reuse_solver="ilu0", delta=1, ras_kind="as", fp32=False,
                 newton_maxit=50, log=None):
    """The subdomain-solver study of the paper's Table 1 on this library: classical AS with
    overlap delta (3 delta mesh layers), the first ``steps`` fixed steps of ``dt`` from ``phi0``
    (default: test A's field) with the tolerances of Sec. 5.  Each solver in ``solvers`` is
    factored at every Newton step (the table's plain columns); ``reuse_solver`` is also run with
    its factors built once per time step (the table's reuse column).  Returns rows with Newton
    iterations, GMRES iterations per Newton step and seconds ("error" when a solve fails, the
    table's n/c)."""
    import torch

    if phi0 is None:
        import pfc_inputs as I
        phi0 = torch.from_numpy(I.noise_ic(shape, 0.07, 0.07, 0)).cuda()
    runs = [(name, -1) for name in solvers] + [(reuse_solver, 0)]
    rows = []
    for name, lag in runs:
        row = {"sub_solver": name, "reuse": lag == 0, "ras_kind": ras_kind, "delta": delta}
        try:
            s = Solver(shape, lengths, gamma, sub, 3 * delta, sub_solver=name, precond_fp32=fp32, guess="previous",
                       dt_min=dt, dt_max=dt, newton_rtol=1e-8, newton_atol=1e-10, lin_rtol=1e-3, lin_atol=1e-11,
                       mass_project=False, ras_kind=ras_kind, precond_lag=lag, newton_maxit=newton_maxit,
                       max_retries=0)
        except (PfcError, ValueError) as e:
            row["error"] = str(e)
            rows.append(row)
            continue
        try:
            phi = phi0.clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            newton = gmres = 0
            for _ in range(steps):
                st = s.step(phi)
                newton += st["newton_its"]
                gmres += st["gmres_its"]
            torch.cuda.synchronize()
            row.update(newton=newton, gmres_per_newton=gmres / max(newton, 1), seconds=time.perf_counter() - t0)
        except PfcError as e:
            row["error"] = str(e)
        finally:
            s.close()
        rows.append(row)
        if log:
            log(f"table1 {row}")
    return rows
