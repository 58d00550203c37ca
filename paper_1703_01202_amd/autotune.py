"""Autotuner for the Schwarz decomposition and factor reuse of one workload.

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
                s.attach_net(net, net_meta["scales"], net_meta["dt_train"])
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
