"""Training of the learned Newton initial guess (include/pfc_net.h).

Data: trajectories of the crystal-growth problem run by the solver with the previous-step
guess (the method without the network).  Each accepted step n -> n+1 with a predecessor
gives one sample: input planes x[0] = (phi^n - mean)/s_a, x[1] = r (phi^n - phi^(n-1))/s_b
with r = dt_n/dt_(n-1), target t = (phi^(n+1) - phi^n)/s_o.  The scales are the standard
deviations of the raw planes over the data set.

Training: Adam on the mean-square loss, mini-batches of whole grids, cosine-decayed step
size, seeded sample order.  Every forward/backward/update runs in libpfc's kernels;
the samples are assembled on the host with numpy and held on the device by torch.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import GuessNet, Solver


def _solver_for(w, sub, overlap):
    return Solver(w.shape, w.lengths, w.gamma, sub, overlap, sub_solver="lu", precond_fp32=True,
                  dt_min=w.dt_min, dt_max=w.dt_max, eta=w.eta, newton_rtol=w.newton_rtol,
                  newton_atol=w.newton_atol, lin_rtol=w.lin_rtol, lin_atol=w.lin_atol, guess="previous",
                  precond_lag=20)


def generate(n=512, trajectories=10, steps=201, seed0=11, sub=(8, 32), overlap=4, log=None):
    """Run the solver and collect samples.

    Returns dict(X=(M, 2, n, n) float32 CUDA, T=(M, n, n) float32 CUDA, scales=(s_a, s_b, s_o),
    dt=time step of the data, stats=solver statistics)."""
    import torch
    from pfc_inputs import crystal_growth

    raw_a, raw_b, raw_t, dts = [], [], [], []
    newton = gmres = 0
    t0 = time.perf_counter()
    for k in range(trajectories):
        w = crystal_growth(n, sub, overlap=overlap, nsteps=steps, seed=seed0 + k)
        s = _solver_for(w, sub, overlap)
        phi = torch.from_numpy(w.initial()).cuda()
        prev = None
        prev_dt = None
        cur = phi.cpu().numpy()
        for _ in range(steps):
            st = s.step(phi)
            nxt = phi.cpu().numpy()
            newton += st["newton_its"]
            gmres += st["gmres_its"]
            if prev is not None:
                r = st["dt"] / prev_dt
                raw_a.append((cur - cur.mean()).astype(np.float32))
                raw_b.append((r * (cur - prev)).astype(np.float32))
                raw_t.append((nxt - cur).astype(np.float32))
                dts.append(st["dt"])
            prev, prev_dt, cur = cur, st["dt"], nxt
        s.close()
        if log:
            log(f"trajectory {k + 1}/{trajectories}: {len(raw_t)} samples, {time.perf_counter() - t0:.1f} s")
    s_a = float(np.sqrt(np.mean([np.mean(a.astype(np.float64) ** 2) for a in raw_a])))
    s_b = float(np.sqrt(np.mean([np.mean(b.astype(np.float64) ** 2) for b in raw_b])))
    s_o = float(np.sqrt(np.mean([np.mean(t.astype(np.float64) ** 2) for t in raw_t])))
    M = len(raw_t)
    X = torch.empty((M, 2, n, n), dtype=torch.float32, device="cuda")
    T = torch.empty((M, n, n), dtype=torch.float32, device="cuda")
    for i in range(M):
        X[i, 0].copy_(torch.from_numpy(raw_a[i] / np.float32(s_a)))
        X[i, 1].copy_(torch.from_numpy(raw_b[i] / np.float32(s_b)))
        T[i].copy_(torch.from_numpy(raw_t[i] / np.float32(s_o)))
    return dict(X=X, T=T, scales=(s_a, s_b, s_o), dt=float(np.median(dts)),
                stats=dict(samples=M, newton_its=newton, gmres_its=gmres, seconds=time.perf_counter() - t0))


def initial_params(seed, out_scale=0.1):
    """Seeded start: weights uniform in +-sqrt(3 / fan_in) (unit variance per layer for unit
    inputs), zero biases, the output layer scaled by out_scale so the first guesses stay near
    phi^n.  Layout as in include/pfc_net.h."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for li, (cout, cin) in enumerate([(32, 2), (32, 32), (32, 32), (1, 32)]):
        w = rng.uniform(-1.0, 1.0, size=cout * cin * 9) * math.sqrt(3.0 / (cin * 9))
        if li == 3:
            w *= out_scale
        parts += [w, np.zeros(cout)]
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == GuessNet.NPARAM
    return p


def train(X, T, epochs=8, lr=2e-3, lr_final=1e-4, batch=4, seed=0, init_seed=0, holdout=64, net=None, log=None):
    """Train a GuessNet on (X, T); the last ``holdout`` samples are kept out for the loss report.

    Returns (net, history): history lists (epoch, optimiser steps, mean held-out loss)."""
    M = X.shape[0]
    ntrain = M - holdout
    if ntrain < batch:
        raise ValueError("not enough samples")
    if net is None:
        net = GuessNet(initial_params(init_seed))
    rng = np.random.Generator(np.random.PCG64(seed))
    total = epochs * (ntrain // batch)
    step = 0
    history = []
    t0 = time.perf_counter()

    def held_out_loss():
        ls = [net.gradient(X[i], T[i]) for i in range(ntrain, M)]
        return float(np.mean(ls)) if ls else float("nan")

    history.append((0, 0, held_out_loss()))
    for ep in range(1, epochs + 1):
        order = rng.permutation(ntrain)
        for b0 in range(0, ntrain - batch + 1, batch):
            idx = order[b0:b0 + batch]
            for k, i in enumerate(idx):
                net.gradient(X[int(i)], T[int(i)], scale=1.0 / len(idx), accumulate=k > 0, want_loss=False)
            frac = step / max(1, total - 1)
            net.adam(lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * frac)))
            step += 1
        history.append((ep, step, held_out_loss()))
        if log:
            log(f"epoch {ep}/{epochs}: held-out loss {history[-1][2]:.4e}  ({time.perf_counter() - t0:.1f} s)")
    return net, history
