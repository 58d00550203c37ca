"""Training of the learned Newton initial guess (include/pfc_net.h).

Data: trajectories of the crystal-growth problem solved by the library's Newton-Krylov
solver (exact-LU RAS, FP32 factors) from the previous solution, the method without the
network.  The step sizes of a trajectory follow a schedule that holds dt at dt_min, then
grows it geometrically to dt_max and holds it there, as the adaptive step of Eq. (16) does
while the system relaxes; the growth factor differs between trajectories.  Each step
n -> n+1 with a predecessor gives one sample: with d = r (phi^n - phi^(n-1)),
r = dt_n / dt_(n-1), l = ln(dt_n / dt_ref) and the step scale g = exp(beta l + gamma l^2),
the input planes x[0] = (phi^n - mean)/s_a, x[1] = d / (s_b g), the condition c = l / s_c
and the target t = (phi^(n+1) - phi^n) / (s_o g).  dt_ref is the geometric mean step of the
data; beta and gamma fit ln rms(phi^(n+1) - phi^n) as a quadratic in l (least squares over
the samples), so that g carries the size of a step's increment over the decades of dt;
s_a, s_b, s_o and s_c are the root-mean-square sizes of the raw planes (divided by g) and of
l over the data set.  All of them are constants at a given dt, so the network sees the
local field as on the 512^2 training grids on any grid of the same mesh size.

Training: Adam on the mean-square loss, mini-batches of whole grids, cosine-decayed step
size, seeded sample order.  Every forward/backward/update runs in libpfc's kernels;
the samples are assembled on the host with numpy and held on the device by torch.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import GuessNet, PfcError, Solver


def _solver_for(w, sub, overlap):
    return Solver(w.shape, w.lengths, w.gamma, sub, overlap, sub_solver="lu", precond_fp32=True,
                  dt_min=w.dt_min, dt_max=w.dt_max, eta=w.eta, newton_rtol=w.newton_rtol,
                  newton_atol=w.newton_atol, lin_rtol=w.lin_rtol, lin_atol=w.lin_atol, guess="previous",
                  precond_lag=20)


GROWTH = (1.1, 1.2, 1.35, 1.6)   # step-size growth factors per step, one per trajectory in turn


def step_schedule(dt_min, dt_max, hold, growth, tail):
    """hold steps at dt_min, then dt multiplied by growth each step up to dt_max, then tail
    steps at dt_max."""
    dts = [dt_min] * hold
    dt = dt_min
    while dt * growth < dt_max:
        dt *= growth
        dts.append(dt)
    return dts + [dt_max] * tail


def generate(n=512, trajectories=8, hold=100, tail=12, seed0=11, sub=(8, 32), overlap=4, dt_max=None, log=None):
    """Run the solver and collect samples (dt_max: the end of the step sweep, the workload's
    dt_max when None; dt_max = dt_min gives trajectories at dt_min only).

    Returns dict(X=(M, 2, n, n) float32 CUDA, C=(M,) float64 conditions, T=(M, n, n) float32
    CUDA, scales=(s_a, s_b, s_o, s_c, beta, gamma), dt_range=(dt_ref, dt_lo, dt_hi),
    stats=solver statistics)."""
    import torch
    from pfc_inputs import crystal_growth

    raw_a, raw_b, raw_t, dts, inc = [], [], [], [], []
    newton = gmres = failed = 0
    t0 = time.perf_counter()
    for k in range(trajectories):
        w = crystal_growth(n, sub, overlap=overlap, seed=seed0 + k)
        s = _solver_for(w, sub, overlap)
        phi = torch.from_numpy(w.initial()).cuda()
        prev = prev_dt = None
        cur = phi.cpu().numpy()
        top = w.dt_max if dt_max is None else dt_max
        for dt in step_schedule(w.dt_min, top, hold + 10 * (k % 3), GROWTH[k % len(GROWTH)], tail if top > w.dt_min else 0):
            try:
                Phi, st = s.newton(phi, dt)
            except PfcError:
                failed += 1
                break
            phi.copy_(Phi)
            nxt = phi.cpu().numpy()
            newton += st["newton_its"]
            gmres += st["gmres_its"]
            if prev is not None:
                t = nxt - cur
                raw_a.append((cur - cur.mean()).astype(np.float32))
                raw_b.append(((dt / prev_dt) * (cur - prev)).astype(np.float32))
                raw_t.append(t.astype(np.float32))
                dts.append(dt)
                inc.append(float(np.sqrt(np.mean(t * t))))
            prev, prev_dt, cur = cur, dt, nxt
        s.close()
        if log:
            log(f"trajectory {k + 1}/{trajectories}: {len(raw_t)} samples, {time.perf_counter() - t0:.1f} s")
    lref = float(np.mean(np.log(dts)))
    l = np.log(np.asarray(dts)) - lref
    beta = gamma = 0.0
    if np.ptp(l) > 1e-9:               # ln rms increment ~ a + beta l + gamma l^2
        keep = np.asarray(inc) > 0
        A = np.stack([np.ones_like(l), l, l * l], axis=1)[keep]
        coef = np.linalg.lstsq(A, np.log(np.asarray(inc)[keep]), rcond=None)[0]
        beta, gamma = float(coef[1]), float(coef[2])
    g = np.exp(beta * l + gamma * l * l)
    s_a = float(np.sqrt(np.mean([np.mean(a.astype(np.float64) ** 2) for a in raw_a])))
    s_b = float(np.sqrt(np.mean([np.mean(b.astype(np.float64) ** 2) / gi ** 2 for b, gi in zip(raw_b, g)])))
    s_o = float(np.sqrt(np.mean([np.mean(t.astype(np.float64) ** 2) / gi ** 2 for t, gi in zip(raw_t, g)])))
    s_c = float(max(np.sqrt(np.mean(l * l)), 1e-3))
    M = len(raw_t)
    X = torch.empty((M, 2, n, n), dtype=torch.float32, device="cuda")
    T = torch.empty((M, n, n), dtype=torch.float32, device="cuda")
    for i in range(M):
        X[i, 0].copy_(torch.from_numpy(raw_a[i] / np.float32(s_a)))
        X[i, 1].copy_(torch.from_numpy((raw_b[i] / (s_b * g[i])).astype(np.float32)))
        T[i].copy_(torch.from_numpy((raw_t[i] / (s_o * g[i])).astype(np.float32)))
    return dict(X=X, C=l / s_c, T=T, scales=(s_a, s_b, s_o, s_c, beta, gamma),
                dt_range=(math.exp(lref), min(dts), max(dts)),
                stats=dict(samples=M, newton_its=newton, gmres_its=gmres, failed_steps=failed,
                           seconds=time.perf_counter() - t0))


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
    parts.append(np.zeros(32))                      # u1: the step size starts without effect
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == GuessNet.NPARAM
    return p


def sweep_weights(C, w_sweep=0.1):
    """Loss weights: 1 for the samples at the smallest step of the data (dt_min, where an
    adaptive run spends most of its steps), w_sweep for those of the step sweep.  With equal
    weights the sweep's samples, whose increments are larger and harder to predict, dominate
    the gradient and the guess at dt_min loses most of its accuracy (the 1024^2 workload's
    Newton count goes back up from 2 to 2.5 per step); at w_sweep = 0.1 the dt_min guess is
    nearly that of a network trained at dt_min alone and the sweep's guess still halves the
    initial residual or better."""
    C = np.asarray(C, dtype=np.float64)
    return np.where(np.abs(C - C.min()) < 1e-9, 1.0, w_sweep)


def torch_mean_sq(T):
    """mean(t^2) of every sample of T (M, ny, nx), as float64 numpy."""
    return (T.double() ** 2).mean(dim=(1, 2)).cpu().numpy()


def train(X, T, C=None, epochs=8, lr=2e-3, lr_final=1e-4, batch=4, seed=0, init_seed=0, holdout=64, net=None,
          relative=False, weights=None, log=None):
    """Train a GuessNet on (X, C, T) (C: per-sample conditions, zero when None); ``holdout``
    samples spread over the data set are kept out for the loss report.  relative: weight
    each sample's loss by 1 / mean(t^2), so that samples with small increments (small dt,
    late in a relaxation) count as much as large ones; the reported loss is then relative.
    weights: per-sample loss weights (multiplying the relative ones when both are given).

    Returns (net, history): history lists (epoch, optimiser steps, mean held-out loss)."""
    M = X.shape[0]
    C = np.zeros(M) if C is None else np.asarray(C, dtype=np.float64)
    wt = (1.0 / np.maximum(torch_mean_sq(T), 1e-30)) if relative else np.ones(M)
    if weights is not None:
        wt = wt * np.asarray(weights, dtype=np.float64)
    held = np.linspace(0, M - 1, min(holdout, M)).astype(int) if holdout > 0 else np.zeros(0, dtype=int)
    train_idx = np.setdiff1d(np.arange(M), held)
    ntrain = train_idx.size
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
        ls = [wt[int(i)] * net.gradient(X[int(i)], T[int(i)], cond=C[int(i)]) for i in held]
        return float(np.mean(ls)) if ls else float("nan")

    history.append((0, 0, held_out_loss()))
    for ep in range(1, epochs + 1):
        order = train_idx[rng.permutation(ntrain)]
        for b0 in range(0, ntrain - batch + 1, batch):
            idx = order[b0:b0 + batch]
            for k, i in enumerate(idx):
                net.gradient(X[int(i)], T[int(i)], cond=C[int(i)], scale=wt[int(i)] / len(idx), accumulate=k > 0,
                             want_loss=False)
            frac = step / max(1, total - 1)
            net.adam(lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * frac)))
            step += 1
        history.append((ep, step, held_out_loss()))
        if log:
            log(f"epoch {ep}/{epochs}: held-out loss {history[-1][2]:.4e}  ({time.perf_counter() - t0:.1f} s)")
    return net, history
