"""Benchmark: PFC time steps per second on the 1024^2 crystal-growth workload.

One "step" is one time step of the scheme: adaptive dt, initial guess, the full
Newton-Krylov-Schwarz solve and the energy/mass evaluation of the accepted state.
Workload: 1024^2 periodic grid on [0, 400]^2, gamma = 0.25, mean density -0.285 with
three hexagonal crystallites (disks of radius 10 cells), adaptive dt in [1e-2, 10]
with eta = 5000, tolerances eps_r = 1e-8, eps_a = 1e-10, xi_r = 1e-3, xi_a = 1e-11.

Warm-up steps run from the initial state, then the solver history is reset and the
timed steps run from the initial state again (the timed region is the first K steps
of the trajectory).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
# The batch runs one HIP stream per instance; HIP maps a process's streams onto this many
# hardware queues (4 unless set).  16 lets up to 16 instances' kernels run side by side.
# Set before anything initialises HIP.
os.environ["GPU_MAX_HW_QUEUES"] = "16"

PEAK_HBM_GBS = 8000.0          # MI355X HBM3E

# HBM bytes per launch of the dominant kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE passes
# (calibrated against a known-size copy; see profiles/), valid only for the kernel source
# they were taken on: the sha256 prefix of the source file must match.
MEASURED_TRAFFIC = {   # keyed by kernel and decomposition: (kernel, sub, overlap, sub_solver, fp32)
    ("ras_apply", (16, 64), 4, "lu", True): {"file": "paper_1703_01202_amd/csrc/ras_lu.hip",
                                             "sha": "fd975203dd0c6493", "bytes": 1.2245e9},
}


def measured_traffic(v, kernel):
    import hashlib
    m = MEASURED_TRAFFIC.get((kernel, tuple(v["sub"]), v["overlap"], v["sub_solver"], v["precond_fp32"]))
    if not m:
        return None
    try:
        sha = hashlib.sha256(open(os.path.join(ROOT, m["file"]), "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    return m["bytes"] if sha == m["sha"] else None

VARIANTS = {
    # the paper's method as configured: FP64 everywhere, 16 x 16 subdomains, overlap 4,
    # exact subdomain LU factored once per step, previous solution as initial guess
    "plain": dict(sub=(16, 16), overlap=4, sub_solver="lu", precond_fp32=False, guess="previous"),
    # FP32 subdomain factors inside flexible GMRES, 24-cell-wide boxes (64 x 16 owned,
    # overlap 4), extrapolated initial guess, factors kept across up to 20 time steps
    # while they stay effective; residual, Arnoldi and energy stay FP64
    "fast": dict(sub=(16, 64), overlap=4, sub_solver="lu", precond_fp32=True, guess="extrap", precond_lag=20),
    # as "fast" with the learned initial guess (include/pfc_net.h), trained before the timed
    # region on solver trajectories of the same physics on 512^2 grids
    "learned": dict(sub=(16, 64), overlap=4, sub_solver="lu", precond_fp32=True, guess="learned", precond_lag=20),
    # as "learned" with the Arnoldi steps replayed from HIP graphs (own stream)
    "learned_graph": dict(sub=(16, 64), overlap=4, sub_solver="lu", precond_fp32=True, guess="learned",
                          precond_lag=20, use_graph=True),
}
LEARNED_TRAINING = dict(n=512, trajectories=8, hold=200, epochs=8, lr=3e-3, w_sweep=0.1)


def apply_bytes_table(shape, sub, overlap, fp32):
    """Algorithmic HBM bytes of one preconditioner apply by the per-DOF figure of the hot-path
    table: FP64 factors 208 omega + 8, FP32 factors 108 omega + 8 bytes per DOF (25 stencil
    factors per extended cell, the gather of r over the extended boxes, the write of z), with
    omega = extended / owned cells.  This is the ILU(0) apply's byte count; the exact-LU apply
    the 1024^2 workload runs reads far more (its band factors), see apply_bytes."""
    ny, nx = shape
    oy, ox = ny // sub[0], nx // sub[1]
    omega = (oy + 2 * overlap) * (ox + 2 * overlap) / (oy * ox)
    return ((108.0 if fp32 else 208.0) * omega + 8.0) * ny * nx


def apply_bytes(shape, sub, overlap, sub_solver, fp32):
    """Bytes one preconditioner apply of this sub-solver must move (factor reads + r gather +
    z write): the exact LU's stored band blocks, or the ILU(0) pattern's factors."""
    ny, nx = shape
    esz = 4 if fp32 else 8
    oy, ox = ny // sub[0], nx // sub[1]
    ey, ex = oy + 2 * overlap, ox + 2 * overlap
    nsub = sub[0] * sub[1]
    if sub_solver == "lu":
        W, H = ex, ey
        fac = H * 7 * W * W                 # [Lh | S^-1 | -Uh] per block row, all dense
    else:
        fac = 0
        for y in range(ey):
            for x in range(ex):
                fac += sum(1 for dy in range(-3, 4) for dx in range(-3, 4)
                           if abs(dx) + abs(dy) <= 3 and 0 <= x + dx < ex and 0 <= y + dy < ey)
    return nsub * (fac * esz + ex * ey * 8) + nx * ny * 8


def cpu_baseline(nsteps=2):
    """The FP64 oracle on the first ``nsteps`` steps of the same workload (host cores)."""
    import numpy as np  # noqa: F401
    import pfc_inputs as I
    from oracle import scheme as S
    w = I.crystal_growth_1024()
    h = S.spacing(w.shape, w.lengths)
    phi = w.initial()
    t0 = time.perf_counter()
    tr = S.run(phi, nsteps, w.gamma, h, w.dt_min, w.dt_max, w.eta, linear="fftgmres", keep_all=False)
    el = time.perf_counter() - t0
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    return {"value": nsteps / el, "unit": "steps/s", "cores": cores, "kind": "oracle",
            "sample": f"first {nsteps} steps of the 1024^2 crystal trajectory (dt = {tr.dts}), "
                      f"Newton + FFT-preconditioned GMRES, scipy/numpy FP64, {el:.1f} s"}


def tune_variant(name, net, net_meta, steps=30):
    """Untimed autotuning of the decomposition and factor lag for a variant (first steps of the
    same run); returns (best, table)."""
    import torch
    import pfc_inputs as I
    from paper_1703_01202_amd import autotune as A
    w = I.crystal_growth_1024()
    v = VARIANTS[name]
    kw = dict(sub_solver=v["sub_solver"], precond_fp32=v["precond_fp32"], guess=v["guess"], dt_min=w.dt_min,
              dt_max=w.dt_max, eta=w.eta, newton_rtol=w.newton_rtol, newton_atol=w.newton_atol,
              lin_rtol=w.lin_rtol, lin_atol=w.lin_atol)
    cands = [(sub, ov, lag) for sub, ov in A.box_candidates(w.shape) for lag in (50, 100)]
    phi0 = torch.tensor(w.initial(), dtype=torch.float64, device="cuda")
    t0 = time.perf_counter()
    best, table = A.autotune(w.shape, w.lengths, w.gamma, phi0, kw, cands, steps=steps, net=net,
                             net_meta=net_meta,
                             log=lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True))
    return best, {"candidates": table, "best": best, "seconds": time.perf_counter() - t0, "steps_each": steps}


def train_guess_net(cfg):
    """Train the learned-guess network (untimed set-up of the "learned" variant)."""
    import torch
    from paper_1703_01202_amd import learned
    log = lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True)   # noqa: E731
    t0 = time.perf_counter()
    data = learned.generate(cfg["n"], trajectories=cfg["trajectories"], hold=cfg["hold"], log=log)
    t1 = time.perf_counter()
    net, hist = learned.train(data["X"], data["T"], data["C"], epochs=cfg["epochs"], lr=cfg["lr"],
                              weights=learned.sweep_weights(data["C"], cfg["w_sweep"]), log=log)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    # inference cost at the benchmark grid
    x = torch.zeros((2, 1024, 1024), dtype=torch.float32, device="cuda")
    y = torch.empty((1024, 1024), dtype=torch.float32, device="cuda")
    for _ in range(3):
        net.forward(x, out=y)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    for _ in range(20):
        net.forward(x, out=y)
    torch.cuda.synchronize()
    fwd_ms = (time.perf_counter() - t3) / 20 * 1e3
    del x, y
    meta = {"scales": data["scales"], "dt_range": data["dt_range"], "samples": data["stats"]["samples"],
            "failed_steps": data["stats"]["failed_steps"],
            "data_seconds": t1 - t0, "train_seconds": t2 - t1, "held_out_loss": hist[-1][2],
            "loss_history": [h[2] for h in hist], "forward_ms_1024": fwd_ms, "config": cfg,
            "arch": "4 x conv3x3 periodic, 2(+log dt plane)-32-32-32-1, tanh; bf16 weights, fp32 accumulate"}
    del data
    torch.cuda.empty_cache()
    return net, meta


# Event timing of the headline run: the preconditioner apply (the roofline kernel) and the
# factorisation, every launch (pfc_opts.timing bits 1 and 8).  Timing every kind costs ~4% of
# the step (a few microseconds per timed dispatch), so the per-kernel breakdown of the other
# kinds comes from a shorter run of its own.
TIMING_HEADLINE = 1 | 8
TIMING_ALL = 0xF


def run_variant(name, steps, warmup, timing=TIMING_HEADLINE, net=None, net_meta=None, tuned=None):
    import torch
    v = dict(VARIANTS[name])
    if not v.get("use_graph"):
        return _run_variant(name, v, steps, warmup, timing, net, net_meta, tuned, None)
    # graph replay needs a stream of its own; per-kernel event timing is off for it
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        res = _run_variant(name, v, steps, warmup, False, net, net_meta, tuned, stream.cuda_stream)
    stream.synchronize()
    return res


def _run_variant(name, v, steps, warmup, timing, net, net_meta, tuned, stream):
    import torch
    import paper_1703_01202_amd as pfc
    import pfc_inputs as I
    w = I.crystal_growth_1024()
    if tuned:
        v.update(sub=tuple(tuned["sub"]), overlap=tuned["overlap"], precond_lag=tuned["precond_lag"])
    phi0 = torch.tensor(w.initial(), dtype=torch.float64, device="cuda")
    s = pfc.Solver(w.shape, w.lengths, w.gamma, v["sub"], v["overlap"], sub_solver=v["sub_solver"],
                   precond_fp32=v["precond_fp32"], guess=v["guess"], dt_min=w.dt_min, dt_max=w.dt_max,
                   eta=w.eta, newton_rtol=w.newton_rtol, newton_atol=w.newton_atol, lin_rtol=w.lin_rtol,
                   lin_atol=w.lin_atol, timing=timing, precond_lag=v.get("precond_lag", 0),
                   use_graph=v.get("use_graph", False), stream=stream)
    if v["guess"] == "learned":
        s.attach_net(net, net_meta["scales"], net_meta["dt_range"])
    phi = phi0.clone()
    for i in range(warmup):
        s.step(phi)
        print(f"[bench] {name} warmup step {i} done", file=sys.stderr, flush=True)
    s.reset()
    phi.copy_(phi0)
    torch.cuda.synchronize()
    newton = gmres = rejected = 0
    guess_ratio, guess_used = [], {0: 0, 1: 0, 2: 0}
    t0 = time.perf_counter()
    last = {}
    for i in range(steps):
        st = s.step(phi)
        newton += st["newton_its"]
        gmres += st["gmres_its"]
        rejected += st["rejected"]
        guess_used[st["guess_used"]] += 1
        if st["res_ref"] > 0:
            guess_ratio.append(st["res0"] / st["res_ref"])
        last = st
        if steps <= 50 or (i + 1) % 25 == 0:
            print(f"[bench] {name} step {i + 1}/{steps} t={st['t']:.2f} dt={st['dt']:.3g} "
                  f"newton={st['newton_its']} gmres={st['gmres_its']}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    kt = {k: s.kernel_time(k) for k in range(5)}
    s.close()
    N = w.shape[0] * w.shape[1]
    res = {"steps": steps, "seconds": el, "steps_per_s": steps / el, "dof_steps_per_s": N * steps / el,
           "newton_its": newton, "gmres_its": gmres, "gmres_per_newton": gmres / max(newton, 1),
           "rejected": rejected, "t_end": last.get("t"), "energy_end": last.get("energy"),
           "mass_end": last.get("mass"), "kernels": kt, "variant": v,
           "guess": {"used": {"previous": guess_used[0], "extrap": guess_used[1], "learned": guess_used[2]},
                     "res0_over_ref_median": sorted(guess_ratio)[len(guess_ratio) // 2] if guess_ratio else None}}
    if net_meta is not None:
        res["guess_net"] = net_meta
    # roofline of the dominant kernel (largest summed event time), with the table's per-DOF
    # bytes; the bytes the sub-solver itself has to stream are reported beside them
    names = {0: "ras_apply", 1: "residual", 2: "jacobian_action", 3: "factorisation"}
    bytes_per = {0: apply_bytes_table(w.shape, v["sub"], v["overlap"], v["precond_fp32"]), 1: 24 * N, 2: 24 * N}
    if not timing:
        res["roofline"] = None
        return res
    dom = max((k for k in (0, 1, 2)), key=lambda k: kt[k][1])
    cnt, ms = kt[dom]
    avg_s = ms / 1e3 / max(cnt, 1)
    gbs = bytes_per[dom] / avg_s / 1e9 if cnt else 0.0
    res["roofline"] = {"kernel": names[dom], "bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS,
                       "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS,
                       "traffic": measured_traffic(v, names[dom]),
                       "bytes_per_launch": bytes_per[dom], "avg_launch_us": avg_s * 1e6, "launches": cnt,
                       "factorisation_ms_total": kt[3][1]}
    if dom == 0:
        own = apply_bytes(w.shape, v["sub"], v["overlap"], v["sub_solver"], v["precond_fp32"])
        res["roofline"].update(
            bytes_basis=f"{'108' if v['precond_fp32'] else '208'} omega + 8 B/DOF (RAS apply, per-DOF table figure)",
            subsolver_bytes_per_launch=own, achieved_subsolver_bytes=own / avg_s / 1e9,
            frac_subsolver_bytes=own / avg_s / 1e9 / PEAK_HBM_GBS)
    for k in (1, 2):                      # the stencils, when this run timed them
        if kt[k][0]:
            sa = kt[k][1] / 1e3 / kt[k][0]
            res["roofline"].setdefault("stencils", {})[names[k]] = {
                "bytes_per_launch": 24 * N, "avg_launch_us": sa * 1e6, "achieved": 24 * N / sa / 1e9,
                "frac": 24 * N / sa / 1e9 / PEAK_HBM_GBS}
    return res


def run_3d(steps):
    """128^3 noise workload on [0, 40 pi]^3 (gamma 0.56, mean -0.2 + U(+-0.1)), adaptive dt
    0.1..10 (eta 500): FGMRES with FP32 ILU(0) subdomain solves on 8 x 8 x 8 boxes, overlap 2,
    FP64 residual / Arnoldi / energy, extrapolated guess, factors lagged up to 50 steps (over
    these 50 steps a lag of 50 takes the same Newton and GMRES iterations as a lag of 10, with
    one factorisation instead of five)."""
    import torch
    import paper_1703_01202_amd as pfc
    import pfc_inputs as I
    w = I.noise_3d_128()
    s = pfc.Solver(w.shape, w.lengths, w.gamma, w.sub, w.overlap, precond_fp32=True, guess="extrap",
                   dt_min=w.dt_min, dt_max=w.dt_max, eta=w.eta, newton_rtol=w.newton_rtol,
                   newton_atol=w.newton_atol, lin_rtol=w.lin_rtol, lin_atol=w.lin_atol, precond_lag=50, timing=True)
    phi = torch.from_numpy(w.initial()).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = [s.step(phi) for _ in range(steps)]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    kt = {k: s.kernel_time(k) for k in range(4)}
    s.close()
    e = [st["energy"] for st in stats]
    m = [st["mass"] for st in stats]
    N = w.shape[0] * w.shape[1] * w.shape[2]
    out = {"workload": "pfc3d_128_noise", "steps": steps, "seconds": el, "steps_per_s": steps / el,
           "dof_steps_per_s": N * steps / el, "newton_its": sum(st["newton_its"] for st in stats),
           "gmres_its": sum(st["gmres_its"] for st in stats), "rejected": sum(st["rejected"] for st in stats),
           "t_end": stats[-1]["t"], "dt_last": stats[-1]["dt"], "energy_monotone": all(b <= a for a, b in zip(e, e[1:])),
           "mass_drift_rel": max(abs(x - m[0]) for x in m) / abs(m[0]), "kernels": kt}
    print(f"[bench] 3-D 128^3: {steps / el:.1f} steps/s", file=sys.stderr, flush=True)
    return out


def hbm_reference(gib=1):
    """What this GPU's HBM sustains for plain streams, beside the roofline's nominal 8 TB/s: a
    read-only reduction (torch sum) and a device copy of `gib` GiB, event-timed, 10 runs each."""
    import torch
    n = gib * (1 << 27)
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = {}
    for name, fn, moved in (("read_sum", lambda: a.sum(), 8 * n), ("copy", lambda: b.copy_(a), 16 * n)):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(10):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 10
        out[name] = {"us": ms * 1e3, "GB_per_s": moved / ms / 1e6}
    del a, b
    torch.cuda.empty_cache()
    return out


def batch_bench(steps, workers_list=(1, 16)):
    """64 independent instances of uneven size (sides 128..512, gamma 0.1..0.4, mean
    -0.35..-0.2, noise 0.05, h = pi/2), adaptive dt, extrapolated guess, exact subdomain LU
    in FP32 on boxes of 64 x 16 owned cells (24-wide with overlap 4, as the 1024^2 fast
    configuration) with lagged factors: instance-steps/s with 1 and with several host workers."""
    import torch
    import paper_1703_01202_amd as pfc
    import pfc_inputs as I
    ws = I.batch_instances(64)
    insts = [dict(shape=w.shape, lengths=w.lengths, gamma=w.gamma, sub=(w.shape[0] // 64, w.shape[1] // 16),
                  overlap=4, dt_min=w.dt_min, dt_max=w.dt_max, eta=w.eta, newton_rtol=w.newton_rtol,
                  newton_atol=w.newton_atol, lin_rtol=w.lin_rtol, lin_atol=w.lin_atol, sub_solver="lu",
                  precond_fp32=True, guess="extrap", precond_lag=20) for w in ws]
    dof = sum(w.shape[0] * w.shape[1] for w in ws)
    out = {"instances": len(ws), "dof_total": dof, "steps": steps,
           "sides": sorted(set(int(w.shape[0]) for w in ws)), "runs": {}}
    for nw in workers_list:
        b = pfc.Batch(insts, workers=nw)
        phis = [torch.from_numpy(w.initial()).cuda() for w in ws]
        b.step(phis)                                       # warm-up step (first factorisations)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        newton = 0
        for _ in range(steps):
            newton += sum(st["newton_its"] for st in b.step(phis))
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        b.close()
        out["runs"][str(nw)] = {"workers": nw, "seconds": el, "instance_steps_per_s": len(ws) * steps / el,
                                "dof_steps_per_s": dof * steps / el, "newton_its": newton}
        print(f"[bench] batch workers={nw}: {len(ws) * steps / el:.1f} instance-steps/s", file=sys.stderr,
              flush=True)
    return out


def run_3d_256(steps):
    """Test D's full grid: 256^3 on [0, 80 pi]^3, three BCC spheres, gamma 0.35, dt 0.1 (see the
    workload's note on ILU(0) above that), FP32 ILU(0) on 16^3 boxes with overlap 3."""
    import torch
    import paper_1703_01202_amd as pfc
    import pfc_inputs as I
    w = I.bcc_growth_3d_256()
    phi = torch.from_numpy(w.initial()).cuda()
    s = pfc.Solver(w.shape, w.lengths, w.gamma, w.sub, w.overlap, precond_fp32=True, guess="extrap",
                   dt_min=w.dt_min, dt_max=w.dt_max, eta=w.eta, precond_lag=10, timing=True)
    s.step(phi)   # untimed: first factorisation and warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = [s.step(phi) for _ in range(steps)]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    kt = {k: s.kernel_time(k) for k in range(4)}
    s.close()
    N = w.shape[0] * w.shape[1] * w.shape[2]
    out = {"workload": "pfc3d_bcc_256", "steps": steps, "seconds": el, "steps_per_s": steps / el,
           "dof_steps_per_s": N * steps / el, "newton_its": sum(st["newton_its"] for st in stats),
           "gmres_its": sum(st["gmres_its"] for st in stats), "dt": w.dt_min, "kernels": kt}
    print(f"[bench] 3-D 256^3: {steps / el:.2f} steps/s", file=sys.stderr, flush=True)
    return out


def _crystal_solver(w, sub, overlap, guess, fp32, lag, net, net_meta, timing=False):
    import paper_1703_01202_amd as pfc
    s = pfc.Solver(w.shape, w.lengths, w.gamma, sub, overlap, sub_solver="lu", precond_fp32=fp32, guess=guess,
                   dt_min=w.dt_min, dt_max=w.dt_max, eta=w.eta, newton_rtol=w.newton_rtol,
                   newton_atol=w.newton_atol, lin_rtol=w.lin_rtol, lin_atol=w.lin_atol, precond_lag=lag,
                   timing=timing)
    if net is not None:
        s.attach_net(net, net_meta["scales"], net_meta["dt_range"])
    return s


def run_ablation(steps, net, net_meta, tuned):
    """Where the speed-up comes from: the headline workload's first steps on the headline
    decomposition for every combination of initial guess (previous solution, linear
    extrapolation, learned), subdomain factor precision (FP32, FP64) and factor lag (0: factor
    once per time step as the paper does; 100), each from the same initial state after one
    untimed step."""
    import torch
    import pfc_inputs as I
    w = I.crystal_growth_1024()
    sub = tuple(tuned["sub"]) if tuned else VARIANTS["learned"]["sub"]
    ov = tuned["overlap"] if tuned else VARIANTS["learned"]["overlap"]
    phi0 = torch.tensor(w.initial(), dtype=torch.float64, device="cuda")
    rows = []
    for guess in ("previous", "extrap", "learned"):
        for fp32 in (True, False):
            for lag in (0, 100):
                s = _crystal_solver(w, sub, ov, guess, fp32, lag, net, net_meta, timing=1 | 8)
                phi = phi0.clone()
                s.step(phi)
                s.reset()
                phi.copy_(phi0)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st = [s.step(phi) for _ in range(steps)]
                torch.cuda.synchronize()
                el = time.perf_counter() - t0
                kt = {k: s.kernel_time(k) for k in (0, 3)}
                s.close()
                rows.append({"guess": guess, "factors": "fp32" if fp32 else "fp64", "lag": lag, "steps": steps,
                             "steps_per_s": steps / el, "newton_its": sum(x["newton_its"] for x in st),
                             "gmres_its": sum(x["gmres_its"] for x in st),
                             "factorisations": kt[3][0], "factorisation_ms": kt[3][1],
                             "apply_launches": kt[0][0], "apply_ms": kt[0][1]})
                print(f"[bench] ablation {rows[-1]}", file=sys.stderr, flush=True)
    return {"workload": "pfc2d_1024_crystal", "sub": list(sub), "overlap": ov, "rows": rows}


def run_dt_sweep(net, net_meta, tuned, hold=10, growth=1.25, tail=10):
    """The headline workload over the decades of dt that the adaptive step (Eq. (16)) spans:
    a fixed schedule (hold steps at dt_min = 0.01, dt growing by `growth` per step to
    dt_max = 10, tail steps at 10), each step's Newton started from the guess of each kind
    (the learned guess conditioned on the step size).  On this workload the controller itself
    keeps dt at dt_min for as long as a run here lasts (|dE/dt| of the total energy stays far
    above the ~14 at which Eq. (16) with eta = 5000 lets dt grow), so the schedule stands in
    for the late stretch of a long run."""
    import torch
    import pfc_inputs as I
    from paper_1703_01202_amd import learned
    w = I.crystal_growth_1024()
    sub = tuple(tuned["sub"]) if tuned else VARIANTS["learned"]["sub"]
    ov = tuned["overlap"] if tuned else VARIANTS["learned"]["overlap"]
    sched = learned.step_schedule(w.dt_min, w.dt_max, hold, growth, tail)
    bands = ((0.0, 0.05), (0.05, 1.0), (1.0, 11.0))
    out = {"workload": "pfc2d_1024_crystal", "schedule": {"hold": hold, "growth": growth, "tail": tail,
                                                          "steps": len(sched)},
           "bands": [list(b) for b in bands], "runs": {}}
    phi0 = torch.tensor(w.initial(), dtype=torch.float64, device="cuda")
    for guess in ("previous", "extrap", "learned"):
        s = _crystal_solver(w, sub, ov, guess, True, 100, net, net_meta)
        phi = phi0.clone()
        prev = dprev = None
        newton = [0] * len(bands)
        ratios = [[] for _ in bands]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for dt in sched:
            X = s.guess("previous", phi) if prev is None else s.guess(guess, phi, prev, dt, dprev)
            r0 = s.residual(X, phi, dt)[1] / s.residual(phi, phi, dt)[1]
            Phi, st = s.newton(phi, dt, Phi0=X)
            b = next(i for i, (lo, hi) in enumerate(bands) if lo <= dt < hi)
            newton[b] += st["newton_its"]
            if prev is not None:
                ratios[b].append(r0)
            prev, dprev, phi = phi, dt, Phi
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        s.close()
        out["runs"][guess] = {"seconds": el, "steps_per_s": len(sched) / el, "newton_its": newton,
                              "res0_over_ref_median": [float(sorted(r)[len(r) // 2]) if r else None for r in ratios]}
        print(f"[bench] dt sweep {guess}: newton per band {newton}, residual ratio "
              f"{out['runs'][guess]['res0_over_ref_median']}", file=sys.stderr, flush=True)
    return out


def run_stencil_sizes(reps=20):
    """The residual and Jacobian-action kernels alone at 1024^2, 2048^2, 4096^2 (2-D: LDS tiles
    below 2^21 cells, sliding sweeps above) and 128^3 (3-D multi-pass), each timed with events
    over `reps` calls after 3 untimed ones; 24 algorithmic bytes per cell (two fields read,
    one written)."""
    import math
    import torch
    import paper_1703_01202_amd as pfc
    out = []
    for shape, sub in (((1024, 1024), (32, 32)), ((2048, 2048), (32, 32)), ((4096, 4096), (32, 32)),
                       ((128, 128, 128), (8, 8, 8))):
        L = tuple(400.0 * n / 1024 for n in shape) if len(shape) == 2 else (40 * math.pi,) * 3
        s = pfc.Solver(shape, L, 0.25, sub, 2, timing=2 | 4, gmres_restart=2)
        g = torch.Generator(device="cuda").manual_seed(0)
        phi = -0.285 + 0.3 * torch.rand(shape, dtype=torch.float64, device="cuda", generator=g)
        Phi = phi + 0.01 * torch.randn(shape, dtype=torch.float64, device="cuda", generator=g)
        v = torch.randn(shape, dtype=torch.float64, device="cuda", generator=g)
        F, J = torch.empty_like(phi), torch.empty_like(phi)
        for _ in range(3):
            s.residual(Phi, phi, 0.1, out=F, want_norm=False)
            s.jv(Phi, phi, 0.1, v, out=J)
        s.reset()
        for _ in range(reps):
            s.residual(Phi, phi, 0.1, out=F, want_norm=False)
            s.jv(Phi, phi, 0.1, v, out=J)
        N = phi.numel()
        row = {"shape": list(shape)}
        for k, name in ((1, "residual"), (2, "jacobian_action")):
            cnt, ms = s.kernel_time(k)
            us = ms / cnt * 1e3
            row[name] = {"avg_us": us, "achieved_GBs": 24 * N / us / 1e3, "frac": 24 * N / us / 1e3 / PEAK_HBM_GBS}
        s.close()
        del phi, Phi, v, F, J
        torch.cuda.empty_cache()
        out.append(row)
        print(f"[bench] stencils {shape}: residual {row['residual']['avg_us']:.1f} us, "
              f"Jv {row['jacobian_action']['avg_us']:.1f} us", file=sys.stderr, flush=True)
    return out


def run_crack(steps):
    """Test C's grid: 4096 x 1024 over the periodic system of 591 x 76 lattice periods (about
    4096 pi/3 x 1024 pi/3), the notched lattice, gamma 1, adaptive dt 1..5 (eta 100); FP32
    exact-LU subdomain solves on 16 x 64 boxes of 64 x 64 owned cells, overlap 3; extrapolated
    guess, factors lagged up to 20 steps."""
    import torch
    import paper_1703_01202_amd as pfc
    import pfc_inputs as I
    w = I.crack_4096x1024()
    phi = torch.from_numpy(w.initial()).cuda()
    s = pfc.Solver(w.shape, w.lengths, w.gamma, w.sub, w.overlap, sub_solver="lu", precond_fp32=True,
                   guess="extrap", dt_min=w.dt_min, dt_max=w.dt_max, eta=w.eta, precond_lag=20, timing=True)
    s.step(phi)   # untimed: first factorisation and warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = [s.step(phi) for _ in range(steps)]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    kt = {k: s.kernel_time(k) for k in range(4)}
    s.close()
    N = w.shape[0] * w.shape[1]
    e = [st["energy"] for st in stats]
    out = {"workload": "pfc2d_crack_4096x1024", "steps": steps, "seconds": el, "steps_per_s": steps / el,
           "dof_steps_per_s": N * steps / el, "newton_its": sum(st["newton_its"] for st in stats),
           "gmres_its": sum(st["gmres_its"] for st in stats), "dt_last": stats[-1]["dt"],
           "energy_monotone": all(b <= a for a, b in zip(e, e[1:])), "kernels": kt}
    print(f"[bench] test C 4096x1024: {steps / el:.1f} steps/s", file=sys.stderr, flush=True)
    return out


def run_test_b_variants(steps):
    """Test B's four variants (Sec. 5: periodic or Neumann-type boundaries, M = 1 or 1 - phi^2) on
    the 1024^2 crystal workload: FP32 exact-LU RAS on 16 x 64 boxes (overlap 4; with the variable
    mobility each subdomain row scaled by its node mobility), the previous solution as the guess
    (the paper's; extrapolating the sign-flipping stiff increments drives M = 1 - phi^2 negative
    in the crystallites and Newton off its root), factors lagged up to 20 steps; the
    variable-mobility and Neumann residual and Jacobian action run as the multi-pass stencil
    kernels."""
    import torch
    import paper_1703_01202_amd as pfc
    import pfc_inputs as I
    out = {}
    for w in I.test_b_variants():
        s = pfc.Solver(w.shape, w.lengths, w.gamma, w.sub, w.overlap, sub_solver="lu", precond_fp32=True,
                       guess="previous", dt_min=w.dt_min, dt_max=w.dt_max, eta=w.eta, newton_rtol=w.newton_rtol,
                       newton_atol=w.newton_atol, lin_rtol=w.lin_rtol, lin_atol=w.lin_atol, precond_lag=20,
                       mobility=w.mobility, boundary=w.boundary)
        phi = torch.from_numpy(w.initial()).cuda()
        try:
            s.step(phi)   # untimed: first factorisation
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            stats = [s.step(phi) for _ in range(steps)]
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
        except pfc.PfcError as e:
            out[w.name] = {"mobility": w.mobility, "boundary": w.boundary, "error": str(e)}
            print(f"[bench] test B variant {w.name}: {e}", file=sys.stderr, flush=True)
            continue
        finally:
            s.close()
        e = [st["energy"] for st in stats]
        m = [st["mass"] for st in stats]
        out[w.name] = {"mobility": w.mobility, "boundary": w.boundary, "steps": steps, "steps_per_s": steps / el,
                       "newton_its": sum(st["newton_its"] for st in stats),
                       "gmres_its": sum(st["gmres_its"] for st in stats),
                       "energy_monotone": all(b <= a for a, b in zip(e, e[1:])),
                       "mass_drift_rel": max(abs(x - m[0]) for x in m) / abs(m[0]), "t_end": stats[-1]["t"]}
        print(f"[bench] test B variant {w.name}: {steps / el:.1f} steps/s", file=sys.stderr, flush=True)
    return out


def run_table1():
    """Table 1's test A row (256^2, first 10 steps of dt = 0.01, classical AS delta 1 on 4 x 4
    boxes): ILU(0), ILU(1), ILU(2), exact LU factored at every Newton step and ILU(0) reused for
    the whole step."""
    from paper_1703_01202_amd.autotune import table1_study

    rows = table1_study()
    for r in rows:
        print(f"[bench] table1 {r}", file=sys.stderr, flush=True)
    return rows


def run_table2():
    """Table 2's Test A block (256^2, first 10 steps of dt = 0.01, ILU(0), 4 x 4 boxes): Newton and
    GMRES counts and seconds for classical AS delta 0..2 and left/right-RAS delta 1..2."""
    from paper_1703_01202_amd.autotune import table2_study

    rows = table2_study()
    for r in rows:
        print(f"[bench] table2 {r}", file=sys.stderr, flush=True)
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--variant", default="learned", choices=sorted(VARIANTS))
    ap.add_argument("--compare", default="plain", help="second variant timed beside (or 'none')")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=4)
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-instance batch measurement")
    ap.add_argument("--no-autotune", action="store_true", help="use the variant's fixed decomposition")
    ap.add_argument("--no-graph", action="store_true", help="skip the HIP-graph replay run of the variant")
    ap.add_argument("--no-hbm-reference", action="store_true",
                    help="skip the 1 GiB read/copy reference (profiled runs: keeps the trace to the solve)")
    ap.add_argument("--no-breakdown", action="store_true",
                    help="skip the short run that times every kernel kind (per-kernel breakdown)")
    ap.add_argument("--train-trajectories", type=int, default=LEARNED_TRAINING["trajectories"])
    ap.add_argument("--train-epochs", type=int, default=LEARNED_TRAINING["epochs"])
    ap.add_argument("--no-3d", action="store_true", help="skip the 128^3 measurement")
    ap.add_argument("--no-table2", action="store_true", help="skip the Test A preconditioner study (Table 2)")
    ap.add_argument("--no-table1", action="store_true", help="skip the Test A subdomain-solver study (Table 1)")
    ap.add_argument("--steps-variants", type=int, default=10,
                    help="steps of each of test B's four variants at 1024^2 (0 skips them)")
    ap.add_argument("--steps-3d-256", type=int, default=6, help="steps of the 256^3 test-D grid (0 skips it)")
    ap.add_argument("--steps-crack", type=int, default=20, help="steps of the 4096x1024 test-C grid (0 skips it)")
    ap.add_argument("--steps-ablation", type=int, default=20,
                    help="steps of each guess x factor precision x lag combination (0 skips the ablation)")
    ap.add_argument("--no-stencil-sizes", action="store_true",
                    help="skip the residual / Jacobian-action timings at 1024^2..4096^2 and 128^3")
    ap.add_argument("--no-dt-sweep", action="store_true",
                    help="skip the guess comparison over a dt schedule from 0.01 to 10")
    ap.add_argument("--steps-3d", type=int, default=50)
    ap.add_argument("--batch-steps", type=int, default=5)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 512 MiB device-to-device copy first (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(how it would shard is described in the design notes)", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        import torch
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    net = net_meta = None
    if "learned" in (args.variant, args.compare):
        net, net_meta = train_guess_net(dict(LEARNED_TRAINING, trajectories=args.train_trajectories,
                                             epochs=args.train_epochs))
    tuned = tune_info = None
    if not args.no_autotune and VARIANTS[args.variant]["sub_solver"] == "lu" and VARIANTS[args.variant]["precond_fp32"]:
        tuned, tune_info = tune_variant(args.variant, net, net_meta)
    main_res = run_variant(args.variant, args.steps, args.warmup, net=net, net_meta=net_meta, tuned=tuned)
    if tune_info is not None:
        main_res["autotune"] = tune_info
    if not args.no_breakdown:
        brk = run_variant(args.variant, min(args.steps, 50), args.warmup, timing=TIMING_ALL, net=net,
                          net_meta=net_meta, tuned=tuned)
        main_res["kernel_breakdown"] = {"steps": brk["steps"], "steps_per_s_all_kinds_timed": brk["steps_per_s"],
                                        "kernels": brk["kernels"]}
        if main_res.get("roofline") and brk.get("roofline") and "stencils" in brk["roofline"]:
            main_res["roofline"]["stencils"] = brk["roofline"]["stencils"]
    graph_res = None
    if not args.no_graph and args.variant == "learned":
        graph_res = run_variant("learned_graph", args.steps, args.warmup, net=net, net_meta=net_meta, tuned=tuned)
    cmp_res = None
    if args.compare != "none" and args.compare != args.variant:
        cmp_res = run_variant(args.compare, args.steps, args.warmup, net=net, net_meta=net_meta)
    cpu = None if args.no_cpu_baseline else cpu_baseline(args.cpu_steps)
    batch = None if args.no_batch else batch_bench(args.batch_steps)
    hbm_ref = None if args.no_hbm_reference else hbm_reference()
    three_d = None if args.no_3d else run_3d(args.steps_3d)
    table2 = None if args.no_table2 else run_table2()
    table1 = None if args.no_table1 else run_table1()
    variants = run_test_b_variants(args.steps_variants) if args.steps_variants > 0 else None
    three_d_256 = run_3d_256(args.steps_3d_256) if args.steps_3d_256 > 0 else None
    crack = run_crack(args.steps_crack) if args.steps_crack > 0 else None
    ablation = run_ablation(args.steps_ablation, net, net_meta, tuned) \
        if args.steps_ablation > 0 and net is not None else None
    dt_sweep = run_dt_sweep(net, net_meta, tuned) if not args.no_dt_sweep and net is not None else None
    stencil_sizes = None if args.no_stencil_sizes else run_stencil_sizes()
    out = {
        "metric": "PFC time steps/s & HBM GB/s, 2D 1024^2 NKS; learned+FP32-precond vs plain",
        "value": main_res["steps_per_s"],
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * main_res["seconds"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "precond_dtype": "f32" if VARIANTS[args.variant]["precond_fp32"] else "f64",
        "data": "synthetic",
        "config": {"workload": "pfc2d_1024_crystal: 1024^2 periodic, [0,400]^2, gamma 0.25, mean -0.285, "
                               "3 hex crystallites r=10 cells, adaptive dt 1e-2..10 eta 5000",
                   "variant": args.variant, "dof": 1024 * 1024},
        "dof_steps_per_s": main_res["dof_steps_per_s"],
        "newton_its": main_res["newton_its"],
        "gmres_per_newton": main_res["gmres_per_newton"],
        "roofline": main_res["roofline"],
        "cpu_baseline": cpu,
        "detail": {args.variant: main_res},
    }
    if cmp_res is not None:
        out["compare"] = {"variant": args.compare, "steps_per_s": cmp_res["steps_per_s"],
                          "newton_its": cmp_res["newton_its"], "gmres_per_newton": cmp_res["gmres_per_newton"],
                          "roofline": cmp_res["roofline"],
                          "speedup": main_res["steps_per_s"] / cmp_res["steps_per_s"]}
        out["detail"][args.compare] = cmp_res
    if graph_res is not None:
        out["detail"]["learned_graph"] = graph_res
    if batch is not None:
        out["detail"]["batch_64_ragged"] = batch
    if three_d is not None:
        out["detail"]["pfc3d_128_noise"] = three_d
    if hbm_ref is not None:
        out["detail"]["hbm_reference"] = hbm_ref
    if table2 is not None:
        out["detail"]["table2_test_a"] = table2
    if table1 is not None:
        out["detail"]["table1_test_a"] = table1
    if variants is not None:
        out["detail"]["test_b_variants_1024"] = variants
    if three_d_256 is not None:
        out["detail"]["pfc3d_bcc_256"] = three_d_256
    if crack is not None:
        out["detail"]["pfc2d_crack_4096x1024"] = crack
    if ablation is not None:
        out["detail"]["ablation_guess_precision_lag"] = ablation
    if dt_sweep is not None:
        out["detail"]["dt_sweep_guess"] = dt_sweep
    if stencil_sizes is not None:
        out["detail"]["stencil_sizes"] = stencil_sizes
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
