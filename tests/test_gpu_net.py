"""GPU parity of the learned-guess network (include/pfc_net.h) against the FP64 oracle.

Tolerances.  The GPU network rounds the convolution weights to bfloat16 exactly as the
oracle does; what differs is (i) FP32 accumulation and its order (the inference pass
forms the output layer as per-tap sums added over the neighbourhood), (ii) the activations
entering the matrix cores as hi + lo bfloat16 parts, |a - hi - lo| <= 2^-17 |a|, and (iii)
tanh from one exponential (absolute error ~1e-7).  Each layer's error is thus a few 1e-5 of the sum of |w a| it accumulates; through
four layers the output agrees to ~1e-4 of its scale, and the gradients, which go through
the same split products once more, to a few 1e-4 per layer.
"""
import numpy as np
import pytest

from oracle import cnn

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pfc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1703_01202_amd as m
    return m


def _params(seed, out_scale=1.0):
    r = np.random.Generator(np.random.PCG64(seed + 100))
    theta = cnn.init_params(seed, out_scale=out_scale, cond_scale=0.5)
    layers, u1 = cnn.unpack(theta)
    for _, b in layers:
        b[:] = 0.1 * r.standard_normal(b.shape)
    return cnn.pack(layers, u1).astype(np.float32).astype(np.float64)


def _data(shape, seed):
    r = np.random.Generator(np.random.PCG64(seed))
    x = r.standard_normal((2,) + shape)
    t = 0.3 * r.standard_normal(shape)
    return x.astype(np.float32).astype(np.float64), t.astype(np.float32).astype(np.float64)


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


# (300, 523): 646 tiles of 32 x 8 cells, more than the persistent conv kernels' resident
# blocks, so blocks walk several tiles and prefetch the next one; ragged in both axes
SHAPES = [(48, 80), (37, 53), (3, 3), (300, 523)]


@pytest.mark.parametrize("shape,cond", [(SHAPES[0], 0.0), (SHAPES[0], 0.8), (SHAPES[1], -1.7), (SHAPES[2], 0.8),
                                        (SHAPES[3], 1.1)])
def test_forward_matches_oracle(pfc, shape, cond):
    theta = _params(1)
    x, _ = _data(shape, 2)
    net = pfc.GuessNet(theta)
    y = net.forward(_cuda(x), cond).double().cpu().numpy()
    ref, _ = cnn.forward(theta, x, cond)
    scale = np.abs(ref).max()
    assert np.abs(y - ref).max() <= 2e-4 * scale, np.abs(y - ref).max() / scale
    assert np.linalg.norm(y - ref) <= 1e-4 * np.linalg.norm(ref)


@pytest.mark.parametrize("shape,cond", [(SHAPES[0], 0.6), (SHAPES[1], -1.2), (SHAPES[3], 0.6)])
def test_gradient_and_loss_match_oracle(pfc, shape, cond):
    theta = _params(3)
    x, t = _data(shape, 4)
    net = pfc.GuessNet(theta)
    loss = net.gradient(_cuda(x), _cuda(t), cond=cond)
    g = net.get_gradient().astype(np.float64)
    y, acts = cnn.forward(theta, x, cond)
    ref = cnn.backward(theta, acts, y, t, cond)
    assert abs(loss - cnn.loss(y, t)) <= 1e-4 * cnn.loss(y, t)
    k = 0
    for (ws, bs) in cnn.layer_shapes():
        n = int(np.prod(ws)) + int(np.prod(bs))
        gl, rl = g[k:k + n], ref[k:k + n]
        assert np.linalg.norm(gl - rl) <= 5e-4 * np.linalg.norm(rl), (k, np.linalg.norm(gl - rl) / np.linalg.norm(rl))
        k += n
    gl, rl = g[k:], ref[k:]                                   # u1 = cond * (layer-1 bias gradient)
    assert gl.size == 32 and np.linalg.norm(gl - rl) <= 5e-4 * np.linalg.norm(rl)


def test_gradient_accumulates_with_scale(pfc):
    theta = _params(5)
    x1, t1 = _data((32, 40), 6)
    x2, t2 = _data((32, 40), 7)
    net = pfc.GuessNet(theta)
    net.gradient(_cuda(x1), _cuda(t1), cond=0.4)
    g1 = net.get_gradient().astype(np.float64)
    net.gradient(_cuda(x2), _cuda(t2), cond=-0.9)
    g2 = net.get_gradient().astype(np.float64)
    net.gradient(_cuda(x1), _cuda(t1), cond=0.4, scale=0.5)
    net.gradient(_cuda(x2), _cuda(t2), cond=-0.9, scale=0.5, accumulate=True, want_loss=False)
    g = net.get_gradient().astype(np.float64)
    np.testing.assert_allclose(g, 0.5 * (g1 + g2), rtol=1e-5, atol=1e-6 * np.abs(g1).max())


def test_adam_step_matches_oracle(pfc):
    theta = _params(8)
    x, t = _data((24, 24), 9)
    net = pfc.GuessNet(theta)
    net.gradient(_cuda(x), _cuda(t), want_loss=False)
    g = net.get_gradient().astype(np.float64)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    ref = theta
    for step in (1, 2):
        net.adam(1e-3)
        ref, m, v = cnn.adam_step(ref, g, m, v, step, 1e-3)
    got = net.get_params().astype(np.float64)
    np.testing.assert_allclose(got, ref, rtol=2e-6, atol=2e-7)


def test_set_params_round_trip_and_bad_sizes(pfc):
    theta = _params(10)
    net = pfc.GuessNet(theta)
    assert np.array_equal(net.get_params(), theta.astype(np.float32))
    with pytest.raises(ValueError):
        net.set_params(theta[:-1])
    with pytest.raises(pfc.PfcError):
        x = torch.zeros((2, 2, 5), dtype=torch.float32, device="cuda")
        net.forward(x)


def test_training_reduces_loss_on_a_learnable_map(pfc):
    # target: a fixed stencil of the second input plane, which the network represents
    r = np.random.Generator(np.random.PCG64(11))
    x = r.standard_normal((2, 32, 32))
    t = -x[1] + 0.25 * (np.roll(x[1], 1, 0) + np.roll(x[1], -1, 0))
    net = pfc.GuessNet(_params(12, out_scale=0.3))
    xc, tc = _cuda(x), _cuda(t)
    l0 = net.gradient(xc, tc)
    for _ in range(300):
        net.adam(3e-3)
        net.gradient(xc, tc, want_loss=False)
    assert net.gradient(xc, tc) < 0.05 * l0


def test_zero_output_layer_gives_the_previous_step_trajectory(pfc):
    # with W4 = b4 = 0 the learned guess equals phi^n exactly, so the whole trajectory is
    # bitwise the one of the previous-step guess
    from pfc_inputs import small_noise_64
    w = small_noise_64()
    layers, u1 = cnn.unpack(_params(13))
    layers[3][0][:] = 0.0
    layers[3][1][:] = 0.0
    net = pfc.GuessNet(cnn.pack(layers, u1))
    runs = []
    for guess in ("previous", "learned"):
        s = pfc.Solver(w.shape, w.lengths, w.gamma, w.sub, w.overlap, dt_min=w.dt_min, dt_max=w.dt_max,
                       newton_rtol=w.newton_rtol, newton_atol=w.newton_atol, guess=guess)
        if guess == "learned":
            s.attach_net(net, (0.1, 0.01, 1.0, 1.0, 0.5, 0.0), (w.dt_min, w.dt_min, w.dt_max))
        phi = torch.from_numpy(w.initial()).cuda()
        used = []
        for _ in range(4):
            used.append(s.step(phi)["guess_used"])
        runs.append((phi.cpu().numpy(), used))
    assert np.array_equal(runs[0][0], runs[1][0])
    assert runs[1][1] == [0, 2, 2, 2]       # first step: no history yet


def test_learned_guess_falls_back_to_extrapolation_off_its_step_range(pfc):
    from pfc_inputs import small_noise_64
    w = small_noise_64()
    net = pfc.GuessNet(_params(14, out_scale=0.0))
    s = pfc.Solver(w.shape, w.lengths, w.gamma, w.sub, w.overlap, dt_min=w.dt_min, dt_max=w.dt_max,
                   newton_rtol=w.newton_rtol, newton_atol=w.newton_atol, guess="learned")
    s.attach_net(net, (0.1, 0.01, 1.0, 1.0, 0.5, 0.0), (10 * w.dt_min, 5 * w.dt_min, 20 * w.dt_min))   # other steps
    phi = torch.from_numpy(w.initial()).cuda()
    used = [s.step(phi)["guess_used"] for _ in range(3)]
    assert used == [0, 1, 1]
    good = (0.1, 0.01, 1.0, 1.0, 0.5, 0.0)
    for sc, dr in [((0.0,) + good[1:], (0.1, 0.1, 0.1)), (good, (0.1, 0.2, 0.1)), (good, (0.0, 0.1, 0.2)),
                   (good[:3] + (-1.0,) + good[4:], (0.1, 0.1, 0.2)), (good[:5] + (float("inf"),), (0.1, 0.1, 0.2))]:
        with pytest.raises(pfc.PfcError):
            s.attach_net(net, sc, dr)
    with pytest.raises(ValueError):
        s.attach_net(net, good[:3], (0.1, 0.1, 0.2))


def test_trained_network_gains_over_the_method_without_it(pfc):
    """Train on solver runs of the crystal-growth physics at 128^2 (same mesh size as the
    1024^2 workload) whose step sizes sweep dt_min = 0.01 .. dt_max = 10, then solve a held-out
    problem two ways with the previous-step guess (the paper's), linear extrapolation and
    the learned guess: (a) 40 adaptive steps (Eq. (16); dt stays at dt_min there), and (b) a
    step schedule from dt_min up to dt_max with Newton started from each guess.  The learned
    guess must start Newton closer to the root at every step size (initial residual at most
    half of F(phi^n) in each decade band) and save Newton iterations, while every variant
    accepts the same solution within the Newton tolerance (in (b): the root Newton reaches
    from the previous solution, at every step of the schedule)."""
    from paper_1703_01202_amd import learned
    from pfc_inputs import crystal_growth
    sub = (4, 8)
    data = learned.generate(128, trajectories=6, seed0=21, sub=sub, overlap=4)
    assert data["dt_range"][1:] == (0.01, 10.0)
    net, hist = learned.train(data["X"], data["T"], data["C"], epochs=12, lr=3e-3, holdout=30,
                              weights=learned.sweep_weights(data["C"]))
    assert hist[-1][2] < 0.2 * hist[0][2]                      # held-out loss falls
    w = crystal_growth(128, sub, overlap=4, seed=5)            # a problem not trained on

    def solver(guess):
        s = pfc.Solver(w.shape, w.lengths, w.gamma, sub, 4, sub_solver="lu", precond_fp32=True, guess=guess,
                       dt_min=w.dt_min, dt_max=w.dt_max, eta=w.eta, newton_rtol=w.newton_rtol,
                       newton_atol=w.newton_atol, lin_rtol=w.lin_rtol, lin_atol=w.lin_atol)
        s.attach_net(net, data["scales"], data["dt_range"])
        return s

    out = {}
    for guess in ("previous", "extrap", "learned"):
        s = solver(guess)
        phi = torch.from_numpy(w.initial()).cuda()
        stats = [s.step(phi) for _ in range(40)]
        out[guess] = dict(phi=phi.cpu().numpy(), newton=sum(st["newton_its"] for st in stats),
                          ratio=float(np.median([st["res0"] / st["res_ref"] for st in stats[1:]])),
                          used=[st["guess_used"] for st in stats],
                          energy=[st["energy"] for st in stats], mass=[st["mass"] for st in stats])
        s.close()
    print({g: (o["newton"], o["ratio"]) for g, o in out.items()})
    assert out["learned"]["used"][1:] == [2] * 39
    assert out["learned"]["ratio"] < 0.5                       # initial residual at most half of F(phi^n)
    assert out["learned"]["newton"] < out["previous"]["newton"]
    assert out["learned"]["newton"] < out["extrap"]["newton"]
    # same accepted trajectory within the Newton tolerance; mass kept; energy non-increasing
    ref = out["previous"]
    for g in ("extrap", "learned"):
        assert np.linalg.norm(out[g]["phi"] - ref["phi"]) <= 1e-8 * np.linalg.norm(ref["phi"])
        assert max(abs(m - ref["mass"][0]) for m in out[g]["mass"]) <= 1e-12 * abs(ref["mass"][0])
        assert all(b <= a + 1e-9 * abs(a) for a, b in zip(out[g]["energy"], out[g]["energy"][1:]))
    # (b) the step schedule: 10 steps at 0.01, growth by 1.25 per step to 10, 10 steps at 10
    sched = learned.step_schedule(w.dt_min, w.dt_max, 10, 1.25, 10)
    bands = ((0.0, 0.05), (0.05, 1.0), (1.0, 11.0))
    res = {}
    for guess in ("previous", "extrap", "learned"):
        s = solver(guess)
        phi = torch.from_numpy(w.initial()).cuda()
        prev = dprev = None
        newton, ratios, worst = 0, [[] for _ in bands], 0.0
        for dt in sched:
            X = s.guess("previous", phi) if prev is None else s.guess(guess, phi, prev, dt, dprev)
            r0 = s.residual(X, phi, dt)[1] / s.residual(phi, phi, dt)[1]
            Phi, st = s.newton(phi, dt, Phi0=X)
            newton += st["newton_its"]
            if guess != "previous":
                P0, _ = s.newton(phi, dt)
                worst = max(worst, float(torch.linalg.norm(Phi - P0) / torch.linalg.norm(P0)))
            if prev is not None:
                ratios[next(i for i, (lo, hi) in enumerate(bands) if lo <= dt < hi)].append(r0)
            prev, dprev, phi = phi, dt, Phi
        res[guess] = dict(newton=newton, ratio=[float(np.median(r)) for r in ratios], worst=worst)
        s.close()
    print({g: (o["newton"], o["ratio"], o["worst"]) for g, o in res.items()})
    assert all(r < 0.5 for r in res["learned"]["ratio"])
    assert res["learned"]["newton"] < res["previous"]["newton"]
    assert res["learned"]["newton"] < res["extrap"]["newton"]
    # Newton stops at rtol 1e-8 of the residual it starts from; at dt = 10 the inverse Jacobian
    # (norm up to ~dt) turns that into root differences of ~1e-6 .. 1e-5 relative, while
    # another root of the nonconvex system would lie O(1e-2) away
    for g in ("extrap", "learned"):
        assert res[g]["worst"] <= 1e-4


@pytest.mark.parametrize("shape,L,sub,ov", [((1024, 1024), (400.0, 400.0), (16, 64), 4),
                                           ((40, 70), (25.0, 44.0), (2, 2), 3)])
def test_solver_learned_guess_matches_oracle(pfc, shape, L, sub, ov):
    """The solver's learned initial guess (pfc_guess, the computation pfc_step makes): the
    input planes (mean removal, step ratio, scales with the step scale g), the step-size
    condition, the network and the epilogue X = phi + s_o g y with its shift to the mass of phi, against
    the oracle's guess on the same weights, at the 1024^2 crystal mesh with the benchmark's
    boxes and on a grid that is ragged against the 32 x 8 network tiles.  y agrees to ~1e-4
    of its scale (module header), so X to a few 1e-4 of s_o g max|y|; the mass of phi is
    kept to rounding."""
    import pfc_inputs as I
    theta = _params(15, out_scale=0.5)
    n = shape[0]
    phi = I.hex_crystallites_ic(n=n, L=L[0], seed=1) if shape[0] == shape[1] else \
        I.noise_ic(shape, -0.285, 0.3, 16)
    prev = phi + 0.02 * np.random.default_rng(17).standard_normal(shape)
    scales = (0.3, 0.02, 0.01, 2.0, 0.8, -0.04)  # s_a, s_b, s_o, s_c, beta, gamma
    dt_ref = 0.05
    dt, dt_prev = 0.012, 0.01
    net = pfc.GuessNet(theta)
    s = pfc.Solver(shape, L, 0.25, sub, ov, sub_solver="lu", precond_fp32=True, guess="learned")
    s.attach_net(net, scales, (dt_ref, 0.001, 10.0))
    P = torch.from_numpy(phi).cuda()
    X = s.guess("learned", P, torch.from_numpy(prev).cuda(), dt, dt_prev).cpu().numpy()
    ref = cnn.guess(theta, phi, prev, dt / dt_prev, dt, scales, dt_ref)
    g = cnn.step_scale(dt, dt_ref, scales[4], scales[5])
    y_ref, _ = cnn.forward(theta, cnn.make_input(phi, prev, dt / dt_prev, scales[0], scales[1], g),
                           cnn.condition(dt, dt_ref, scales[3]))
    bound = 4e-4 * scales[2] * g * np.abs(y_ref).max()
    assert np.abs(X - ref).max() <= bound, (np.abs(X - ref).max(), bound)
    assert abs(X.sum() - phi.sum()) <= 1e-12 * np.abs(phi).sum()
    # the previous-step and extrapolated kinds are their closed forms
    Xp = s.guess("previous", P).cpu().numpy()
    assert np.array_equal(Xp, phi)
    Xe = s.guess("extrap", P, torch.from_numpy(prev).cuda(), dt, dt_prev).cpu().numpy()
    e = phi + (dt / dt_prev) * (phi - prev)
    e += np.mean(phi) - np.mean(e)
    assert np.abs(Xe - e).max() <= 1e-13 * np.abs(e).max()
    with pytest.raises(pfc.PfcError):
        s.guess("extrap", P, None, dt, dt_prev)
    s.close()
