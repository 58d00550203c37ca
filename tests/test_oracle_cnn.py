"""Pins of the FP64 network reference (oracle/cnn.py) against library routines, brute force,
adjoint identities, finite differences, the closed form of Adam's first steps, the
constant-plane reading of the step-size input and the scale invariance of the guess."""
import numpy as np
import pytest
import scipy.ndimage
import torch

from oracle import cnn


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def test_bf16_round_matches_torch_cast():
    r = _rng(0)
    a = np.concatenate([r.standard_normal(10000) * 10.0 ** r.integers(-6, 6, 10000),
                        [0.0, -0.0, 1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, -(1.0 + 2 ** -8), 65504.0]])
    ref = torch.from_numpy(a.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(cnn.bf16_round(a), ref)
    # ties go to the even neighbour: 1 + 2^-8 lies halfway between 1 and 1 + 2^-7
    assert cnn.bf16_round(np.array([1.0 + 2 ** -8]))[0] == 1.0
    assert cnn.bf16_round(np.array([1.0 + 3 * 2 ** -8]))[0] == 1.0 + 2 ** -6


def test_conv3x3_matches_scipy_periodic_correlation():
    r = _rng(1)
    a = r.standard_normal((3, 7, 9))
    w = r.standard_normal((4, 3, 3, 3))
    b = r.standard_normal(4)
    z = cnn.conv3x3(a, w, b)
    for o in range(4):
        ref = b[o] + sum(scipy.ndimage.correlate(a[c], w[o, c], mode="wrap") for c in range(3))
        np.testing.assert_allclose(z[o], ref, rtol=1e-13, atol=1e-13)


def test_conv3x3_brute_force_and_shift_kernels():
    r = _rng(2)
    a = r.standard_normal((2, 4, 5))
    w = r.standard_normal((2, 2, 3, 3))
    z = cnn.conv3x3(a, w, np.zeros(2))
    for o in range(2):
        for y in range(4):
            for x in range(5):
                s = 0.0
                for c in range(2):
                    for dy in range(3):
                        for dx in range(3):
                            s += w[o, c, dy, dx] * a[c, (y + dy - 1) % 4, (x + dx - 1) % 5]
                assert abs(z[o, y, x] - s) < 1e-12
    # a single tap at (dy, dx) = (0, 2) reads a[y - 1, x + 1]
    wt = np.zeros((1, 1, 3, 3))
    wt[0, 0, 0, 2] = 1.0
    z1 = cnn.conv3x3(a[:1], wt, np.zeros(1))
    np.testing.assert_array_equal(z1[0], np.roll(a[0], shift=(1, -1), axis=(0, 1)))


def test_adjoints_satisfy_inner_product_identities():
    r = _rng(3)
    a = r.standard_normal((3, 6, 5))
    w = r.standard_normal((4, 3, 3, 3))
    g = r.standard_normal((4, 6, 5))
    lhs = np.sum(cnn.conv3x3(a, w, np.zeros(4)) * g)
    assert abs(lhs - np.sum(a * cnn.conv3x3_adjoint_input(g, w))) < 1e-11 * abs(lhs) + 1e-11
    assert abs(lhs - np.sum(w * cnn.conv3x3_adjoint_weight(g, a))) < 1e-11 * abs(lhs) + 1e-11


@pytest.mark.parametrize("cond", [0.0, 0.7])
def test_backward_matches_central_differences(cond):
    width = 4
    r = _rng(4)
    theta = cnn.init_params(5, cin=2, width=width, out_scale=1.0, cond_scale=0.5)
    theta += 0.1 * r.standard_normal(theta.size)     # non-zero biases too
    x = r.standard_normal((2, 5, 6))
    t = r.standard_normal((5, 6))
    y, acts = cnn.forward(theta, x, cond, round_weights=False, width=width)
    g = cnn.backward(theta, acts, y, t, cond, round_weights=False, width=width)
    # 60 sampled parameters and every entry of u1 (the last `width` ones)
    idx = np.concatenate([r.choice(theta.size - width, 60, replace=False), theta.size - width + np.arange(width)])
    h = 1e-6
    for k in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        lp = cnn.loss(cnn.forward(tp, x, cond, round_weights=False, width=width)[0], t)
        lm = cnn.loss(cnn.forward(tm, x, cond, round_weights=False, width=width)[0], t)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd)), (k, fd, g[k])
    if cond == 0.0:
        assert not np.any(g[-width:])


def test_step_size_input_is_a_constant_third_plane():
    """Layer 1 at condition c equals a three-channel periodic correlation (scipy) whose third
    input plane is the constant c and whose third-channel taps (unrounded) sum to u1."""
    width = 4
    r = _rng(12)
    theta = cnn.init_params(13, width=width, out_scale=1.0, cond_scale=1.0)
    layers, u1 = cnn.unpack(theta, width=width)
    x = r.standard_normal((2, 6, 7))
    c = -1.3
    taps = r.uniform(0.5, 1.5, (width, 3, 3))
    taps *= (u1 / taps.sum(axis=(1, 2)))[:, None, None]      # any taps with these sums
    w1 = cnn.bf16_round(layers[0][0])
    planes = [x[0], x[1], np.full((6, 7), c)]
    z1 = np.stack([layers[0][1][o] + sum(scipy.ndimage.correlate(planes[k], w1[o, k], mode="wrap") for k in range(2))
                   + scipy.ndimage.correlate(planes[2], taps[o], mode="wrap") for o in range(width)])
    a = np.tanh(z1)
    for w, b in layers[1:3]:
        a = np.tanh(np.stack([b[o] + sum(scipy.ndimage.correlate(a[k], cnn.bf16_round(w)[o, k], mode="wrap")
                                         for k in range(width)) for o in range(width)]))
    w4, b4 = layers[3]
    y = b4[0] + sum(scipy.ndimage.correlate(a[k], cnn.bf16_round(w4)[0, k], mode="wrap") for k in range(width))
    np.testing.assert_allclose(cnn.forward(theta, x, c, width=width)[0], y, rtol=1e-12, atol=1e-12)


def test_step_size_enters_through_its_scale_and_condition_only():
    """At dt = dt_ref the scale g is 1 and c = 0: the guess is the unconditioned network on
    x1 = d / s_b with output s_o y.  At another dt it is that network with x1 / g, c and the
    output times g; and a zero history with a zero output layer gives phi^n."""
    r = _rng(14)
    phi = -0.3 + 0.1 * r.standard_normal((8, 8))
    d = 0.01 * r.standard_normal((8, 8))
    theta = cnn.init_params(15, out_scale=1.0, cond_scale=0.3)
    sc = (0.1, 0.02, 0.5, 2.0, 0.8, -0.05)
    x = np.stack([(phi - phi.mean()) / sc[0], 1.3 * d / sc[1]])
    y0, _ = cnn.forward(theta, x, 0.0)
    g0 = phi + sc[2] * y0
    np.testing.assert_allclose(cnn.guess(theta, phi, phi - d, 1.3, 0.05, sc, 0.05), g0 + (phi.mean() - g0.mean()),
                               rtol=0, atol=1e-15)
    l = np.log(0.7 / 0.05)
    gs = np.exp(0.8 * l - 0.05 * l * l)
    assert abs(cnn.step_scale(0.7, 0.05, 0.8, -0.05) - gs) < 1e-15 * gs
    y1, _ = cnn.forward(theta, np.stack([x[0], x[1] / gs]), l / 2.0)
    g1 = phi + sc[2] * gs * y1
    np.testing.assert_allclose(cnn.guess(theta, phi, phi - d, 1.3, 0.7, sc, 0.05), g1 + (phi.mean() - g1.mean()),
                               rtol=0, atol=1e-14)
    layers, u1 = cnn.unpack(theta)
    layers[3][0][:] = 0.0
    layers[3][1][:] = 0.0
    np.testing.assert_array_equal(cnn.guess(cnn.pack(layers, u1), phi, phi, 1.3, 0.7, sc, 0.05), phi)


def test_guess_is_the_same_on_a_periodically_repeated_domain():
    """The network is a periodic convolution and the mean does not change when a periodic
    field is repeated 2 x 3 times, so the guess on the repeated field is the repeated guess
    (what lets a network trained on one grid size serve a larger one)."""
    r = _rng(16)
    phi = -0.3 + 0.1 * r.standard_normal((8, 6))
    prev = phi - 0.01 * r.standard_normal((8, 6))
    theta = cnn.init_params(17, out_scale=1.0, cond_scale=0.3)
    sc = (0.1, 0.02, 0.5, 2.0, 0.8, -0.05)
    g = cnn.guess(theta, phi, prev, 1.1, 0.3, sc, 0.05)
    gt = cnn.guess(theta, np.tile(phi, (2, 3)), np.tile(prev, (2, 3)), 1.1, 0.3, sc, 0.05)
    np.testing.assert_allclose(gt, np.tile(g, (2, 3)), rtol=0, atol=1e-14)


def test_gradient_uses_rounded_weights():
    # straight-through rounding: the gradient equals the exact gradient of the network
    # whose weights are the rounded ones
    width = 4
    theta = cnn.init_params(6, cin=2, width=width, out_scale=1.0)
    r = _rng(6)
    x = r.standard_normal((2, 4, 4))
    t = r.standard_normal((4, 4))
    layers, u1 = cnn.unpack(theta, width=width)
    rounded = cnn.pack([(cnn.bf16_round(w), b) for w, b in layers], u1)
    y1, a1 = cnn.forward(theta, x, width=width)
    y2, a2 = cnn.forward(rounded, x, round_weights=False, width=width)
    np.testing.assert_array_equal(y1, y2)
    np.testing.assert_allclose(cnn.backward(theta, a1, y1, t, width=width),
                               cnn.backward(rounded, a2, y2, t, round_weights=False, width=width), rtol=0, atol=0)


def test_adam_closed_form_first_steps():
    r = _rng(7)
    theta = r.standard_normal(50)
    g = r.standard_normal(50)
    m = np.zeros(50)
    v = np.zeros(50)
    lr, eps = 1e-3, 1e-8
    th1, m, v = cnn.adam_step(theta, g, m, v, 1, lr, eps=eps)
    # bias correction makes the first moments exactly g and g^2
    np.testing.assert_allclose(th1, theta - lr * g / (np.abs(g) + eps), rtol=1e-15, atol=1e-15)
    th2, m, v = cnn.adam_step(th1, g, m, v, 2, lr, eps=eps)
    np.testing.assert_allclose(th2, th1 - lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-15)


def test_parameter_count_and_layout():
    assert cnn.n_params() == 32 * 2 * 9 + 32 + 2 * (32 * 32 * 9 + 32) + 32 * 9 + 1 + 32 == 19425
    theta = np.arange(cnn.n_params(), dtype=np.float64)
    layers, u1 = cnn.unpack(theta)
    assert layers[0][0][0, 0, 0, 0] == 0 and layers[0][1][0] == 576
    assert layers[3][1][0] == 19392 and u1[0] == 19393 and u1[-1] == cnn.n_params() - 1
    np.testing.assert_array_equal(cnn.pack(layers, u1), theta)


def test_guess_keeps_mass_and_reduces_to_previous_without_output_layer():
    r = _rng(8)
    phi = -0.3 + 0.1 * r.standard_normal((8, 8))
    prev = phi + 0.01 * r.standard_normal((8, 8))
    theta = cnn.init_params(9, out_scale=1.0, cond_scale=0.5)
    g = cnn.guess(theta, phi, prev, 1.0, 0.3, (0.1, 0.01, 1.0, 1.0, 1.0, 0.0), 0.01)
    assert abs(g.mean() - phi.mean()) < 1e-15
    layers, u1 = cnn.unpack(theta)
    layers[3][0][:] = 0.0
    layers[3][1][:] = 0.0
    g0 = cnn.guess(cnn.pack(layers, u1), phi, prev, 1.0, 0.3, (0.1, 0.01, 1.0, 1.0, 1.0, 0.0), 0.01)
    np.testing.assert_allclose(g0, phi, rtol=0, atol=1e-15)


@pytest.mark.parametrize("width", [4])
def test_training_reduces_loss_on_a_learnable_map(width):
    # target: a fixed stencil of the second input plane (a linear map a CNN represents)
    r = _rng(10)
    x = r.standard_normal((2, 12, 12))
    t = -x[1] + 0.25 * (np.roll(x[1], 1, 0) + np.roll(x[1], -1, 0))
    theta = cnn.init_params(11, width=width, out_scale=1.0)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    y, acts = cnn.forward(theta, x, round_weights=False, width=width)
    l0 = cnn.loss(y, t)
    for it in range(1, 301):
        g = cnn.backward(theta, acts, y, t, round_weights=False, width=width)
        theta, m, v = cnn.adam_step(theta, g, m, v, it, 1e-2)
        y, acts = cnn.forward(theta, x, round_weights=False, width=width)
    assert cnn.loss(y, t) < 0.05 * l0
