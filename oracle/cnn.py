"""FP64 reference of the learned Newton initial guess: a four-layer 3x3 convolutional network
conditioned on the time step.

TEST INFRASTRUCTURE ONLY (see the package header).

The paper solves each time step by Newton from the previous solution (Sec. 4); the
network here is an addition that predicts the time increment phi^(n+1) - phi^n from
planes built from the history and the step size, so that Newton starts closer to its root.
Newton's own residual test (Sec. 4, Eq. (20)) still decides when a step is solved, so the
accepted solution does not depend on the guess.  The adaptive step of Sec. 3 (Eq. (16))
moves dt over three decades, so the step size is an input of the network.

Definition (what both this reference and the GPU kernels compute)
  step   l = ln(dt_n / dt_ref), the log step size;  c = l / s_c;
         g = exp(beta l + gamma l^2), the typical size of one step's increment at dt_n
         relative to dt_ref (a fit over the training data)
  input  x: (2, ny, nx) -- x[0] = (phi^n - mean(phi^n)) / s_a,
                           x[1] = d / (s_b g),  d = (dt_n / dt_(n-1)) (phi^n - phi^(n-1)),
                                  the linear-extrapolation increment
         c, a constant third input plane
  layer l = 1..4: z_l = b_l + sum_{c, dy, dx} bf16(W_l)[o, c, dy, dx] a_(l-1)[c, y+dy-1, x+dx-1]
         (periodic wrap, i.e. cross-correlation on the torus), a_0 = x,
         a_l = tanh(z_l) for l < 4, output y = z_4: (ny, nx);
         layer 1 also sees the constant plane c: its 3x3 taps of that plane sum to u1[o], so
         it adds c u1[o] to z_1 (u1 full precision, like the biases)
  channels 2 (+ the constant plane) -> 32 -> 32 -> 32 -> 1; the convolution weights are
  rounded to bfloat16 (round to nearest, ties to even) before use, biases and u1 stay in
  full precision.
  guess  G = phi^n + s_o g y, then shifted to the mass of phi^n.
  loss   L = mean over cells of (y - t)^2 with target t = (phi^(n+1) - phi^n) / (s_o g).
  At one step size the scales are constants, so the network acts on the local field the
  same way on any grid of the same mesh size.

The gradient is taken with respect to the rounded weights and applied to the FP32
master copy (straight-through rounding).  Adam follows Kingma & Ba (2015), Algorithm 1,
with bias-corrected moments.

Flat parameter layout (float32 on the GPU side, float64 here):
  W1 (32, 2, 3, 3), b1 (32), W2 (32, 32, 3, 3), b2 (32), W3 (32, 32, 3, 3), b3 (32),
  W4 (1, 32, 3, 3), b4 (1), u1 (32)   -- 19425 numbers for width 32.
"""
from __future__ import annotations

import numpy as np

CIN = 2
WIDTH = 32


def layer_shapes(cin=CIN, width=WIDTH):
    return [((width, cin, 3, 3), (width,)), ((width, width, 3, 3), (width,)),
            ((width, width, 3, 3), (width,)), ((1, width, 3, 3), (1,))]


def n_params(cin=CIN, width=WIDTH):
    return sum(int(np.prod(w)) + int(np.prod(b)) for w, b in layer_shapes(cin, width)) + width


def unpack(theta, cin=CIN, width=WIDTH):
    """Flat vector -> ([(W1, b1), ..., (W4, b4)], u1) (views, float64)."""
    theta = np.asarray(theta, dtype=np.float64)
    out, k = [], 0
    for ws, bs in layer_shapes(cin, width):
        nw, nb = int(np.prod(ws)), int(np.prod(bs))
        out.append((theta[k:k + nw].reshape(ws), theta[k + nw:k + nw + nb].reshape(bs)))
        k += nw + nb
    u1 = theta[k:k + width]
    assert k + width == theta.size, "parameter vector has the wrong length"
    return out, u1


def pack(layers, u1):
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in layers] + [np.ravel(u1)])


def bf16_round(a):
    """Round to the nearest bfloat16 (ties to even) and return float64.

    A float32 keeps its top 16 bits; the discarded low half decides the rounding:
    above half an ulp rounds up, exactly half rounds to the even neighbour."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    low = u & 0xFFFF
    keep = u >> 16
    up = (low > 0x8000) | ((low == 0x8000) & ((keep & 1) == 1))
    keep = keep + up.astype(np.uint64)
    r = (keep << 16).astype(np.uint32).view(np.float32)
    return r.astype(np.float64).reshape(np.shape(a))


def init_params(seed, cin=CIN, width=WIDTH, out_scale=0.1, cond_scale=0.0):
    """Seeded initial parameters: uniform(-1, 1) * sqrt(3 / fan_in) weights, zero biases;
    the last layer is scaled by out_scale so that the first guess stays near phi^n; u1
    uniform(-1, 1) * cond_scale (drawn after the weights)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    layers = []
    for i, (ws, bs) in enumerate(layer_shapes(cin, width)):
        fan_in = ws[1] * 9
        w = rng.uniform(-1.0, 1.0, size=ws) * np.sqrt(3.0 / fan_in)
        if i == 3:
            w *= out_scale
        layers.append((w, np.zeros(bs)))
    u1 = rng.uniform(-1.0, 1.0, size=width) * cond_scale
    return pack(layers, u1)


def conv3x3(a, w, b):
    """z[o, y, x] = b[o] + sum_{c, dy, dx} w[o, c, dy, dx] a[c, (y+dy-1) % ny, (x+dx-1) % nx]."""
    cout = w.shape[0]
    ny, nx = a.shape[1:]
    z = np.empty((cout, ny, nx))
    z[:] = np.asarray(b)[:, None, None]
    for dy in range(3):
        for dx in range(3):
            # shifted[c, y, x] = a[c, y + dy - 1, x + dx - 1]
            shifted = np.roll(a, shift=(1 - dy, 1 - dx), axis=(1, 2))
            z += np.einsum("oc,cyx->oyx", w[:, :, dy, dx], shifted)
    return z


def conv3x3_adjoint_input(g, w):
    """Adjoint of conv3x3 in its input: da[c, y, x] = sum_{o, dy, dx} w[o, c, dy, dx] g[o, y-dy+1, x-dx+1]."""
    cin = w.shape[1]
    ny, nx = g.shape[1:]
    da = np.zeros((cin, ny, nx))
    for dy in range(3):
        for dx in range(3):
            shifted = np.roll(g, shift=(dy - 1, dx - 1), axis=(1, 2))
            da += np.einsum("oc,oyx->cyx", w[:, :, dy, dx], shifted)
    return da


def conv3x3_adjoint_weight(g, a):
    """dW[o, c, dy, dx] = sum_{y, x} g[o, y, x] a[c, y+dy-1, x+dx-1]."""
    dw = np.empty((g.shape[0], a.shape[0], 3, 3))
    for dy in range(3):
        for dx in range(3):
            shifted = np.roll(a, shift=(1 - dy, 1 - dx), axis=(1, 2))
            dw[:, :, dy, dx] = np.einsum("oyx,cyx->oc", g, shifted)
    return dw


def forward(theta, x, cond=0.0, round_weights=True, cin=CIN, width=WIDTH):
    """Network output y (ny, nx) at condition c = cond and the activations [a_0, ..., a_3]
    for the backward pass."""
    layers, u1 = unpack(theta, cin, width)
    acts = [np.asarray(x, dtype=np.float64)]
    a = acts[0]
    for i, (w, b) in enumerate(layers):
        wq = bf16_round(w) if round_weights else w
        z = conv3x3(a, wq, b + cond * u1 if i == 0 else b)
        if i < 3:
            a = np.tanh(z)
            acts.append(a)
        else:
            y = z[0]
    return y, acts


def loss(y, t):
    return float(np.mean((y - t) ** 2))


def backward(theta, acts, y, t, cond=0.0, round_weights=True, cin=CIN, width=WIDTH):
    """Gradient of loss(y, t) with respect to the flat parameters (rounded weights) for the
    forward pass at condition c = cond: d/du1 = c d/db1, as z_1 depends on b1 + c u1."""
    layers, _ = unpack(theta, cin, width)
    g = (2.0 / y.size) * (y - t)[None]          # dL/dz_4
    grads = [None] * 4
    for i in range(3, -1, -1):
        w, _ = layers[i]
        wq = bf16_round(w) if round_weights else w
        a_prev = acts[i]
        grads[i] = (conv3x3_adjoint_weight(g, a_prev), g.sum(axis=(1, 2)))
        if i > 0:
            da = conv3x3_adjoint_input(g, wq)
            g = da * (1.0 - a_prev ** 2)         # through tanh: a_prev = tanh(z_prev)
    return pack(grads, cond * grads[0][1])


def adam_step(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step number t >= 1); returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    theta = theta - lr * mhat / (np.sqrt(vhat) + eps)
    return theta, m, v


def step_scale(dt, dt_ref, beta, gamma):
    """g = exp(beta l + gamma l^2), l = ln(dt / dt_ref)."""
    l = float(np.log(dt / dt_ref))
    return float(np.exp(beta * l + gamma * l * l))


def make_input(phi_n, phi_nm1, ratio, s_a, s_b, g=1.0):
    """The two input planes of the definition above."""
    phi_n = np.asarray(phi_n, dtype=np.float64)
    x0 = (phi_n - phi_n.mean()) / s_a
    x1 = ratio * (phi_n - np.asarray(phi_nm1, dtype=np.float64)) / (s_b * g)
    return np.stack([x0, x1])


def condition(dt, dt_ref, s_c):
    """c = ln(dt / dt_ref) / s_c."""
    return float(np.log(dt / dt_ref) / s_c)


def guess(theta, phi_n, phi_nm1, ratio, dt, scales, dt_ref):
    """G = phi^n + s_o g y at c = ln(dt / dt_ref) / s_c, shifted to the mass of phi^n;
    scales = (s_a, s_b, s_o, s_c, beta, gamma)."""
    s_a, s_b, s_o, s_c, beta, gamma = scales
    g = step_scale(dt, dt_ref, beta, gamma)
    y, _ = forward(theta, make_input(phi_n, phi_nm1, ratio, s_a, s_b, g), condition(dt, dt_ref, s_c))
    G = np.asarray(phi_n, dtype=np.float64) + s_o * g * y
    return G + (np.mean(phi_n) - np.mean(G))
