"""FP64 CPU oracle of the learned smoother: a three-layer 3x3 complex
convolutional network, its loss on (error, residual) pairs, the analytic
backward pass and one Adam step.

TEST INFRASTRUCTURE ONLY: the reference the HIP training and inference
kernels are checked against.  Only the tests, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import it; it shares no code with
the GPU library.

The paper smooths with weighted Jacobi (Sec. 4) and remarks that other
smoothers can take its place in the cycle; the learned smoother is such a
replacement, defined here (not in the paper):

  smoothing step      u <- u + s h^2 N(r / s, kappa h^2),  r = b - A u,
                      s = RMS of r over the grid, kappa = k0^2 + q
  network N           inputs r~ = r / s, kappa~ = kappa h^2
                      a  = W1[:, :, 0] * r~,  m = W1[:, :, 1] * kappa~
                      x1 = a (1 + m)                     (16 channels)
                      x2 = W2 * x1                       (16 channels)
                      N  = W3 * x2                       (1 channel)
                      N is complex-linear in r~ (a learned stencil of radius
                      3 whose weights the gate 1 + m adapts to the local
                      coefficient), so the smoothing step is a linear
                      iteration and N(0, kappa~) = 0.
  3x3 convolution     (W * x)_o(p) = sum_t sum_i W[t, o, i] x_i(p + d_t),
                      tap t = 3 (dy + 1) + (dx + 1), d_t = (dy, dx), zero
                      outside the array (the Dirichlet boundary)
  loss (one patch)    mean over the masked points of |L5 (e~ - N)|^2
                      + ALPHA max(0, ||e~ - N||^2 / ||e~||^2 - 1),
                      e~ = e / (s h^2), L5 d = 4 d - (the 4 neighbours),
                      norms over the masked points: the high-frequency part
                      of the error left after the smoothing step (the part a
                      smoother must remove), plus a penalty on any growth of
                      the patch's error, which keeps the step from amplifying
                      smooth error (L5 does not see it) without asking the
                      network to remove it.

Arrays are (channels, ny, nx), x fastest.  Complex gradients follow the
convention g = dL/dRe + i dL/dIm; then for y = W x:
  dL/dW = g_y conj(x),  g_x = conj(W) g_y.
"""
from __future__ import annotations

import numpy as np

C_IN, C_HID, C_OUT = 2, 16, 1
ALPHA = 1.0
SHAPES = ((9, C_HID, C_IN), (9, C_HID, C_HID), (9, C_OUT, C_HID))
TAPS = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def n_params() -> int:
    return sum(int(np.prod(s)) for s in SHAPES)


def bf16(a):
    """Round to the nearest BF16 (ties to even), real and imaginary parts
    separately, through float32."""
    a = np.asarray(a)
    if np.iscomplexobj(a):
        return bf16(a.real) + 1j * bf16(a.imag)
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return (u.astype(np.uint32).view(np.float32)).astype(np.float64)


def init_weights(seed: int):
    """He-style complex initialisation (variance 2 / fan-in over Re and Im)."""
    rng = np.random.default_rng(seed)
    Ws = []
    for s in SHAPES:
        fan_in = 9 * s[2]
        sd = np.sqrt(1.0 / fan_in)
        Ws.append(rng.normal(0.0, sd, s) + 1j * rng.normal(0.0, sd, s))
    return Ws


def shift(x, dy, dx):
    """y(p) = x(p + (dy, dx)) with zeros outside (last two axes)."""
    y = np.zeros_like(x)
    ny, nx = x.shape[-2:]
    ys, yd = (slice(0, ny - dy), slice(dy, ny)) if dy >= 0 else (slice(-dy, ny), slice(0, ny + dy))
    xs, xd = (slice(0, nx - dx), slice(dx, nx)) if dx >= 0 else (slice(-dx, nx), slice(0, nx + dx))
    y[..., ys, xs] = x[..., yd, xd]
    return y


def conv(W, x):
    """(W * x)_o = sum_t sum_i W[t, o, i] shift(x_i, d_t)."""
    out = np.zeros((W.shape[1],) + x.shape[1:], dtype=np.complex128)
    for t, (dy, dx) in enumerate(TAPS):
        xs = shift(x, dy, dx)
        out += np.tensordot(W[t], xs, axes=([1], [0]))
    return out


def conv_backward(W, x, g):
    """Gradients of a real loss through y = W * x: (dW, g_x)."""
    dW = np.zeros_like(W)
    gx = np.zeros_like(x, dtype=np.complex128)
    for t, (dy, dx) in enumerate(TAPS):
        xs = shift(x, dy, dx)
        dW[t] = np.tensordot(g, np.conj(xs), axes=([1, 2], [1, 2]))
        # y(p) uses x(p + d): the gradient flows back to q = p + d
        gx += shift(np.tensordot(np.conj(W[t]).T, g, axes=([1], [0])), -dy, -dx)
    return dW, gx


def forward(Ws, rt, kt, quant=False):
    """Activations (x0r, x0k, a, m, x1, x2, y).  quant: weights and the layer
    inputs rounded to BF16 (the GPU kernels' storage precision)."""
    W1, W2, W3 = (bf16(W) for W in Ws) if quant else Ws
    q = bf16 if quant else (lambda z: z)
    x0r, x0k = q(rt)[None], q(kt)[None]
    a = conv(W1[:, :, 0:1], x0r)
    m = conv(W1[:, :, 1:2], x0k)
    x1 = q(a * (1.0 + m))
    x2 = q(conv(W2, x1))
    y = conv(W3, x2)[0]
    return x0r, x0k, a, m, x1, x2, y


def lap5(d):
    """4 d(p) - sum of the 4 neighbours (zeros outside)."""
    return 4.0 * d - shift(d, 0, 1) - shift(d, 0, -1) - shift(d, 1, 0) - shift(d, -1, 0)


def loss_and_grad_y(y, et, mask):
    d = et - y
    z = lap5(d) * mask
    cnt = float(mask.sum())
    E = float(np.sum(np.abs(et) ** 2 * mask))
    D = float(np.sum(np.abs(d) ** 2 * mask))
    L = float(np.sum(np.abs(z) ** 2) / cnt)
    gy = -lap5(2.0 * z) / cnt
    if E > 0.0 and D > E:
        L += ALPHA * (D / E - 1.0)
        gy = gy - 2.0 * ALPHA * mask * d / E
    return L, gy


def loss_and_grads(Ws, rt, kt, et, mask, quant=False):
    """Loss of one patch and dL/dW for W1, W2, W3 (analytic backward)."""
    x0r, x0k, a, m, x1, x2, y = forward(Ws, rt, kt, quant)
    W1, W2, W3 = (bf16(W) for W in Ws) if quant else Ws
    L, gy = loss_and_grad_y(y, et, mask)
    dW3, gx2 = conv_backward(W3, x2, gy[None])
    dW2, gx1 = conv_backward(W2, x1, gx2)
    # x1 = a c with c = 1 + m: g_a = conj(c) g_x1, g_m = conj(a) g_x1
    ga = np.conj(1.0 + m) * gx1
    gm = np.conj(a) * gx1
    dW1a, _ = conv_backward(W1[:, :, 0:1], x0r, ga)
    dW1m, _ = conv_backward(W1[:, :, 1:2], x0k, gm)
    dW1 = np.concatenate([dW1a, dW1m], axis=2)
    return L, [dW1, dW2, dW3]


def interior_mask(ny, nx, border=4):
    m = np.zeros((ny, nx))
    m[border:ny - border, border:nx - border] = 1.0
    return m


def adam_step(Ws, grads, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step on the real and imaginary parts separately (step >= 1)."""
    out = []
    for i, (W, g) in enumerate(zip(Ws, grads)):
        gr = np.stack([g.real, g.imag])
        m[i] = beta1 * m[i] + (1.0 - beta1) * gr
        v[i] = beta2 * v[i] + (1.0 - beta2) * gr * gr
        mh = m[i] / (1.0 - beta1 ** step)
        vh = v[i] / (1.0 - beta2 ** step)
        upd = lr * mh / (np.sqrt(vh) + eps)
        out.append(W - (upd[0] + 1j * upd[1]))
    return out


def smooth_step(Ws, r, kappa_h2, h2, quant=False):
    """The learned smoothing update s h^2 N(r / s, kappa h^2) on a whole grid
    (s = RMS of r)."""
    s = float(np.sqrt(np.mean(np.abs(r) ** 2)))
    if s == 0.0:
        return np.zeros_like(r)
    return s * h2 * forward(Ws, r / s, kappa_h2, quant)[-1]
