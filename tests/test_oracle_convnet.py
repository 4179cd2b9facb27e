"""Pins of the learned-smoother oracle (oracle/convnet.py) against facts
that do not come from its own code: finite differences, brute-force loops,
a closed-form linear construction (weighted Jacobi), the eigenvalues of the
5-point Laplacian, textbook properties of Adam and the BF16 conversion of a
library.  CPU only."""
import math

import numpy as np
import pytest

from oracle import convnet as cn


def rnd(seed, shape):
    r = np.random.default_rng(seed)
    return r.standard_normal(shape) + 1j * r.standard_normal(shape)


def test_parameter_count():
    # 3x3 taps: 2 -> 16, 16 -> 16, 16 -> 1 complex channels
    assert cn.n_params() == 9 * (16 * 2 + 16 * 16 + 16) == 2736


def test_gradients_match_central_differences():
    ny, nx = 10, 12
    Ws = cn.init_weights(3)
    rt, kt, et = rnd(1, (ny, nx)), rnd(2, (ny, nx)) * 0.3, rnd(4, (ny, nx))
    mask = cn.interior_mask(ny, nx, border=2)
    L0, grads = cn.loss_and_grads(Ws, rt, kt, et, mask)
    rng = np.random.default_rng(9)
    eps = 1e-6
    worst = 0.0
    for li, W in enumerate(Ws):
        gscale = np.max(np.abs(grads[li]))
        for _ in range(12):
            idx = tuple(rng.integers(0, s) for s in W.shape)
            for part, unit in ((0, 1.0), (1, 1j)):
                Wp = [w.copy() for w in Ws]
                Wm = [w.copy() for w in Ws]
                Wp[li][idx] += eps * unit
                Wm[li][idx] -= eps * unit
                fd = (cn.loss_and_grads(Wp, rt, kt, et, mask)[0] - cn.loss_and_grads(Wm, rt, kt, et, mask)[0]) / (2 * eps)
                an = grads[li][idx].real if part == 0 else grads[li][idx].imag
                worst = max(worst, abs(fd - an) / gscale)
    assert worst < 1e-6, worst


def test_gradients_with_growth_penalty_match_central_differences():
    """Large weights make the step amplify the patch error, so the growth
    penalty is active."""
    ny, nx = 10, 12
    Ws = [W * 3.0 for W in cn.init_weights(4)]
    rt, kt, et = rnd(1, (ny, nx)), rnd(2, (ny, nx)) * 0.3, rnd(4, (ny, nx)) * 0.01
    mask = cn.interior_mask(ny, nx, border=2)
    x = cn.forward(Ws, rt, kt)
    d = et - x[-1]
    assert np.sum(np.abs(d) ** 2 * mask) > np.sum(np.abs(et) ** 2 * mask)
    L0, grads = cn.loss_and_grads(Ws, rt, kt, et, mask)
    rng = np.random.default_rng(10)
    eps = 1e-6
    for li, W in enumerate(Ws):
        gscale = np.max(np.abs(grads[li]))
        for _ in range(6):
            idx = tuple(rng.integers(0, s) for s in W.shape)
            Wp = [w.copy() for w in Ws]
            Wm = [w.copy() for w in Ws]
            Wp[li][idx] += eps
            Wm[li][idx] -= eps
            fd = (cn.loss_and_grads(Wp, rt, kt, et, mask)[0] - cn.loss_and_grads(Wm, rt, kt, et, mask)[0]) / (2 * eps)
            assert abs(fd - grads[li][idx].real) < 1e-5 * gscale


def test_tap_orientation_brute_force():
    ny, nx = 5, 6
    x = rnd(5, (2, ny, nx))
    for t, (dy, dx) in enumerate(cn.TAPS):
        W = np.zeros(cn.SHAPES[0], dtype=np.complex128)
        W[t, 3, 1] = 2.0 - 1.0j
        y = cn.conv(W, x)
        for j in range(ny):
            for i in range(nx):
                jj, ii = j + dy, i + dx
                src = x[1, jj, ii] if 0 <= jj < ny and 0 <= ii < nx else 0.0
                assert y[3, j, i] == (2.0 - 1.0j) * src
                assert np.all(y[np.arange(16) != 3, j, i] == 0)


def jacobi_weights(c):
    """Weights with N(r~, kappa~) = c r~ exactly: the centre taps pass r~
    through channel 0 (gate 1 + 0) and layer 3 scales it by c."""
    W1 = np.zeros(cn.SHAPES[0], dtype=np.complex128)
    W2 = np.zeros(cn.SHAPES[1], dtype=np.complex128)
    W3 = np.zeros(cn.SHAPES[2], dtype=np.complex128)
    W1[4, 0, 0] = 1.0
    W2[4, 0, 0] = 1.0
    W3[4, 0, 0] = c
    return [W1, W2, W3]


def test_network_is_complex_linear_in_the_residual():
    """N(alpha r~ + beta r2~, kappa~) = alpha N(r~) + beta N(r2~) for complex
    alpha, beta, and N(0, kappa~) = 0."""
    Ws = cn.init_weights(21)
    r1, r2, k = rnd(1, (9, 10)), rnd(2, (9, 10)), rnd(3, (9, 10)) * 0.2
    al, be = 0.3 - 1.7j, -2.1 + 0.4j
    N = lambda r: cn.forward(Ws, r, k)[-1]
    np.testing.assert_allclose(N(al * r1 + be * r2), al * N(r1) + be * N(r2), rtol=1e-12, atol=1e-12)
    assert np.all(N(np.zeros_like(r1)) == 0)


def test_linear_construction_is_weighted_jacobi():
    """With constant kappa, weighted Jacobi (Sec. 4) adds omega r / D, D the
    diagonal of the contour operator of eq. csg: e^{-2 i gamma} 4 / h^2 - kappa.
    The network with the weights above reproduces it."""
    gamma, h, omega = math.pi / 6, 0.05, 0.8
    kappa = 4.0 + 0.3j
    D = np.exp(-2j * gamma) * 4.0 / h ** 2 - kappa
    r = rnd(6, (9, 11))
    c = omega / (D * h * h)
    upd = cn.smooth_step(jacobi_weights(c), r, np.full(r.shape, kappa * h * h), h * h)
    np.testing.assert_allclose(upd, omega * r / D, rtol=1e-13, atol=0)


def test_lap5_sine_eigenvalues():
    """Dirichlet sine modes are eigenvectors of the 5-point Laplacian:
    lambda = 4 - 2 cos(pi a / (nx + 1)) - 2 cos(pi b / (ny + 1))."""
    ny, nx, a, b = 9, 13, 3, 5
    j, i = np.meshgrid(np.arange(1, ny + 1), np.arange(1, nx + 1), indexing="ij")
    d = np.sin(math.pi * a * i / (nx + 1)) * np.sin(math.pi * b * j / (ny + 1)) * (1 + 2j)
    lam = 4 - 2 * math.cos(math.pi * a / (nx + 1)) - 2 * math.cos(math.pi * b / (ny + 1))
    np.testing.assert_allclose(cn.lap5(d), lam * d, rtol=0, atol=1e-13)
    mask = cn.interior_mask(ny, nx, border=2)
    L, gy = cn.loss_and_grad_y(np.zeros_like(d), d, mask)
    assert abs(L - lam ** 2 * np.sum(np.abs(d) ** 2 * mask) / mask.sum()) < 1e-12
    # an output that doubles the error: the growth penalty adds ALPHA (4 - 1)
    L2, _ = cn.loss_and_grad_y(-d, d, mask)
    assert abs(L2 - (4 * lam ** 2 * np.sum(np.abs(d) ** 2 * mask) / mask.sum() + 3 * cn.ALPHA)) < 1e-10


def test_adam_first_step_is_sign_descent():
    """After bias correction the first Adam step is lr g / (|g| + eps)."""
    Ws = [rnd(7, (3, 2, 2))]
    g = [rnd(8, (3, 2, 2))]
    m = [np.zeros((2,) + Ws[0].shape)]
    v = [np.zeros((2,) + Ws[0].shape)]
    lr = 1e-3
    out = cn.adam_step(Ws, g, m, v, 1, lr, eps=1e-12)
    exp = Ws[0] - lr * (np.sign(g[0].real) + 1j * np.sign(g[0].imag))
    np.testing.assert_allclose(out[0], exp, rtol=0, atol=1e-12)


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    x = np.concatenate([np.random.default_rng(3).standard_normal(4000) * 10.0 ** np.arange(-20, 20, 0.01),
                        [1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -8), 0.0, 3e38]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(cn.bf16(x), ref)
    assert cn.bf16(np.array([1 + 2 ** -8]))[0] == 1.0
    assert cn.bf16(np.array([1 + 3 * 2 ** -8]))[0] == 1 + 2 ** -6
