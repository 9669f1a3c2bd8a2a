"""Pins of the FP64 oracle of the surrogate network (CPU only).

The oracle's gradient is pinned by central finite differences of its own
loss (the definition of the derivative), its forward pass by hand-built
networks whose output is a closed form that a transposed or misplaced weight
would change, and its Adam step by the closed form of the first step.
"""
import numpy as np
import pytest

from oracle import mlp_oracle as mo
from paper_1905_00141_amd import synth

LO = np.log([0.25, 0.02, 1e-3])
HI = np.log([4.0, 0.3, 1e-1])


def _batch(seed, B):
    rng = np.random.default_rng(seed)
    x = LO + rng.random((B, 3)) * (HI - LO)
    y = 3.0 + 2.0 * np.sin(x[:, 0]) - x[:, 1] ** 2 + 0.5 * x[:, 2]
    return x, y


def test_parameter_count():
    assert mo.NPARAM == 50177 == len(synth.mlp_init(0))


def test_silu_and_its_derivative():
    z = np.linspace(-6, 6, 101)
    np.testing.assert_allclose(mo.silu(z), z * (1 / (1 + np.exp(-z))), rtol=1e-15)
    h = 1e-6
    np.testing.assert_allclose(mo.dsilu(z), (mo.silu(z + h) - mo.silu(z - h)) / (2 * h), rtol=1e-8, atol=1e-9)


def test_hand_built_network_closed_form():
    """One active path: input 2 -> unit 5 -> unit 7 -> unit 1 -> unit 9 -> output."""
    p = np.zeros(mo.NPARAM)
    L = mo.unpack(p)  # views into a float64 copy: rebuild p from the pieces
    W1, b1 = np.zeros((128, 3)), np.zeros(128)
    W2, W3, W4 = np.zeros((128, 128)), np.zeros((128, 128)), np.zeros((128, 128))
    w5 = np.zeros((1, 128))
    W1[5, 2] = 0.7; b1[5] = 0.1
    W2[7, 5] = -1.3
    W3[1, 7] = 0.9
    W4[9, 1] = 2.0
    w5[0, 9] = 1.5
    b5 = np.array([0.25])
    p = np.concatenate([W1.ravel(), b1, W2.ravel(), np.zeros(128), W3.ravel(), np.zeros(128), W4.ravel(),
                        np.zeros(128), w5.ravel(), b5])
    assert len(p) == mo.NPARAM and len(L) == 5
    x = np.array([[0.1, -2.0, -4.0], [1.0, -3.0, -2.5]])
    u2 = 2 * (x[:, 2] - LO[2]) / (HI[2] - LO[2]) - 1
    s = 1.5 * mo.silu(2.0 * mo.silu(0.9 * mo.silu(-1.3 * mo.silu(0.7 * u2 + 0.1)))) + 0.25
    np.testing.assert_allclose(mo.forward(p, x, LO, HI, 10.0, 3.0), 10.0 + 3.0 * s, rtol=1e-15)


def test_gradient_matches_central_differences():
    x, y = _batch(1, 64)
    p = synth.mlp_init(3).astype(np.float64)
    p[mo.NPARAM - 129:] *= 3.0  # larger output weights: every layer's gradient well above rounding
    ym, ys = y.mean(), y.std()
    _, g = mo.loss_grad(p, x, y, LO, HI, ym, ys)
    rng = np.random.default_rng(0)
    # a sample of every tensor: W1, b1, W2..W4, b2..b4, w5, b5
    bounds = np.cumsum([0] + [s for o, i in mo.SHAPES for s in (o * i, o)])
    idx = np.concatenate([rng.choice(np.arange(a, b), size=min(6, b - a), replace=False)
                          for a, b in zip(bounds[:-1], bounds[1:])])
    h = 1e-6
    for k in idx:
        pp, pm = p.copy(), p.copy()
        pp[k] += h; pm[k] -= h
        fd = (mo.loss_grad(pp, x, y, LO, HI, ym, ys)[0] - mo.loss_grad(pm, x, y, LO, HI, ym, ys)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(abs(g).max(), 1e-12) + 1e-7 * abs(g[k]), (k, fd, g[k])


def test_zero_residual_gives_zero_gradient():
    x, _ = _batch(2, 16)
    p = synth.mlp_init(4).astype(np.float64)
    y = mo.forward(p, x, LO, HI, 1.0, 2.0)
    loss, g = mo.loss_grad(p, x, y, LO, HI, 1.0, 2.0)
    assert loss < 1e-28 and np.abs(g).max() < 1e-13


def test_first_adam_step_closed_form():
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    p = np.array([1.0, 2.0, 3.0, 4.0])
    lr, eps = 1e-2, 1e-8
    p1, m, v = mo.adam(p, g, np.zeros(4), np.zeros(4), 1, lr, 0.9, 0.999, eps)
    np.testing.assert_allclose(p1, p - lr * g / (np.abs(g) + eps), rtol=1e-13)
    # second step with the same gradient: the bias-corrected moments are still g and g^2
    p2, _, _ = mo.adam(p1, g, m, v, 2, lr, 0.9, 0.999, eps)
    np.testing.assert_allclose(p2, p1 - lr * g / (np.abs(g) + eps), rtol=1e-12)


def test_training_fits_a_smooth_function():
    """Full-batch Adam on the oracle drives the loss down on a smooth target."""
    x, y = _batch(5, 256)
    p = synth.mlp_init(6).astype(np.float64)
    m, v = np.zeros_like(p), np.zeros_like(p)
    ym, ys = y.mean(), y.std()
    l0 = mo.loss_grad(p, x, y, LO, HI, ym, ys)[0]
    for t in range(1, 301):
        loss, g = mo.loss_grad(p, x, y, LO, HI, ym, ys)
        p, m, v = mo.adam(p, g, m, v, t, 3e-3, 0.9, 0.999, 1e-8)
    assert loss < 0.02 * l0, (l0, loss)
