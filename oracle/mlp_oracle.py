"""FP64 NumPy oracle of the surrogate network: forward, loss gradient and Adam.

TEST INFRASTRUCTURE ONLY: only the test suite may import it; the library's
HIP kernels share no code with it.

Network: u = 2 (x - lo) / (hi - lo) - 1; h_1 = silu(W_1 u + b_1);
h_k = silu(W_k h_{k-1} + b_k), k = 2..4; s = w_5 . h_4 + b_5;
y = y_mean + y_std s.  Loss L = mean_b (s_b - (y_b - y_mean) / y_std)^2.
Adam as published by Kingma & Ba (bias-corrected moments).
Parameter vector order: W1 (128x3), b1, W2, b2, W3, b3, W4, b4, w5 (1x128), b5.
"""
import numpy as np

SHAPES = [(128, 3), (128, 128), (128, 128), (128, 128), (1, 128)]
NPARAM = sum(o * i + o for o, i in SHAPES)


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    out, off = [], 0
    for o, i in SHAPES:
        Wm = p[off:off + o * i].reshape(o, i)
        off += o * i
        b = p[off:off + o]
        off += o
        out.append((Wm, b))
    assert off == NPARAM
    return out


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def _scaled_input(x, lo, hi):
    x = np.asarray(x, dtype=np.float64)
    return 2.0 * (x - np.asarray(lo)) / (np.asarray(hi) - np.asarray(lo)) - 1.0


def forward_s(p, x, lo, hi):
    """Standardised output s and the pre-activations / activations per layer."""
    layers = unpack(p)
    h = _scaled_input(x, lo, hi)
    hs, zs = [h], []
    for Wm, b in layers[:-1]:
        z = h @ Wm.T + b
        h = silu(z)
        zs.append(z)
        hs.append(h)
    Wm, b = layers[-1]
    s = (h @ Wm.T + b)[:, 0]
    return s, zs, hs


def forward(p, x, lo, hi, y_mean, y_std):
    return y_mean + y_std * forward_s(p, x, lo, hi)[0]


def loss_grad(p, x, y, lo, hi, y_mean, y_std):
    """Loss and its gradient (flat, parameter order) by the chain rule."""
    layers = unpack(p)
    s, zs, hs = forward_s(p, x, lo, hi)
    B = len(s)
    t = (np.asarray(y, dtype=np.float64) - y_mean) / y_std
    d = s - t
    loss = float(np.mean(d * d))
    ds = 2.0 * d / B                        # dL/ds
    grads = [None] * len(layers)
    Wm = layers[-1][0]
    grads[-1] = (ds[None, :] @ hs[-1], np.array([ds.sum()]))
    dh = ds[:, None] * Wm                   # dL/dh_4
    for k in range(len(layers) - 2, -1, -1):
        dz = dh * dsilu(zs[k])
        grads[k] = (dz.T @ hs[k], dz.sum(axis=0))
        dh = dz @ layers[k][0]
    flat = np.concatenate([np.concatenate([g.ravel(), gb.ravel()]) for g, gb in grads])
    return loss, flat


def adam(p, g, m, v, t, lr, b1, b2, eps):
    """One Adam update at step t (1-based); returns (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
