"""GPU parity of the surrogate network's FP32 kernels (through the C ABI)
against the FP64 oracle.

Tolerances follow FP32 arithmetic: inner products of length <= 2048 in FP32
carry relative errors of order sqrt(K) * 6e-8 of the sum of |terms|, so
outputs are held to 2e-5 of their scale and gradients to 1e-4 of the largest
gradient entry of their tensor.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

LO = np.log([0.25, 0.02, 1e-3])
HI = np.log([4.0, 0.3, 1e-1])


@pytest.fixture(scope="module")
def mra():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1905_00141_amd import mra as m
    return m


@pytest.fixture(scope="module")
def mo():
    from oracle import mlp_oracle
    return mlp_oracle


def _batch(seed, B):
    rng = np.random.default_rng(seed)
    x = LO + rng.random((B, 3)) * (HI - LO)
    y = 3.0 + 2.0 * np.sin(x[:, 0]) - x[:, 1] ** 2 + 0.5 * x[:, 2]
    return x.astype(np.float32), y


def _net(mra, seed, ym, ys):
    from paper_1905_00141_amd import synth
    p = synth.mlp_init(seed)
    p[-129:] *= 3.0
    net = mra.Mlp(p)
    net.set_scaling(LO, HI, ym, ys)
    return net, p


@pytest.mark.parametrize("B", [1, 7, 64, 1000, 2048])
def test_forward_matches_oracle(mra, mo, B):
    x, y = _batch(B, B)
    net, p = _net(mra, 11, 5.0, 2.0)
    got = net.forward(x)
    ref = mo.forward(p.astype(np.float64), x.astype(np.float64), LO, HI, 5.0, 2.0)
    s_ref = (ref - 5.0) / 2.0
    assert np.all(np.abs(got - ref) <= 2.0 * 2e-5 * (1.0 + np.abs(s_ref))), np.abs(got - ref).max()


def test_forward_large_batch_chunks(mra, mo):
    x, _ = _batch(3, 70000)  # more than one 65536-row chunk
    net, p = _net(mra, 12, 0.0, 1.0)
    got = net.forward(x)
    idx = np.r_[0:50, 65530:65542, 69950:70000]
    ref = mo.forward(p.astype(np.float64), x[idx].astype(np.float64), LO, HI, 0.0, 1.0)
    assert np.all(np.abs(got[idx] - ref) <= 2e-5 * (1.0 + np.abs(ref)))


@pytest.mark.parametrize("B", [5, 300, 2048])
def test_loss_and_gradient_match_oracle(mra, mo, B):
    x, y = _batch(100 + B, B)
    ym, ys = float(y.mean()), float(y.std())
    net, p = _net(mra, 13, ym, ys)
    loss, g = net.loss_grad(x, y)
    lref, gref = mo.loss_grad(p.astype(np.float64), x.astype(np.float64), y, LO, HI, ym, ys)
    assert abs(loss[0] - lref) <= 2e-5 * lref
    bounds = np.cumsum([0] + [s for o, i in mo.SHAPES for s in (o * i, o)])
    for a, b in zip(bounds[:-1], bounds[1:]):
        scale = np.abs(gref[a:b]).max()
        assert np.abs(g[a:b] - gref[a:b]).max() <= 1e-4 * scale + 1e-12, (a, b, np.abs(g[a:b] - gref[a:b]).max(), scale)


def test_device_pointers_and_determinism(mra, mo):
    import torch
    x, y = _batch(7, 512)
    net, p = _net(mra, 14, float(y.mean()), float(y.std()))
    dev = torch.device("cuda:0")
    xd, yd = torch.tensor(x, device=dev), torch.tensor(y, device=dev)
    s = torch.cuda.Stream()
    l1, g1 = net.loss_grad(xd, yd, stream=s)
    s.synchronize()
    l2, g2 = net.loss_grad(x, y)
    assert np.array_equal(g1.cpu().numpy(), g2) and l1.item() == l2[0]
    f1 = net.forward(xd).cpu().numpy()
    assert np.array_equal(f1, net.forward(x))


def test_adam_steps_match_oracle(mra, mo):
    """Ten full-batch Adam steps on the GPU and in the oracle from the same
    start.  Adam normalises each step to about lr, so a gradient entry whose
    FP32 error flips its sign can move its parameter by up to 2 lr per step;
    entries away from zero agree far more closely."""
    x, y = _batch(8, 1024)
    ym, ys = float(y.mean()), float(y.std())
    net, p0 = _net(mra, 15, ym, ys)
    p = p0.astype(np.float64)
    m, v = np.zeros_like(p), np.zeros_like(p)
    lr, steps = 1e-3, 10
    for t in range(1, steps + 1):
        net.train_step(x, y, lr=lr)
        _, g = mo.loss_grad(p, x.astype(np.float64), y, LO, HI, ym, ys)
        p, m, v = mo.adam(p, g, m, v, t, lr, 0.9, 0.999, 1e-8)
    got = net.params().astype(np.float64)
    d = np.abs(got - p)
    assert d.max() <= 2 * lr * steps
    assert np.quantile(d, 0.99) <= 1e-2 * lr * steps, np.quantile(d, 0.99)


def test_training_reduces_loss(mra):
    x, y = _batch(9, 2048)
    net, _ = _net(mra, 16, float(y.mean()), float(y.std()))
    l0 = net.loss_grad(x, y)[0][0]
    for _ in range(400):
        loss = net.train_step(x, y, lr=3e-3)[0]
    assert loss < 0.01 * l0, (l0, loss)


def test_errors(mra):
    with pytest.raises(ValueError):
        mra.Mlp(np.zeros(10, dtype=np.float32))
    net = mra.Mlp(np.zeros(mra.MLP_NPARAM, dtype=np.float32))
    with pytest.raises(mra.MraError):
        net.set_scaling([0, 0, 0], [1, 1, 0], 0.0, 1.0)
    with pytest.raises(mra.MraError):
        net.set_scaling([0, 0, 0], [1, 1, 1], 0.0, 0.0)
    x, y = _batch(1, 4)
    with pytest.raises(mra.MraError):
        net.train_step(x, y, lr=-1.0)
