"""Pins of the oracle's kriging (prediction mode): textbook simple kriging at
M = 1, the two-level closed form, the recursion against the dense definition,
and invariants of the posterior."""
import numpy as np
import pytest

from oracle.oracle import MATERN, OracleError, Tree
from paper_1905_00141_amd import synth


def _cov_np(d, alpha, beta, nu):
    t = d / beta
    return alpha * np.exp(-t) if nu == 0.5 else alpha * (1.0 + t) * np.exp(-t)


def _dist(ax, ay, bx, by):
    return np.hypot(ax[:, None] - bx[None, :], ay[:, None] - by[None, :])


def _krige(Sss, Sps, spp, z, tau):
    K = Sss + tau * np.eye(len(z))
    mean = Sps @ np.linalg.solve(K, z)
    var = spp - np.einsum("ij,ji->i", Sps, np.linalg.solve(K, Sps.T))
    return mean, var


@pytest.mark.parametrize("nu", [0.5, 1.5])
def test_M1_is_simple_kriging(nu):
    rng = np.random.default_rng(3)
    n = 250
    x, y, z = rng.random(n), rng.random(n), rng.standard_normal(n)
    px, py = rng.random(40), rng.random(40)
    th = (1.4, 0.15, 0.02)
    t = Tree(x, y, z, J=4, r=16, M=1, domain=[0, 1, 0, 1])
    a = t.arrays()
    Sss = _cov_np(_dist(a["x"], a["y"], a["x"], a["y"]), th[0], th[1], nu)
    Sps = _cov_np(_dist(px, py, a["x"], a["y"]), th[0], th[1], nu)
    rm, rv = _krige(Sss, Sps, np.full(40, th[0]), a["z"], th[2])
    m, v = t.predict(th, px, py, MATERN, nu)
    np.testing.assert_allclose(m, rm, rtol=0, atol=1e-11)
    np.testing.assert_allclose(v, rv, rtol=0, atol=1e-11)


def _grid_knots_np(box, r, f=np.e / 100):
    nx = int(np.ceil(np.sqrt(r)))
    ny = r // nx
    L, H = box[1] - box[0], box[3] - box[2]
    xb = box[0] + f * L + np.arange(nx) * L * (1 - 2 * f) / (nx - 1)
    yb = box[2] + f * H + np.arange(ny) * H * (1 - 2 * f) / (ny - 1)
    X, Y = np.meshgrid(xb, yb)
    return X.ravel(), Y.ravel()


@pytest.mark.parametrize("nu", [0.5, 1.5])
def test_M2_closed_form_prediction(nu):
    """Two levels: Sigma(a,b) = C(a,b) for a, b in the same leaf, otherwise
    C(a,Q) C(Q,Q)^{-1} C(Q,b); a prediction point joins its leaf."""
    rng = np.random.default_rng(4)
    n = 220
    x, y, z = rng.random(n), rng.random(n), rng.standard_normal(n)
    px, py = rng.random(30), rng.random(30)
    th = (0.9, 0.25, 0.05)
    dom = [0.0, 1.0, 0.0, 1.0]
    t = Tree(x, y, z, J=4, r=16, M=2, domain=dom)
    a = t.arrays()
    qx, qy = _grid_knots_np(dom, 16)
    allx, ally = np.concatenate([a["x"], px]), np.concatenate([a["y"], py])
    Cqq = _cov_np(_dist(qx, qy, qx, qy), th[0], th[1], nu)
    Caq = _cov_np(_dist(allx, ally, qx, qy), th[0], th[1], nu)
    low = Caq @ np.linalg.solve(Cqq, Caq.T)
    leaf = (allx >= 0.5).astype(int) + 2 * (ally >= 0.5).astype(int)
    S = np.where(leaf[:, None] == leaf[None, :], _cov_np(_dist(allx, ally, allx, ally), th[0], th[1], nu), low)
    rm, rv = _krige(S[:n, :n], S[n:, :n], np.diag(S)[n:], a["z"], th[2])
    m, v = t.predict(th, px, py, MATERN, nu)
    np.testing.assert_allclose(m, rm, rtol=0, atol=1e-11)
    np.testing.assert_allclose(v, rv, rtol=0, atol=1e-11)
    md, vd = t.predict(th, px, py, MATERN, nu, dense=True)
    np.testing.assert_allclose(md, rm, rtol=0, atol=1e-11)
    np.testing.assert_allclose(vd, rv, rtol=0, atol=1e-11)


CASES = [(4, 3, 9, 500, True, 0.5), (4, 4, 16, 700, True, 1.5), (2, 4, 16, 500, False, 1.5), (4, 3, 30, 600, False, 0.5)]


@pytest.mark.parametrize("J,M,r,n,cluster,nu", CASES)
def test_recursion_matches_dense_prediction(J, M, r, n, cluster, nu):
    c = synth.small_case(200 + M, n, J=J, r=r, M=M, cluster=cluster)
    t = Tree(c["x"], c["y"], c["z"], J=J, r=r, M=M, domain=[0, 1, 0, 1])
    rng = np.random.default_rng(9)
    px, py = rng.random(60), rng.random(60)
    for th in [(1.0, 0.05, 0.05), (2.0, 0.3, 0.001)]:
        m, v = t.predict(th, px, py, MATERN, nu)
        md, vd = t.predict(th, px, py, MATERN, nu, dense=True)
        scale = np.abs(md).max() + 1.0
        np.testing.assert_allclose(m, md, rtol=0, atol=1e-10 * scale)
        np.testing.assert_allclose(v, vd, rtol=0, atol=1e-10 * th[0])


def test_posterior_variance_bounds_and_interpolation():
    c = synth.small_case(7, 400, M=3, r=16)
    th = (1.3, 0.1, 1e-9)
    t = Tree(c["x"], c["y"], c["z"], J=4, r=16, M=3, domain=[0, 1, 0, 1])
    a = t.arrays()
    rng = np.random.default_rng(2)
    px, py = rng.random(50), rng.random(50)
    m, v = t.predict(th, px, py)
    assert np.all(v <= th[0] + 1e-12) and np.all(v >= -1e-12)
    # at observed locations with a vanishing nugget the predictor interpolates
    mo, vo = t.predict(th, a["x"][:20], a["y"][:20])
    np.testing.assert_allclose(mo, a["z"][:20], atol=1e-5)
    assert np.all(np.abs(vo) < 1e-5)


def test_prediction_outside_root_is_an_error():
    c = synth.small_case(8, 100, M=2)
    t = Tree(c["x"], c["y"], c["z"], J=4, r=9, M=2, domain=[0, 1, 0, 1])
    with pytest.raises(OracleError):
        t.predict((1, 0.1, 0.1), np.array([1.5]), np.array([0.5]))
