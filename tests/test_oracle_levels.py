"""Pins of the oracle's per-level sums, its subtree evaluation, duplicate
elimination and the zero-nugget option.

Per-level sums (level_sums) and the subtree sums (oracle_mra_subtree, the work
the benchmark's CPU baseline times) are outputs the likelihood alone does not
check: a wrong ancestor index in the subtree path or a term booked at the wrong
level would leave the total unchanged.  They are pinned here by the identity
that they partition the total, by a two-level closed form written in NumPy
from the definitions of Sec. 1.1, and by sums over every subtree of a level.
"""
import numpy as np
import pytest

from oracle.oracle import (ALLOW_ZERO_NUGGET, ELIM_DUPLICATES, MATERN, OracleError, Tree,
                           subtree_du)
from paper_1905_00141_amd import synth

LOG2PI = np.log(2 * np.pi)


def _cov_np(d, alpha, beta, nu):
    t = d / beta
    return alpha * np.exp(-t) if nu == 0.5 else alpha * (1.0 + t) * np.exp(-t)


def _dist(ax, ay, bx, by):
    return np.hypot(ax[:, None] - bx[None, :], ay[:, None] - by[None, :])


def _grid_knots_np(box, r, f=np.e / 100):
    nx = int(np.ceil(np.sqrt(r)))
    while (nx - 1) * (nx - 1) >= r:
        nx -= 1
    ny = r // nx
    L, H = box[1] - box[0], box[3] - box[2]
    xb = box[0] + f * L + np.arange(nx) * L * (1 - 2 * f) / (nx - 1)
    yb = box[2] + f * H + np.arange(ny) * H * (1 - 2 * f) / (ny - 1)
    X, Y = np.meshgrid(xb, yb)
    return X.ravel(), Y.ravel()


def _logdet_quad(K, z):
    L = np.linalg.cholesky(K)
    y = np.linalg.solve(L, z)
    return 2.0 * np.log(np.diag(L)).sum(), float(y @ y)


@pytest.mark.parametrize("J,M,r,n,cluster,nu", [(4, 3, 16, 700, True, 0.5), (4, 4, 9, 900, False, 1.5),
                                                (2, 5, 4, 500, True, 1.5)])
def test_level_sums_partition_the_total(J, M, r, n, cluster, nu):
    c = synth.small_case(500 + n, n, J=J, r=r, M=M, cluster=cluster, nu=nu)
    t = Tree(c["x"], c["y"], c["z"], J=J, r=r, M=M)
    th = np.array([[1.0, 0.1, 0.02], [2.0, 0.03, 0.1]])
    ll, ls = t.loglik(th, MATERN, nu, level_sums=True)
    total = -2.0 * ll - t.n_used * LOG2PI
    np.testing.assert_allclose(ls.sum(axis=1), total, rtol=1e-12)


@pytest.mark.parametrize("nu", [0.5, 1.5])
def test_level_sums_two_level_closed_form(nu):
    """M = 2 with Q the root knots.  Level 2: every leaf's log det + quadratic
    form under its remainder C_2(S,S) + tau I, C_2 = C - C(S,Q) C(Q,Q)^{-1} C(Q,S).
    Level 1: the rest of the log-density of the data under Sigma_MRA + tau I."""
    rng = np.random.default_rng(17)
    n = 300
    x, y, z = rng.random(n), rng.random(n), rng.standard_normal(n)
    dom = [0.0, 1.0, 0.0, 1.0]
    th = (1.4, 0.15, 0.03)
    t = Tree(x, y, z, J=4, r=16, M=2, domain=dom)
    a = t.arrays()
    sx, sy, sz = a["x"], a["y"], a["z"]
    qx, qy = _grid_knots_np(dom, 16)
    Cqq = _cov_np(_dist(qx, qy, qx, qy), th[0], th[1], nu)
    Csq = _cov_np(_dist(sx, sy, qx, qy), th[0], th[1], nu)
    Css = _cov_np(_dist(sx, sy, sx, sy), th[0], th[1], nu)
    low = Csq @ np.linalg.solve(Cqq, Csq.T)
    leaf = (sx >= 0.5).astype(int) + 2 * (sy >= 0.5).astype(int)
    lev2 = 0.0
    for k in range(4):
        s = leaf == k
        if s.any():
            K = (Css - low)[np.ix_(s, s)] + th[2] * np.eye(int(s.sum()))
            d, q = _logdet_quad(K, sz[s])
            lev2 += d + q
    same = leaf[:, None] == leaf[None, :]
    Sig = np.where(same, Css, low) + th[2] * np.eye(n)
    d, q = _logdet_quad(Sig, sz)
    _, ls = t.loglik(th, MATERN, nu, level_sums=True)
    assert abs(ls[0, 1] - lev2) <= 1e-10 * abs(lev2)
    assert abs(ls[0, 0] - (d + q - lev2)) <= 1e-10 * abs(d + q)


@pytest.mark.parametrize("J,M", [(4, 4), (2, 5)])
def test_subtree_sums(J, M):
    """The subtree of the root is the whole evaluation; the subtrees of any
    level, plus the levels above them, sum to the whole evaluation."""
    c = synth.small_case(900 + M, 800, J=J, r=9, M=M, cluster=True, nu=1.5)
    t = Tree(c["x"], c["y"], c["z"], J=J, r=9, M=M)
    th = (1.2, 0.08, 0.02)
    ll, ls = t.loglik(th, MATERN, 1.5, level_sums=True)
    total = -2.0 * ll[0] - t.n_used * LOG2PI
    assert abs(subtree_du(t, th, 1, 0, MATERN, 1.5) - total) <= 1e-12 * abs(total)
    for lev in range(2, M + 1):
        s = sum(subtree_du(t, th, lev, k, MATERN, 1.5) for k in range(J ** (lev - 1)))
        above = ls[0, :lev - 1].sum()
        assert abs(s + above - total) <= 1e-11 * abs(total), lev


def test_subtree_of_a_leaf_is_its_leaf_term():
    """A finest-level subtree is one leaf: log det + quadratic form of its
    remainder matrix, here at M = 2 against the NumPy closed form."""
    rng = np.random.default_rng(23)
    n = 200
    x, y, z = rng.random(n), rng.random(n), rng.standard_normal(n)
    dom = [0.0, 1.0, 0.0, 1.0]
    th = (0.9, 0.2, 0.05)
    t = Tree(x, y, z, J=4, r=9, M=2, domain=dom)
    a = t.arrays()
    sx, sy, sz = a["x"], a["y"], a["z"]
    qx, qy = _grid_knots_np(dom, 9)
    Cqq = _cov_np(_dist(qx, qy, qx, qy), th[0], th[1], 0.5)
    for k in range(4):
        s = slice(a["leaf_off"][k], a["leaf_off"][k + 1])
        Csq = _cov_np(_dist(sx[s], sy[s], qx, qy), th[0], th[1], 0.5)
        K = _cov_np(_dist(sx[s], sy[s], sx[s], sy[s]), th[0], th[1], 0.5) - Csq @ np.linalg.solve(Cqq, Csq.T)
        d, q = _logdet_quad(K + th[2] * np.eye(K.shape[0]), sz[s])
        got = subtree_du(t, th, 2, k, MATERN, 0.5)
        assert abs(got - (d + q)) <= 1e-11 * abs(d + q), k


# ------------------------------------------------------ duplicate locations

def _with_duplicates(seed, n, ndup):
    rng = np.random.default_rng(seed)
    x, y, z = rng.random(n), rng.random(n), rng.standard_normal(n)
    src = rng.choice(n, size=ndup, replace=False)
    # repeats appended and interleaved: a later copy of an earlier location
    x = np.concatenate([x, x[src]]); y = np.concatenate([y, y[src]])
    z = np.concatenate([z, rng.standard_normal(ndup)])
    perm = rng.permutation(len(x))
    return x[perm], y[perm], z[perm]


def _first_occurrence(x, y):
    seen, keep = set(), np.zeros(len(x), dtype=bool)
    for i in range(len(x)):
        k = (x[i], y[i])
        if k not in seen:
            seen.add(k)
            keep[i] = True
    return keep


def test_duplicate_elimination_keeps_first():
    x, y, z = _with_duplicates(3, 600, 40)
    keep = _first_occurrence(x, y)
    t = Tree(x, y, z, J=4, r=16, M=3, flags=ELIM_DUPLICATES)
    ref = Tree(x[keep], y[keep], z[keep], J=4, r=16, M=3)
    plain = Tree(x, y, z, J=4, r=16, M=3)
    assert t.n_dup == 40 and t.n_used == 600 and plain.n_used == 640 and plain.n_dup == 0
    # the kept observations are the first of each location, in input order
    assert np.array_equal(np.sort(t.arrays()["orig"]), np.flatnonzero(keep))
    th = np.array([[1.0, 0.1, 0.02], [0.5, 0.04, 0.1]])
    # the root box of the deduplicated input is the same (repeats add no extreme)
    np.testing.assert_array_equal(t.arrays()["box"], ref.arrays()["box"])
    np.testing.assert_allclose(t.loglik(th), ref.loglik(th), rtol=1e-13)
    assert np.all(np.abs(t.loglik(th) - plain.loglik(th)) > 1.0)


def test_duplicates_and_nan_values():
    """A NaN-valued location is not an observation: it neither counts as the
    first copy of a location nor is dropped as a repeat."""
    x = np.array([0.1, 0.1, 0.1, 0.7, 0.7, 0.3])
    y = np.array([0.2, 0.2, 0.2, 0.8, 0.8, 0.4])
    z = np.array([np.nan, 1.0, 2.0, 0.5, 0.6, -1.0])
    t = Tree(x, y, z, J=4, r=4, M=2, flags=ELIM_DUPLICATES, domain=[0, 1, 0, 1])
    assert t.n_nan == 1 and t.n_dup == 2 and t.n_used == 3
    assert sorted(t.arrays()["orig"].tolist()) == [1, 3, 5]


# ------------------------------------------------------------ zero nugget

@pytest.mark.parametrize("nu", [0.5, 1.5])
def test_zero_nugget_recursion_matches_definition(nu):
    c = synth.small_case(33, 500, J=4, r=16, M=3, cluster=False, nu=nu)
    t = Tree(c["x"], c["y"], c["z"], J=4, r=16, M=3, flags=ALLOW_ZERO_NUGGET)
    th = (1.0, 0.05, 0.0)
    a = t.loglik(th, MATERN, nu)[0]
    b = t.dense_loglik(th, MATERN, nu)
    assert abs(a - b) <= 1e-9 * abs(b), (a, b)
    with pytest.raises(OracleError):
        Tree(c["x"], c["y"], c["z"], J=4, r=16, M=3).loglik(th, MATERN, nu)


def test_zero_nugget_M1_is_the_noise_free_gaussian():
    from scipy.stats import multivariate_normal
    rng = np.random.default_rng(41)
    n = 150
    x, y, z = rng.random(n), rng.random(n), rng.standard_normal(n)
    th = (1.3, 0.08, 0.0)
    t = Tree(x, y, z, J=4, r=16, M=1, flags=ALLOW_ZERO_NUGGET)
    a = t.arrays()
    K = _cov_np(_dist(a["x"], a["y"], a["x"], a["y"]), th[0], th[1], 0.5)
    ref = multivariate_normal(mean=np.zeros(n), cov=K).logpdf(a["z"])
    assert abs(t.loglik(th, MATERN, 0.5)[0] - ref) <= 1e-9 * abs(ref)


# ---------------------------------------------------- per-level log-determinants

@pytest.mark.parametrize("J,M,r,n,cluster,nu", [(4, 3, 16, 600, True, 0.5), (4, 4, 9, 800, False, 1.5),
                                                (2, 5, 4, 500, True, 1.5)])
def test_level_logdets_add_up_to_the_dense_log_determinant(J, M, r, n, cluster, nu):
    """The per-level log-determinant terms add up to log det(Sigma_MRA + tau I),
    computed by NumPy from the oracle's definitional dense covariance."""
    c = synth.small_case(700 + n, n, J=J, r=r, M=M, cluster=cluster, nu=nu)
    t = Tree(c["x"], c["y"], c["z"], J=J, r=r, M=M)
    th = (1.3, 0.09, 0.02)
    lev = t.level_logdets(th, MATERN, nu)[0]
    S = t.dense_sigma(th, MATERN, nu) + th[2] * np.eye(t.n_used)
    sign, ld = np.linalg.slogdet(S)
    assert sign > 0 and abs(lev.sum() - ld) <= 1e-10 * abs(ld)


def test_level_logdets_two_level_closed_form():
    """M = 2: the finest level holds the leaves' log det(C_2(S,S) + tau I)."""
    rng = np.random.default_rng(29)
    n = 250
    x, y, z = rng.random(n), rng.random(n), rng.standard_normal(n)
    dom = [0.0, 1.0, 0.0, 1.0]
    th = (0.8, 0.12, 0.04)
    t = Tree(x, y, z, J=4, r=9, M=2, domain=dom)
    a = t.arrays()
    sx, sy = a["x"], a["y"]
    qx, qy = _grid_knots_np(dom, 9)
    Cqq = _cov_np(_dist(qx, qy, qx, qy), th[0], th[1], 1.5)
    Csq = _cov_np(_dist(sx, sy, qx, qy), th[0], th[1], 1.5)
    R = _cov_np(_dist(sx, sy, sx, sy), th[0], th[1], 1.5) - Csq @ np.linalg.solve(Cqq, Csq.T)
    leaf = (sx >= 0.5).astype(int) + 2 * (sy >= 0.5).astype(int)
    want = sum(np.linalg.slogdet(R[np.ix_(leaf == k, leaf == k)] + th[2] * np.eye(int((leaf == k).sum())))[1]
               for k in range(4) if (leaf == k).any())
    lev = t.level_logdets(th, MATERN, 1.5)[0]
    assert abs(lev[1] - want) <= 1e-10 * abs(want)
