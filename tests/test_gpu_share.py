"""Parameter vectors that share alpha and range share the prior (levels
1..M-1 and the observations' whitened rows involve neither the nugget nor the
data; Sec. 1.1: the nugget enters the finest level only).  A batch with such
repeats must give, per theta, the same log-likelihood, bit for bit, as the
same theta evaluated alone, as the batch with sharing switched off, and the
oracle's within 1e-10; graph replays must follow new values whose sharing
pattern differs; and a prior factor that fails for the first theta of a
group is reported for every theta of the group."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

RTOL = 1e-10
# repeats of (alpha, range) in scrambled order, an exact duplicate, and a
# pattern that crosses the chunk boundary of a small-memory split
THETAS = np.array([
    [1.0, 0.05, 0.01], [1.0, 0.12, 0.01], [1.0, 0.05, 0.1], [2.0, 0.05, 0.01], [1.0, 0.12, 0.05],
    [1.0, 0.05, 0.01], [2.0, 0.05, 0.003], [1.0, 0.05, 0.002], [1.0, 0.3, 0.02], [1.0, 0.12, 0.001],
])


@pytest.fixture(scope="module")
def mra():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1905_00141_amd import mra as m
    return m


@pytest.fixture(scope="module")
def case():
    from paper_1905_00141_amd import synth
    # clustered: leaves on the one-wave finisher and on the workgroup finisher
    x, y = synth.mixture_locations(6000, 21, k=6, sigma_range=(0.03, 0.15))
    z = np.random.default_rng(22).standard_normal(len(x))
    return dict(x=x, y=y, z=z)


def _rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)) / np.abs(np.asarray(b))


def _tree(mra, c):
    return mra.Tree(c["x"], c["y"], c["z"], J=4, r=16, M=5, domain=[0, 1, 0, 1])


def test_case_has_large_leaves(case):
    from oracle import oracle as o
    t = o.Tree(case["x"], case["y"], case["z"], J=4, r=16, M=5, domain=[0, 1, 0, 1])
    cnt = np.diff(t.arrays()["leaf_off"])
    assert cnt.max() > 64 and np.count_nonzero((cnt > 0) & (cnt <= 64)) > 10


def test_shared_prior_is_bit_identical_to_single_theta(mra, case):
    t = _tree(mra, case)
    got = t.loglik(THETAS, "matern", 1.5)
    alone = np.array([t.loglik(th[None, :], "matern", 1.5)[0] for th in THETAS])
    assert np.array_equal(got, alone), (got - alone)
    os.environ["MRA_SHARE_PRIOR"] = "0"
    try:
        off = t.loglik(THETAS, "matern", 1.5)
    finally:
        del os.environ["MRA_SHARE_PRIOR"]
    assert np.array_equal(got, off)
    assert got[0] == got[5]


def test_shared_prior_matches_oracle(mra, case):
    from oracle import oracle as o
    t = _tree(mra, case)
    ref = o.Tree(case["x"], case["y"], case["z"], J=4, r=16, M=5, domain=[0, 1, 0, 1]).loglik(THETAS, o.MATERN, 1.5)
    got = t.loglik(THETAS, "matern", 1.5)
    assert np.all(_rel(got, ref) <= RTOL), _rel(got, ref)


def test_graph_replays_follow_a_new_sharing_pattern(mra, case):
    import torch
    t = _tree(mra, case)
    dev = torch.device("cuda:0")
    th = torch.tensor(THETAS, dtype=torch.float64, device=dev)
    out = torch.empty(len(THETAS), dtype=torch.float64, device=dev)
    s = torch.cuda.Stream()
    variants = [THETAS, THETAS[::-1].copy(), np.repeat(THETAS[:1], len(THETAS), axis=0) * [1, 1, 1],
                np.column_stack([THETAS[:, 0], np.linspace(0.03, 0.2, len(THETAS)), THETAS[:, 2]])]
    for v in variants:
        th.copy_(torch.tensor(v, dtype=torch.float64))
        torch.cuda.synchronize()
        t.loglik(th, "matern", 1.5, out=out, stream=s)
        s.synchronize()
        eager = t.loglik(v, "matern", 1.5)
        assert np.array_equal(out.cpu().numpy(), eager)


def test_failed_prior_fails_every_theta_of_its_group(mra):
    """A Gaussian covariance with a range far beyond the domain leaves the
    knot matrices singular in FP64: the first theta of the group fails in the
    prior and the second, which shares it, is reported too; a theta with a
    short range in the same batch is unaffected."""
    import torch
    from paper_1905_00141_amd import synth
    c = synth.small_case(41, 2000, J=4, r=16, M=3)
    t = mra.Tree(c["x"], c["y"], c["z"], J=4, r=16, M=3, domain=[0, 1, 0, 1])
    th = torch.tensor([[1.0, 50.0, 0.01], [1.0, 0.02, 0.01], [1.0, 50.0, 0.1]], dtype=torch.float64,
                      device=torch.device("cuda:0"))
    out = t.loglik(th, "gauss", 0.0)
    o = out.cpu().numpy()
    assert np.isnan(o[0]) and np.isnan(o[2]) and np.isfinite(o[1]), o
    with pytest.raises(mra.MraError) as e:
        t.status()
    assert e.value.code == mra.MRA_ENOTPD


def test_chunk_multiple(mra, case):
    t = _tree(mra, case)
    ref = t.loglik(THETAS, "matern", 1.5)
    t.set_chunk_multiple(3)
    assert np.array_equal(t.loglik(THETAS, "matern", 1.5), ref)
    with pytest.raises(mra.MraError) as e:
        t.set_chunk_multiple(0)
    assert e.value.code == mra.MRA_EINVAL


def test_failed_leaf_inside_a_shared_group(mra):
    """The finest-level finishers of a group run in one launch, the
    representative's task waiting for the others to have read its rows.  A
    leaf of 80 observations at one location with a vanishing nugget fails
    for the representative (theta 0) and for one other theta of its group
    (theta 2); the other theta of the group, and a theta of another group,
    must still give the values they give alone, bit for bit."""
    import torch
    rng = np.random.default_rng(5)
    x = np.r_[np.full(80, 0.3), rng.uniform(0, 1, 600)]
    y = np.r_[np.full(80, 0.3), rng.uniform(0, 1, 600)]
    z = rng.standard_normal(len(x))
    t = mra.Tree(x, y, z, J=4, r=16, M=3, domain=[0, 1, 0, 1])
    dev = torch.device("cuda:0")
    th = np.array([[1.0, 0.1, 1e-300], [1.0, 0.1, 0.1], [1.0, 0.1, 1e-300], [1.0, 0.1, 0.05], [1.0, 0.3, 0.1]])
    out = t.loglik(torch.tensor(th, dtype=torch.float64, device=dev)).cpu().numpy()
    with pytest.raises(mra.MraError) as e:
        t.status()
    assert e.value.code == mra.MRA_ENOTPD and "theta 0" in str(e.value)
    assert np.isnan(out[0]) and np.isnan(out[2]), out
    for i in (1, 3, 4):
        alone = t.loglik(th[i][None, :])[0]
        assert out[i] == alone, (i, out[i], alone)


def test_shared_groups_over_many_workgroup_leaves(mra):
    """In the single leaf launch a region's representatives are queued 64
    regions after its other theta.  A tree with more than 64 leaves on the
    workgroup finisher (99 of 65 to 1688 observations) and theta in groups of
    three, two and one must match the oracle within 1e-10 and each theta's
    single evaluation bit for bit."""
    from oracle import oracle as o
    from paper_1905_00141_amd import synth
    x, y = synth.mixture_locations(30000, 9, k=6, sigma_range=(0.02, 0.2))
    z = np.random.default_rng(9).standard_normal(len(x))
    th = np.array([[1.0, 0.05, 0.01], [1.0, 0.2, 0.01], [1.0, 0.05, 0.002], [1.5, 0.1, 0.02],
                   [1.0, 0.2, 0.001], [1.0, 0.05, 0.05]])
    ot = o.Tree(x, y, z, J=4, r=16, M=6, domain=[0, 1, 0, 1])
    assert np.count_nonzero(np.diff(ot.arrays()["leaf_off"]) > 64) > 64
    print("many-leaves case: oracle on 6 theta", flush=True)
    ref = ot.loglik(th, o.MATERN, 1.5)
    t = mra.Tree(x, y, z, J=4, r=16, M=6, domain=[0, 1, 0, 1])
    got = t.loglik(th, "matern", 1.5)
    assert np.all(_rel(got, ref) <= RTOL), _rel(got, ref)
    alone = np.array([t.loglik(v[None, :], "matern", 1.5)[0] for v in th])
    assert np.array_equal(got, alone), got - alone
