"""The partition built on the GPU (Sec. 1.2) against the oracle's, bit for
bit: the leaf of every observation, the order within leaves, eliminations and
counts, at the batched workload's size and on boundary cases (points on
midpoints, on knots, with missing values, J = 2), and against the library's
host build."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mra():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1905_00141_amd import mra as m
    return m


@pytest.fixture(scope="module")
def oracle():
    from oracle import oracle as o
    return o


def _same(t, o):
    a, b = t.arrays(), o.arrays()
    for k in ["x", "y", "z", "orig", "leaf_off"]:
        assert np.array_equal(a[k], b[k], equal_nan=True), k
    assert t.info["n_used"] == o.n_used and t.info["n_elim"] == o.n_elim and t.info["n_nan"] == o.n_nan


def test_partition_at_2_20(mra, oracle):
    from paper_1905_00141_amd import synth
    x, y = synth.mixture_locations(1 << 20, 3)
    z = np.random.default_rng(3).standard_normal(1 << 20)
    z[::97] = np.nan
    print("2^20 partition", flush=True)
    t = mra.Tree(x, y, z, J=4, r=64, M=9, domain=[0, 1, 0, 1])
    o = oracle.Tree(x, y, z, J=4, r=64, M=9, domain=[0, 1, 0, 1])
    _same(t, o)
    tb = mra.Tree(x, y, z, J=4, r=64, M=9)  # root box from the data (1 % extension)
    ob = oracle.Tree(x, y, z, J=4, r=64, M=9)
    _same(tb, ob)


def test_boundary_points_and_knots(mra, oracle):
    rng = np.random.default_rng(4)
    n = 4000
    x, y = rng.random(n), rng.random(n)
    # midpoints of levels 1..4 (they belong to the upper child) and exact knots
    g = np.arange(1, 16) / 16.0
    x[:15], y[:15] = g, g[::-1]
    kx, ky = oracle.box_knots([0, 1, 0, 1], 16, np.e / 100)  # the root region's knots
    x[15:31], y[15:31] = kx, ky
    z = rng.standard_normal(n)
    z[40:60] = np.nan
    for J, M in [(4, 5), (2, 7)]:
        t = mra.Tree(x, y, z, J=J, r=16, M=M, domain=[0, 1, 0, 1])
        o = oracle.Tree(x, y, z, J=J, r=16, M=M, domain=[0, 1, 0, 1])
        _same(t, o)
        assert t.info["n_elim"] > 0 and t.info["n_nan"] == 20


def test_gpu_and_host_builds_agree(mra):
    from paper_1905_00141_amd import synth
    c = synth.small_case(41, 20000, J=4, r=30, M=6, cluster=True)
    t = mra.Tree(c["x"], c["y"], c["z"], J=4, r=30, M=6)
    os.environ["MRA_HOST_TREE"] = "1"
    try:
        h = mra.Tree(c["x"], c["y"], c["z"], J=4, r=30, M=6)
    finally:
        del os.environ["MRA_HOST_TREE"]
    a, b = t.arrays(), h.arrays()
    for k in ["x", "y", "z", "orig", "leaf_off"]:
        assert np.array_equal(a[k], b[k]), k
    th = np.array([[1.0, 0.1, 0.01], [2.0, 0.05, 0.1]])
    assert np.array_equal(t.loglik(th), h.loglik(th))


def test_build_errors(mra):
    x, y, z = np.array([0.1, np.inf, 0.3]), np.array([0.1, 0.2, 0.3]), np.ones(3)
    with pytest.raises(mra.MraError) as e:
        mra.Tree(x, y, z, J=4, r=4, M=2, domain=[0, 1, 0, 1])
    assert e.value.code == mra.MRA_EINVAL and "index 1" in str(e.value)
    with pytest.raises(mra.MraError) as e:
        mra.Tree(np.array([0.1, 0.5, 1.5]), y, z, J=4, r=4, M=2, domain=[0, 1, 0, 1])
    assert e.value.code == mra.MRA_EDOMAIN and "2" in str(e.value)
