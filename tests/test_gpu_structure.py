"""GPU log-likelihood parity at the tree structure of the batched n = 2^20
workload (r = 64, deep tree, strongly uneven leaves), small enough for the
oracle.

The case (12,000 points from a 6-component Gaussian mixture with sigmas
log-uniform in [0.008, 0.15], M = 6, r = 64) makes every kernel path of the
full workload run:
  * the observation-row chain with 5 ancestor levels, i.e. three ancestor
    groups of two levels (the earlier-groups branch that reads back V rows);
  * leaves of up to ~420 observations (the blocked workgroup Cholesky, more
    than four 64-row diagonal blocks);
  * level-5 regions of 65-192 observations (observation-space folds on the
    workgroup kernel) next to larger ones folded in knot space, with the Schur
    blocks in 128 x 128 super-blocks;
  * plans that send 17-64-row leaves and every fold to the workgroup kernels.
Bar: 1e-10 relative per theta, and repeated evaluations bit-identical.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

RTOL = 1e-10
THETAS = np.array([[1.0, 0.02, 0.001], [1.0, 0.1, 0.01], [1.0, 0.3, 0.1]])
N, M, R = 12000, 6, 64


@pytest.fixture(scope="module")
def mra():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1905_00141_amd import mra as m
    return m


@pytest.fixture(scope="module")
def case():
    from oracle import oracle as o
    from paper_1905_00141_amd import synth
    x, y = synth.mixture_locations(N, 5, k=6, sigma_range=(0.008, 0.15))
    z = np.random.default_rng(6).standard_normal(N)
    print("structure case: oracle on 3 theta", flush=True)
    ot = o.Tree(x, y, z, J=4, r=R, M=M, domain=[0, 1, 0, 1])
    ref = ot.loglik(THETAS, o.MATERN, 1.5)
    counts = np.diff(ot.arrays()["leaf_off"])
    return dict(x=x, y=y, z=z, ref=ref, counts=counts)


def _rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)) / np.abs(np.asarray(b))


def test_case_has_the_structure(case):
    c = case["counts"]
    lvl5 = c.reshape(-1, 4).sum(axis=1)
    assert c.max() > 256
    assert np.count_nonzero((lvl5 > 64) & (lvl5 <= 192)) >= 10
    assert lvl5.max() > 192


@pytest.mark.parametrize("plan", ["default", "gram", "factor", "wg_leaves", "falling"])
def test_structure_loglik_matches_oracle(mra, case, plan):
    flags = {"gram": mra.MRA_FOLD_GRAM, "factor": mra.MRA_FOLD_FACTOR}.get(plan, 0)
    print(f"structure case plan {plan}", flush=True)
    t = mra.Tree(case["x"], case["y"], case["z"], J=4, r=R, M=M, flags=flags, domain=[0, 1, 0, 1])
    if plan == "wg_leaves":
        t.set_plan([0] * (M - 1), 16)       # every fold in knot space, leaves > 16 rows on the workgroup kernel
    elif plan == "falling":
        t.set_plan([-1, -1, 4096, 0, 128], 64)  # a threshold that falls with depth
    mra.profile_enable(True)
    got = t.loglik(THETAS, "matern", 1.5)
    stats = mra.profile_read()
    mra.profile_enable(False)
    ran = {(s["name"], s["level"]) for s in stats}
    print(plan, sorted(ran), _rel(got, case["ref"]))
    assert np.all(_rel(got, case["ref"]) <= RTOL), (got, case["ref"], _rel(got, case["ref"]))
    assert ("k_chain", M) in ran
    if plan == "default":
        assert ("k_fold_factor", M - 1) in ran and ("k_leaf_finish", M) in ran
        assert any(n == "k_gram_tile2" for n, _ in ran)
    for _ in range(3):
        assert np.array_equal(t.loglik(THETAS, "matern", 1.5), got)


def test_per_level_log_determinants_match_the_oracle(mra, case):
    """The per-level breakdown of the log-determinant (mra_loglik_levels)
    against the oracle's, level by level, on the same tree: bar 1e-10 of the
    total log-determinant's magnitude per level."""
    from oracle import oracle as o
    th = THETAS[1:2]
    t = mra.Tree(case["x"], case["y"], case["z"], J=4, r=R, M=M, domain=[0, 1, 0, 1])
    ll, lev = t.level_logdets(th, "matern", 1.5)
    ot = o.Tree(case["x"], case["y"], case["z"], J=4, r=R, M=M, domain=[0, 1, 0, 1])
    ref = ot.level_logdets(th, o.MATERN, 1.5)
    scale = np.abs(ref).sum()
    print("levels gpu", lev, "oracle", ref)
    assert np.all(np.abs(lev - ref) <= 1e-10 * scale), np.abs(lev - ref) / scale
    assert abs(ll[0] - case["ref"][1]) <= 1e-10 * abs(case["ref"][1])
