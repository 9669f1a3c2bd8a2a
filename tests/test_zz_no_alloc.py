"""mra_loglik_noalloc (the entry point that allocates nothing) against
mra_loglik with device pointers: two calls in a row on different trees, the
second smaller, each equal to the allocating call's result (the same kernels
on the same plan: equal up to rounding, bar 1e-10 relative per theta)."""
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


def _rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)) / np.abs(np.asarray(b))


def test_noalloc_matches_loglik_twice(mra):
    import torch
    from paper_1905_00141_amd import synth
    dev = torch.device("cuda:0")
    s = torch.cuda.Stream()
    big = synth.config1()
    small = synth.small_case(5, 1500, J=4, r=16, M=3, cluster=True, nu=1.5)
    th_big = np.vstack([big["theta"], synth.theta_grid(3, 3)])
    th_small = synth.theta_grid(2, 2)[:3]
    for c, th, fam, nu in [(big, th_big, "exp", 0.5), (small, th_small, "matern", 1.5)]:
        t = mra.Tree(c["x"], c["y"], c["z"], J=c["J"], r=c["r"], M=c["M"])
        tt = torch.tensor(th, dtype=torch.float64, device=dev)
        ref = t.loglik(tt, fam, nu, stream=s)
        out = torch.full((len(th),), np.nan, dtype=torch.float64, device=dev)
        t.loglik_noalloc(tt, out, fam, nu, stream=s)
        s.synchronize()
        got, want = out.cpu().numpy(), ref.cpu().numpy()
        print("noalloc", c.get("name", "small"), got, "max rel", _rel(got, want).max(), flush=True)
        assert np.all(np.isfinite(got)) and np.all(_rel(got, want) <= 1e-10)


def test_noalloc_rejects_a_tree_beyond_its_scratch(mra):
    import torch
    rng = np.random.default_rng(3)
    n = 200000
    t = mra.Tree(rng.random(n), rng.random(n), rng.standard_normal(n), J=4, r=64, M=5)
    dev = torch.device("cuda:0")
    th = torch.tensor([[1.0, 0.1, 0.01]], dtype=torch.float64, device=dev)
    out = torch.empty(1, dtype=torch.float64, device=dev)
    with pytest.raises(mra.MraError) as e:
        t.loglik_noalloc(th, out)
    assert e.value.code == mra.MRA_ENOMEM and "limit" in str(e.value)
    with pytest.raises(mra.MraError) as e:
        t.loglik_noalloc(th.cpu().numpy(), out)
    assert e.value.code == mra.MRA_EINVAL
