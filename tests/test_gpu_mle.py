"""The surrogate-guided MLE search against the plain grid and against the same
search without the surrogate, on a reduced mixture workload (exact MRA judges
every value)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def result():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1905_00141_amd import mle, mra, synth
    c = synth.config3(n=1 << 14, M=5, device="cuda")
    t = mra.Tree(c["x"], c["y"], c["z"], J=4, r=64, M=5, domain=c["domain"])
    res = mle.run(t, n_train=512, train_steps=1500, log=print)
    print(res)
    return res


def test_surrogate_reaches_the_mle_in_fewer_exact_evals_than_the_grid(result):
    s, g = result["surrogate"], result["grid"]
    assert s["evals_to_mle"] is not None
    assert s["evals_to_mle"] < g["evals"]
    assert s["loglik"] >= result["best_loglik"] - 0.5


def test_surrogate_proposal_is_close(result):
    # the network's maximum alone is already within a few nats of the MLE
    s = result["surrogate"]
    assert s["proposal_loglik"] >= result["best_loglik"] - 25.0, s


def test_grid_is_within_its_resolution(result):
    assert result["grid"]["loglik"] >= result["best_loglik"] - 5.0
