"""Host logic of the MLE searches (no GPU): the pattern search and the
evaluation counter on an analytic objective in the same (log beta, log lam)
box."""
import numpy as np

from paper_1905_00141_amd import mle


class Quadratic:
    def __init__(self, xstar):
        self.xstar = np.asarray(xstar)
        self.evals, self.history, self.best, self.best_x = 0, [], -np.inf, None

    def __call__(self, X):
        X = np.atleast_2d(X)
        f = -np.sum(((X - self.xstar) / np.array([0.3, 0.7])) ** 2, axis=1) * 50.0
        for i in range(len(X)):
            self.evals += 1
            if f[i] > self.best:
                self.best, self.best_x = f[i], X[i].copy()
            self.history.append((self.evals, self.best))
        return f

    evals_to_reach = mle.ExactObjective.evals_to_reach


def test_compass_converges_inside_the_box():
    lo, hi = mle.box2()
    xs = lo + np.array([0.3, 0.6]) * (hi - lo)
    obj = Quadratic(xs)
    x, fx = mle.compass_search(obj, (lo + hi) / 2, (hi - lo) / 4, min_step=1e-4)
    assert np.allclose(x, xs, atol=3e-4) and fx > -1e-4
    assert obj.evals_to_reach(-0.5) <= obj.evals


def test_compass_stays_in_the_box_at_a_corner_optimum():
    lo, hi = mle.box2()
    obj = Quadratic(hi + 1.0)  # optimum outside: the search ends at the corner
    x, _ = mle.compass_search(obj, (lo + hi) / 2, (hi - lo) / 4)
    assert np.allclose(x, hi)


def test_grid_order_and_count():
    lo, hi = mle.box2()
    obj = Quadratic(lo + 0.5 * (hi - lo))
    x, f = mle.grid_search(obj, 8)
    assert obj.evals == 64 and f == obj.best


def test_nelder_mead_converges_and_counts():
    lo, hi = mle.box2()
    xs = lo + np.array([0.7, 0.25]) * (hi - lo)
    obj = Quadratic(xs)
    x, fx = mle.nelder_mead(obj, (lo + hi) / 2, (hi - lo) / 4, tol=1e-6)
    assert fx > -1e-3 and np.allclose(x, xs, atol=0.01)
    assert obj.evals < 150 and obj.evals_to_reach(-0.5) < obj.evals


def test_nelder_mead_from_a_face_of_the_box():
    lo, hi = mle.box2()
    obj = Quadratic(lo + np.array([0.5, 0.5]) * (hi - lo))
    x, fx = mle.nelder_mead(obj, hi, (hi - lo) / 8, tol=1e-6)
    assert fx > -1e-3
