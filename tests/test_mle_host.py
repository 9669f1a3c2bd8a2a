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


def test_trust_region_converges_inside_the_box():
    lo, hi = mle.box2()
    xs = lo + np.array([0.3, 0.6]) * (hi - lo)
    obj = Quadratic(xs)
    x, fx = mle.trust_region(obj, (lo + hi) / 2, 0.25, rho_end=1e-4)
    assert fx > -1e-6 and np.allclose(x, xs, atol=1e-3)
    assert obj.evals < 40  # a quadratic is fitted exactly after the initial design


def test_trust_region_curved_valley():
    """A banana-shaped objective (Rosenbrock form in scaled box units): not a
    quadratic, so the models must be refitted along the valley."""
    lo, hi = mle.box2()

    class Banana(Quadratic):
        def __call__(self, X):
            X = np.atleast_2d(X)
            u = (X - lo) / (hi - lo) * 2.0 - 1.0
            f = -(10.0 * (u[:, 1] - u[:, 0] ** 2) ** 2 + (0.6 - u[:, 0]) ** 2)
            for i in range(len(X)):
                self.evals += 1
                if f[i] > self.best:
                    self.best, self.best_x = f[i], X[i].copy()
                self.history.append((self.evals, self.best))
            return f

    obj = Banana(np.zeros(2))
    x, fx = mle.trust_region(obj, lo + 0.1 * (hi - lo), 0.2, rho_end=1e-5, max_evals=400)
    u = (x - lo) / (hi - lo) * 2.0 - 1.0
    assert fx > -1e-4 and np.allclose(u, [0.6, 0.36], atol=0.02), (u, fx)


def test_trust_region_stops_at_an_active_bound():
    lo, hi = mle.box2()
    obj = Quadratic(np.array([hi[0] + 1.0, lo[1] + 0.4 * (hi[1] - lo[1])]))
    x, _ = mle.trust_region(obj, (lo + hi) / 2, 0.25, rho_end=1e-4)
    assert abs(x[0] - hi[0]) < 1e-9 and abs(x[1] - obj.xstar[1]) < 1e-2


def test_trust_region_on_the_oracle_likelihood():
    """The optimiser driven by the CPU oracle's profiled log-likelihood on a
    small tree reaches the maximum of a fine grid of oracle evaluations."""
    from oracle import oracle as o
    from paper_1905_00141_amd import synth

    c = synth.small_case(91, 900, J=4, r=16, M=3, cluster=True, nu=1.5)
    t = o.Tree(c["x"], c["y"], c["z"], J=4, r=16, M=3)
    n = t.n_used

    class OracleProfiled(Quadratic):
        def __call__(self, X):
            X = np.atleast_2d(X)
            f = np.empty(len(X))
            for i, (lb, ll) in enumerate(X):
                b, lam = np.exp(lb), np.exp(ll)
                l1, l2 = t.loglik(np.array([[1.0, b, lam], [2.0, b, 2.0 * lam]]), o.MATERN, 1.5)
                k1 = -2 * l1 - n * np.log(2 * np.pi)               # D + Q
                k2 = -2 * l2 - n * np.log(2 * np.pi) - n * np.log(2.0)  # D + Q / 2
                Q = 2.0 * (k1 - k2)
                D = k1 - Q
                f[i] = -0.5 * (n * np.log(2 * np.pi) + D + n * np.log(Q / n) + n)
                self.evals += 1
                if f[i] > self.best:
                    self.best, self.best_x = f[i], X[i].copy()
                self.history.append((self.evals, self.best))
            return f

    lo, hi = mle.box2()
    grid = OracleProfiled(np.zeros(2))
    gx = np.linspace(lo[0], hi[0], 17)
    gy = np.linspace(lo[1], hi[1], 17)
    gf = grid(np.array([(u, v) for u in gx for v in gy]))
    tr = OracleProfiled(np.zeros(2))
    x, fx = mle.trust_region(tr, (lo + hi) / 2, 0.25, rho_end=1e-4)
    assert fx >= gf.max() - 1e-6, (fx, gf.max())
    assert tr.evals < 120
