"""Maximum-likelihood search over the covariance parameters with exact MRA
evaluations, with and without the learned surrogate.

The paper's optimisation mode is a sequence of likelihood evaluations
(Sec. 2.2).  Here every exact evaluation is one row of a batched
mra_loglik_terms call.  The sill is profiled out in closed form: at fixed
range beta and nugget-to-sill ratio lam = tau / alpha, the MRA covariance
scales with alpha, so

    loglik(alpha) = -1/2 [ n log 2 pi + n log alpha + D + Q / alpha ]

with D, Q the log-determinant and quadratic form at alpha = 1; it peaks at
alpha_hat = Q / n.  The searches therefore run in the plane (log beta, log lam).

Three searches, each counting exact evaluations:
  * grid: the plain 32 x 32 grid over (beta, lam), log-spaced;
  * local: a derivative-free Nelder-Mead search on exact values from the
    centre of the box (the method without the surrogate);
  * surrogate: the network (include/mra_mlp.h) is trained on exact
    log-likelihoods (monotonically compressed near their maximum) at Sobol
    points of the (log alpha, log beta, log tau) box,
    its maximum over a dense grid is the proposal, and the same Nelder-Mead
    search on exact values starts there with a smaller simplex.
The exact MRA stays the judge of every reported value.

This module is orchestration only: every log-likelihood and every network
step runs in the library's kernels.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import mra, synth

LOG2PI = math.log(2.0 * math.pi)

# scale (nats) of the compression of the surrogate's training targets
TARGET_SCALE = 10.0

# search box of the profiled problem: range and nugget-to-sill ratio
BETA_LO, BETA_HI = 0.02, 0.3
LAM_LO, LAM_HI = 1e-3, 1e-1


class ExactObjective:
    """Profiled exact log-likelihood in (log beta, log lam), with an eval counter."""

    def __init__(self, tree: mra.Tree, family="matern", nu=1.5):
        self.tree, self.family, self.nu = tree, family, nu
        self.n = float(tree.info["n_used"])
        self.evals = 0
        self.history = []  # (eval count after the batch, best value so far)
        self.best = -np.inf
        self.best_x = None

    def __call__(self, X):
        X = np.atleast_2d(np.asarray(X, dtype=np.float64))
        th = np.stack([np.ones(len(X)), np.exp(X[:, 0]), np.exp(X[:, 1])], axis=1)
        _, ld, q = self.tree.loglik_terms(th, self.family, self.nu)
        ahat = q / self.n
        f = -0.5 * (self.n * LOG2PI + ld + self.n * np.log(ahat) + self.n)
        for i in range(len(X)):
            self.evals += 1
            if f[i] > self.best:
                self.best, self.best_x = float(f[i]), X[i].copy()
            self.history.append((self.evals, self.best))
        return f

    def alpha_hat(self, x):
        th = np.array([[1.0, math.exp(x[0]), math.exp(x[1])]])
        _, _, q = self.tree.loglik_terms(th, self.family, self.nu)
        return float(q[0]) / self.n

    def evals_to_reach(self, target):
        for e, b in self.history:
            if b >= target:
                return e
        return None


def box2():
    return np.log([BETA_LO, LAM_LO]), np.log([BETA_HI, LAM_HI])


def grid_search(obj: ExactObjective, k=32, batch=64, log=None):
    lo, hi = box2()
    b = np.linspace(lo[0], hi[0], k)
    lam = np.linspace(lo[1], hi[1], k)
    X = np.array([(u, v) for u in b for v in lam])  # range-major, ratio-minor
    f = np.empty(len(X))
    for s in range(0, len(X), batch):
        f[s:s + batch] = obj(X[s:s + batch])
        if log:
            log(f"[mle] grid: {min(s + batch, len(X))} of {len(X)} evaluated, best {obj.best:.3f}")
    i = int(np.argmax(f))  # first maximum in (range-major, ratio-minor) order
    return X[i], float(f[i])


def compass_search(obj: ExactObjective, x0, step, min_step=1e-3, max_evals=400):
    """Pattern search on the exact objective: poll the 4 compass points of the
    current step in one batch, move to the best improving one, else halve."""
    lo, hi = box2()
    x = np.clip(np.asarray(x0, dtype=np.float64), lo, hi)
    fx = float(obj(x)[0])
    dirs = np.array([[1.0, 0.0], [-1.0, 0.0], [0.0, 1.0], [0.0, -1.0]])
    step = np.asarray(step, dtype=np.float64)
    while np.all(step >= min_step) and obj.evals < max_evals:
        Y = np.clip(x + dirs * step, lo, hi)
        keep = np.any(Y != x, axis=1)
        if not keep.any():
            step = step / 2
            continue
        Y = Y[keep]
        fy = obj(Y)
        j = int(np.argmax(fy))
        if fy[j] > fx + 1e-9:
            x, fx = Y[j], float(fy[j])
        else:
            step = step / 2
    return x, fx


def nelder_mead(obj, x0, step, tol=0.02, max_evals=400):
    """Nelder-Mead simplex search (Nelder & Mead, 1965) maximising the exact
    objective in the box (points are clipped into it).  Standard coefficients:
    reflection 1, expansion 2, contraction 1/2, shrink 1/2.  Stops when the
    simplex's values span less than tol nats or the budget is spent."""
    lo, hi = box2()
    x0 = np.clip(np.asarray(x0, dtype=np.float64), lo, hi)
    step = np.asarray(step, dtype=np.float64)
    S = [x0]
    for d in (np.array([step[0], 0.0]), np.array([0.0, step[1]])):
        v = np.clip(x0 + d, lo, hi)
        if np.allclose(v, x0):  # clipped onto x0 at a face of the box: step the other way
            v = np.clip(x0 - d, lo, hi)
        S.append(v)
    S = np.array(S)
    F = obj(S)
    while obj.evals < max_evals:
        o = np.argsort(-F)
        S, F = S[o], F[o]
        if F[0] - F[-1] < tol:
            break
        c = S[:-1].mean(axis=0)
        xr = np.clip(c + (c - S[-1]), lo, hi)
        fr = float(obj(xr)[0])
        if fr > F[0]:
            xe = np.clip(c + 2.0 * (c - S[-1]), lo, hi)
            fe = float(obj(xe)[0])
            S[-1], F[-1] = (xe, fe) if fe > fr else (xr, fr)
        elif fr > F[-2]:
            S[-1], F[-1] = xr, fr
        else:
            inside = fr <= F[-1]
            xc = np.clip(c + 0.5 * ((S[-1] if inside else xr) - c), lo, hi)
            fc = float(obj(xc)[0])
            if fc > max(F[-1], fr if not inside else -np.inf):
                S[-1], F[-1] = xc, fc
            else:
                S[1:] = S[0] + 0.5 * (S[1:] - S[0])
                F[1:] = obj(S[1:])
    i = int(np.argmax(F))
    return S[i], float(F[i])


def train_surrogate(tree: mra.Tree, n_train=2048, seed=5, steps=3000, lr=3e-3, family="matern", nu=1.5,
                    log=None):
    """Exact log-likelihoods at n_train Sobol points of the log box, then
    full-batch Adam on the network.  Returns (net, exact evals used)."""
    lo, hi = synth.SURROGATE_BOX_LO, synth.SURROGATE_BOX_HI
    X = synth.sobol_box(n_train, lo, hi, seed)
    t0 = time.time()
    y = np.empty(n_train)
    for s in range(0, n_train, 64):  # batches of 64 parameter vectors per launch sequence
        y[s:s + 64] = tree.loglik(np.exp(X[s:s + 64]), family, nu)
        if log:
            log(f"[mle] surrogate training set: {min(s + 64, n_train)} of {n_train} exact evaluations")
    t_exact = time.time() - t0
    # The log-likelihood spans many orders of nats over the box; the network
    # is fitted to a monotone compression of it, -log(1 + (max - y) / s),
    # which keeps its maximiser and resolves the region near the best
    # training value (s = 10 nats) instead of the far tails.
    yt = -np.log1p((y.max() - y) / TARGET_SCALE)
    net = mra.Mlp(synth.mlp_init(seed))
    net.set_scaling(lo, hi, float(yt.mean()), float(yt.std()))
    y = yt
    xf = X.astype(np.float32)
    t0 = time.time()
    loss = None
    for k in range(steps):
        # cosine decay of the step size to 5 % of lr
        lr_k = lr * (0.05 + 0.95 * 0.5 * (1 + math.cos(math.pi * k / steps)))
        loss = net.train_step(xf, y, lr=float(lr_k))
    t_train = time.time() - t0
    if log:
        log(f"[mle] surrogate: {n_train} exact evals in {t_exact:.1f} s, {steps} Adam steps in {t_train:.1f} s, "
            f"final standardised MSE {float(loss[0]):.2e}")
    return net, n_train


def surrogate_proposal(net: mra.Mlp, k=48):
    """Maximum of the network over a k^3 grid of the log box (log alpha, log beta, log tau),
    returned as (log beta, log lam) clipped to the profiled search box."""
    lo, hi = synth.SURROGATE_BOX_LO, synth.SURROGATE_BOX_HI
    axes = [np.linspace(lo[i], hi[i], k) for i in range(3)]
    G = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, 3).astype(np.float32)
    s = net.forward(G)
    g = G[int(np.argmax(s))].astype(np.float64)
    lo2, hi2 = box2()
    return np.clip(np.array([g[1], g[2] - g[0]]), lo2, hi2)


def run(tree: mra.Tree, family="matern", nu=1.5, n_train=2048, grid_k=32, seed=5, train_steps=3000, log=None):
    """All three searches on one tree; evaluation counts to within 0.5 nats of
    the best exact value any of them found."""
    lo, hi = box2()
    width = hi - lo
    g = ExactObjective(tree, family, nu)
    xg, fg = grid_search(g, grid_k, log=log)

    c = ExactObjective(tree, family, nu)
    xc, fc = nelder_mead(c, (lo + hi) / 2, width / 4)
    if log:
        log(f"[mle] local search without the surrogate: {c.evals} evals, best {fc:.3f}")

    net, n_tr = train_surrogate(tree, n_train, seed, train_steps, family=family, nu=nu, log=log)
    s = ExactObjective(tree, family, nu)
    x0 = surrogate_proposal(net)
    f0 = float(s(x0)[0])
    xs, fs = nelder_mead(s, x0, width / 32)

    best = max(fg, fc, fs)
    target = best - 0.5
    res = {
        "best_loglik": best,
        "grid": {"evals": g.evals, "evals_to_mle": g.evals if fg >= target else None, "loglik": fg,
                 "beta": math.exp(xg[0]), "lam": math.exp(xg[1]), "alpha": g.alpha_hat(xg)},
        "local": {"evals": c.evals, "evals_to_mle": c.evals_to_reach(target), "loglik": fc,
                    "beta": math.exp(xc[0]), "lam": math.exp(xc[1])},
        "surrogate": {"train_evals": n_tr, "search_evals": s.evals, "evals_to_mle": s.evals_to_reach(target),
                      "proposal_loglik": f0, "loglik": fs, "beta": math.exp(xs[0]), "lam": math.exp(xs[1]),
                      "proposal_beta": math.exp(x0[0]), "proposal_lam": math.exp(x0[1])},
    }
    if log:
        log(f"[mle] grid {grid_k}x{grid_k}: {g.evals} evals, best {fg:.3f}; local search: {c.evals} evals, best {fc:.3f}; "
            f"surrogate: proposal {f0:.3f}, {s.evals} search evals, best {fs:.3f}")
    return res
