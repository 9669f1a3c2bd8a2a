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

Searches, each counting exact evaluations and the sequential calls they need:
  * grid: the plain 32 x 32 grid over (beta, lam), log-spaced;
  * local: a derivative-free Nelder-Mead search on exact values from the
    centre of the box (a method without the surrogate);
  * trust region: a derivative-free trust-region search with quadratic
    interpolation models in the box, after Powell's methods (UOBYQA 2002,
    BOBYQA 2009; the paper's optimisation mode uses BOBYQA, Sec. 2.2);
  * surrogate (sequential design): the network (include/mra_mlp.h) is fitted
    to the exact values of a 64-point Sobol design of the box, proposes the
    maximum of its prediction and a few distinct near-maximal points, the
    exact MRA evaluates them in one batch, the network is refitted, and so
    on until the best exact value stops improving;
  * surrogate (pre-trained): the network trained once on 2048 exact values
    in the (log alpha, log beta, log tau) box proposes a start for
    Nelder-Mead (kept for comparison; its training set outweighs the grid).
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
        self.calls = 0     # sequential exact calls (batches)
        self.history = []  # (eval count after the batch, best value so far)
        self.best = -np.inf
        self.best_x = None

    def __call__(self, X):
        X = np.atleast_2d(np.asarray(X, dtype=np.float64))
        self.calls += 1
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


def trust_region(obj, x0, rho_beg, rho_end=1e-3, max_evals=200, lo=None, hi=None):
    """Derivative-free trust-region maximisation in a box with quadratic
    interpolation models (after Powell's UOBYQA and BOBYQA).  The model
    q(x) = c + g.(x - xb) + (x - xb)^T H (x - xb) / 2 interpolates the
    objective at (n+1)(n+2)/2 points around the best point xb; each iteration
    maximises q over the trust region |d| <= delta intersected with the box,
    evaluates the step, compares the actual with the predicted increase to
    enlarge or shrink delta, and replaces the interpolation point farthest
    from the best one (or, when the model step is too short, moves that point
    to a distance delta along a coordinate to restore the geometry).  Stops
    when delta falls below rho_end or the budget is spent."""
    if lo is None or hi is None:
        lo, hi = box2()
    lo, hi = np.asarray(lo, dtype=np.float64), np.asarray(hi, dtype=np.float64)
    n = len(lo)
    x0 = np.clip(np.asarray(x0, dtype=np.float64), lo, hi)
    scale = hi - lo

    def clip(p, ref):
        q = np.clip(p, lo, hi)
        if np.allclose(q, ref):
            q = np.clip(ref - (p - ref), lo, hi)
        return q

    pts = [x0]
    for i in range(n):
        e = np.zeros(n)
        e[i] = rho_beg * scale[i]
        pts.append(clip(x0 + e, x0))
        pts.append(clip(x0 - e, x0))
    for i in range(n):
        for j in range(i + 1, n):
            e = np.zeros(n)
            e[i], e[j] = rho_beg * scale[i], rho_beg * scale[j]
            pts.append(clip(x0 + e, x0))
    Y = np.array(pts)
    F = np.asarray(obj(Y), dtype=np.float64)
    delta = rho_beg

    def basis(D):  # quadratic monomials of the scaled displacement
        cols = [np.ones(len(D))] + [D[:, i] for i in range(n)]
        cols += [D[:, i] * D[:, j] * (0.5 if i == j else 1.0) for i in range(n) for j in range(i, n)]
        return np.stack(cols, axis=1)

    while obj.evals < max_evals and delta >= rho_end:
        b = int(np.argmax(F))
        xb, fb = Y[b], F[b]
        D = (Y - xb) / scale
        coef, *_ = np.linalg.lstsq(basis(D), F, rcond=None)
        g = coef[1:1 + n]
        H = np.zeros((n, n))
        k = 1 + n
        for i in range(n):
            for j in range(i, n):
                H[i, j] = H[j, i] = coef[k]
                k += 1
        q = lambda d: float(coef[0] + g @ d + 0.5 * d @ H @ d)
        # trust-region step: the better of the model's stationary point (if
        # it is a maximum inside the region) and a dense search of the
        # region's boundary, each kept inside the box
        cands = []
        try:
            s = -np.linalg.solve(H, g)
            if np.all(np.linalg.eigvalsh(H) < 0) and np.linalg.norm(s) <= delta:
                cands.append(s)
        except np.linalg.LinAlgError:
            pass
        ang = np.linspace(0.0, 2.0 * np.pi, 256, endpoint=False)
        if n == 2:
            ring = np.stack([np.cos(ang), np.sin(ang)], axis=1)
        else:
            ring = np.random.default_rng(0).standard_normal((512, n))
            ring /= np.linalg.norm(ring, axis=1, keepdims=True)
        for fr in (1.0, 0.5, 0.25):
            cands.extend(list(ring * delta * fr))
        dl, dh = (lo - xb) / scale, (hi - xb) / scale
        cands = [np.clip(c, dl, dh) for c in cands]
        d = max(cands, key=q)
        pred = q(d) - fb
        if np.linalg.norm(d) < 0.1 * delta or pred <= 1e-12:
            # model step too short: improve the geometry, then shrink
            far = int(np.argmax(np.linalg.norm(D, axis=1)))
            if np.linalg.norm(D[far]) > 2.0 * delta:
                e = np.zeros(n)
                e[obj.evals % n] = delta
                Y[far] = clip(xb + e * scale, xb)
                F[far] = float(obj(Y[far])[0])
            else:
                delta *= 0.5
            continue
        xn = xb + d * scale
        fn = float(obj(xn)[0])
        ratio = (fn - fb) / pred
        if ratio > 0.7 and np.linalg.norm(d) > 0.9 * delta:
            delta = min(2.0 * delta, 0.5)
        elif ratio < 0.1:
            delta *= 0.5
        # replace the point farthest from the (new) best point
        ref = xn if fn > fb else xb
        dist = np.linalg.norm((Y - ref) / scale, axis=1)
        if fn <= fb:
            dist[b] = -1.0
        far = int(np.argmax(dist))
        Y[far], F[far] = xn, fn
    b = int(np.argmax(F))
    return Y[b], float(F[b])


def surrogate_sequential(tree: mra.Tree, family="matern", nu=1.5, n_init=64, per_round=8, max_rounds=12,
                         steps_first=1500, steps=400, lr=3e-3, seed=5, log=None):
    """Sequential design with the network in the profiled plane (log beta,
    log lam): fit, propose the maximum of the prediction and near-maximal
    points at least a grid step apart from every evaluated point, evaluate
    them exactly in one batch, refit.  Stops after two rounds without an
    improvement of 0.05 nats.  Returns (objective, best x, best value, net)."""
    obj = ExactObjective(tree, family, nu)
    lo, hi = box2()
    from scipy.stats import qmc
    X = lo + qmc.Sobol(d=2, scramble=True, seed=seed).random(n_init) * (hi - lo)
    F = np.asarray(obj(X), dtype=np.float64)
    lo3 = np.array([-1.0, lo[0], lo[1]])
    hi3 = np.array([1.0, hi[0], hi[1]])
    net = mra.Mlp(synth.mlp_init(seed))
    k = 128
    gx = np.linspace(lo[0], hi[0], k)
    gy = np.linspace(lo[1], hi[1], k)
    G = np.array([(u, v) for u in gx for v in gy])
    G3 = np.concatenate([np.zeros((len(G), 1)), G], axis=1).astype(np.float32)
    min_sep = 1.5 * (hi - lo) / (k - 1)
    stall = 0
    for r in range(max_rounds):
        yt = -np.log1p((F.max() - F) / TARGET_SCALE)
        net.set_scaling(lo3, hi3, float(yt.mean()), float(yt.std()))
        x3 = np.concatenate([np.zeros((len(X), 1)), X], axis=1).astype(np.float32)
        nst = steps_first if r == 0 else steps
        for s in range(nst):
            lr_k = lr * (0.05 + 0.95 * 0.5 * (1 + math.cos(math.pi * s / nst)))
            net.train_step(x3, yt, lr=float(lr_k))
        pred = np.asarray(net.forward(G3))
        order = np.argsort(-pred)
        chosen = []
        for i in order:
            p = G[i]
            if np.all(np.any(np.abs(X - p) > min_sep, axis=1)) and \
                    all(np.any(np.abs(c - p) > min_sep) for c in chosen):
                chosen.append(p)
                if len(chosen) == per_round:
                    break
        if not chosen:
            break
        C = np.array(chosen)
        fc = np.asarray(obj(C), dtype=np.float64)
        improved = fc.max() > F.max() + 0.05
        X = np.concatenate([X, C])
        F = np.concatenate([F, fc])
        if log:
            log(f"[mle] surrogate round {r + 1}: {len(C)} proposals, best proposal {fc.max():.3f}, "
                f"best {F.max():.3f}, {obj.evals} exact evals")
        stall = 0 if improved else stall + 1
        if stall >= 2:
            break
    b = int(np.argmax(F))
    return obj, X[b], float(F[b]), net


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


def run(tree: mra.Tree, family="matern", nu=1.5, n_train=2048, grid_k=32, seed=5, train_steps=3000, log=None,
        pretrained=True):
    """All searches on one tree: exact evaluations, sequential exact calls and
    evaluations to within 0.5 nats of the best exact value any of them found."""
    lo, hi = box2()
    width = hi - lo
    t0 = time.time()
    g = ExactObjective(tree, family, nu)
    xg, fg = grid_search(g, grid_k, log=log)
    tg = time.time() - t0

    t0 = time.time()
    c = ExactObjective(tree, family, nu)
    xc, fc = nelder_mead(c, (lo + hi) / 2, width / 4)
    tc = time.time() - t0
    if log:
        log(f"[mle] Nelder-Mead without the surrogate: {c.evals} evals, best {fc:.3f}")

    t0 = time.time()
    b = ExactObjective(tree, family, nu)
    xb, fb = trust_region(b, (lo + hi) / 2, 0.25)
    tb = time.time() - t0
    if log:
        log(f"[mle] trust region (quadratic models): {b.evals} evals, best {fb:.3f}")

    t0 = time.time()
    q, xq, fq, _ = surrogate_sequential(tree, family, nu, seed=seed, log=log)
    tq = time.time() - t0

    found = [fg, fc, fb, fq]
    res_p = None
    if pretrained:
        net, n_tr = train_surrogate(tree, n_train, seed, train_steps, family=family, nu=nu, log=log)
        s = ExactObjective(tree, family, nu)
        x0 = surrogate_proposal(net)
        f0 = float(s(x0)[0])
        xs, fs = nelder_mead(s, x0, width / 32)
        found.append(fs)
        res_p = {"train_evals": n_tr, "search_evals": s.evals, "total_evals": n_tr + s.evals,
                 "proposal_loglik": f0, "loglik": fs, "beta": math.exp(xs[0]), "lam": math.exp(xs[1])}

    best = max(found)
    target = best - 0.5

    def entry(o, x, f, wall):
        return {"evals": o.evals, "calls": o.calls, "evals_to_mle": o.evals_to_reach(target), "loglik": f,
                "beta": math.exp(x[0]), "lam": math.exp(x[1]), "alpha": o.alpha_hat(x), "wall_s": wall}

    res = {
        "best_loglik": best,
        "grid": entry(g, xg, fg, tg),
        "local": entry(c, xc, fc, tc),
        "trust_region": entry(b, xb, fb, tb),
        "surrogate": entry(q, xq, fq, tq),
    }
    if res_p is not None:
        res_p["evals_to_mle"] = s.evals_to_reach(target)
        res["surrogate_pretrained"] = res_p
    if log:
        log(f"[mle] grid {grid_k}x{grid_k}: {g.evals} evals, best {fg:.3f}; Nelder-Mead {c.evals} evals "
            f"({c.calls} calls), best {fc:.3f}; trust region {b.evals} evals ({b.calls} calls), best {fb:.3f}; "
            f"surrogate {q.evals} evals ({q.calls} calls), best {fq:.3f}")
    return res
