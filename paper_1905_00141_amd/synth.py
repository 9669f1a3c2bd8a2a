"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds only input generation: locations, field values and
covariance-parameter sets.  It contains none of the MRA arithmetic (no tree,
no knots, no recursion); both the HIP path and the CPU oracle consume what it
produces.

The paper's workloads (gridded satellite land-surface temperature with a
missing-value mask, and sea-surface-temperature swaths with strongly uneven
leaf counts, Sec. 4 and 5) are not available here; these generators stand in
for them with the same structure: uniform and clustered 2-D locations,
mean-zero Gaussian-process-like values and a nugget.

Value generators:
  * exact draw: z = chol(C + tau I) e for an exponential covariance (small n);
  * random Fourier features (Rahimi & Recht): for the Matern family with
    unscaled distance t = d / range (nu = 1/2: exp(-t); nu = 3/2:
    (1 + t) exp(-t)) the spectral measure is a bivariate Student-t with
    2 nu degrees of freedom, sampled as w = g / (range * sqrt(c)), g ~ N(0, I2),
    c ~ chi^2_{2 nu}; f(s) = sqrt(alpha) sqrt(2/D) sum_j cos(w_j . s + b_j).
"""
from __future__ import annotations

import math

import numpy as np

LN_OFFSET_DEFAULT = math.e / 100.0


def uniform_locations(n: int, seed: int):
    rng = np.random.default_rng(seed)
    return rng.random(n), rng.random(n)


# Component scales of the batched n = 2^20 workload, calibrated so that the
# finest-level counts (M = 9, 65536 leaves, seed 3) reach the stated top of
# about 512: the realised counts are 0..515 (median 9, 1 % of leaves at most
# 1, 133 empty).  A 16-component mixture cannot keep every leaf at 8 or more
# observations; the widest components (sigma near 2) act as a background.
MIXTURE_SIGMA_RANGE = (0.015, 2.0)


def mixture_locations(n: int, seed: int, k: int = 16, sigma_range=MIXTURE_SIGMA_RANGE):
    """n points from k equal-weight isotropic Gaussians on [0,1]^2 (rejection
    outside the unit square).  Means ~ U[0.1, 0.9]^2, sigmas log-uniform."""
    rng = np.random.default_rng(seed)
    mu = rng.uniform(0.1, 0.9, size=(k, 2))
    sig = np.exp(rng.uniform(np.log(sigma_range[0]), np.log(sigma_range[1]), size=k))
    xs, ys = [], []
    need = n
    while need > 0:
        m = int(need * 1.3) + 64
        comp = rng.integers(0, k, size=m)
        p = mu[comp] + sig[comp, None] * rng.standard_normal((m, 2))
        ok = (p[:, 0] >= 0) & (p[:, 0] < 1) & (p[:, 1] >= 0) & (p[:, 1] < 1)
        p = p[ok][:need]
        xs.append(p[:, 0]); ys.append(p[:, 1])
        need -= len(p)
    return np.concatenate(xs), np.concatenate(ys)


def exact_exponential_draw(x, y, alpha, beta, tau, seed):
    """z ~ N(0, alpha exp(-d/beta) + tau I) by a dense Cholesky (n up to a few thousand)."""
    rng = np.random.default_rng(seed)
    d = np.hypot(x[:, None] - x[None, :], y[:, None] - y[None, :])
    K = alpha * np.exp(-d / beta) + tau * np.eye(len(x))
    return np.linalg.cholesky(K) @ rng.standard_normal(len(x))


def rff_field(xs, ys, alpha, beta, nu, n_features, seed, device="cpu", chunk=1 << 16):
    """Random-Fourier-feature draw of a Matern(nu) field at every (x, y) set in
    xs/ys (lists of arrays), all from one set of features.  Evaluated in FP64
    with torch on `device` (cpu or cuda) for speed; returns numpy arrays."""
    import torch

    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n_features, 2))
    c = rng.chisquare(2.0 * nu, size=n_features)
    w = g / (beta * np.sqrt(c))[:, None]
    b = rng.uniform(0.0, 2.0 * np.pi, size=n_features)
    scale = math.sqrt(alpha) * math.sqrt(2.0 / n_features)
    W = torch.tensor(w.T.copy(), dtype=torch.float64, device=device)  # 2 x D
    Bt = torch.tensor(b, dtype=torch.float64, device=device)
    outs = []
    for x, y in zip(xs, ys):
        out = np.empty(len(x))
        for s in range(0, len(x), chunk):
            P = torch.tensor(np.stack([x[s:s + chunk], y[s:s + chunk]], axis=1),
                             dtype=torch.float64, device=device)
            out[s:s + chunk] = (torch.cos(P @ W + Bt).sum(dim=1) * scale).cpu().numpy()
        outs.append(out)
    return outs


def log_spaced(lo, hi, k):
    return np.exp(np.linspace(np.log(lo), np.log(hi), k))


def theta_grid(n_range=8, n_nugget=8, alpha=1.0, r_lo=0.02, r_hi=0.3, t_lo=1e-3, t_hi=1e-1):
    """Range-major, nugget-minor grid of (alpha, range, nugget) rows."""
    th = [(alpha, b, t) for b in log_spaced(r_lo, r_hi, n_range) for t in log_spaced(t_lo, t_hi, n_nugget)]
    return np.array(th, dtype=np.float64)


# ---------------------------------------------------------------------------
# The five workloads.  Each returns a dict with locations, values, tree shape,
# covariance family and parameter sets.  `scale` < 1 shrinks n (and M where it
# keeps the per-leaf count) for parity cases the oracle finishes in seconds.
# ---------------------------------------------------------------------------

def config1(seed=1):
    n = 4096
    x, y = uniform_locations(n, seed)
    z = exact_exponential_draw(x, y, 1.0, 0.05, 0.05, seed + 100)
    return dict(name="cfg1_uniform4096_exp_M4_J4_r32", x=x, y=y, z=z, J=4, r=32, M=4,
                domain=None, family="matern", nu=0.5, theta=np.array([[1.0, 0.05, 0.05]]))


def config2(seed=2, device="cpu", n=131072, M=7, n_pred=16384):
    x, y = uniform_locations(n, seed)
    rng = np.random.default_rng(seed + 1000)
    px, py = rng.random(n_pred), rng.random(n_pred)
    f, fp = rff_field([x, px], [y, py], 1.0, 0.1, 1.5, 4096, seed + 200, device=device)
    z = f + math.sqrt(0.01) * np.random.default_rng(seed + 300).standard_normal(n)
    return dict(name=f"cfg2_uniform{n}_matern1.5_M{M}_J4_r64", x=x, y=y, z=z, J=4, r=64, M=M,
                domain=np.array([0.0, 1.0, 0.0, 1.0]), family="matern", nu=1.5,
                theta=np.array([[1.0, 0.1, 0.01]]), px=px, py=py, truth=fp)


def config3(seed=3, device="cpu", n=1 << 20, M=9, n_theta=(8, 8)):
    x, y = mixture_locations(n, seed)
    (f,) = rff_field([x], [y], 1.0, 0.1, 1.5, 4096, seed + 200, device=device)
    z = f + math.sqrt(0.01) * np.random.default_rng(seed + 300).standard_normal(n)
    return dict(name=f"cfg3_mixture{n}_matern1.5_M{M}_J4_r64_theta{n_theta[0] * n_theta[1]}",
                x=x, y=y, z=z, J=4, r=64, M=M,
                domain=np.array([0.0, 1.0, 0.0, 1.0]), family="matern", nu=1.5,
                theta=theta_grid(*n_theta))


def config4(seed=4, device="cpu", n=1 << 23, M=10):
    x, y = uniform_locations(n, seed)
    (f,) = rff_field([x], [y], 1.0, 0.05, 0.5, 1024, seed + 200, device=device)
    z = f + math.sqrt(0.02) * np.random.default_rng(seed + 300).standard_normal(n)
    return dict(name=f"cfg4_uniform{n}_matern0.5_M{M}_J4_r32", x=x, y=y, z=z, J=4, r=32, M=M,
                domain=np.array([0.0, 1.0, 0.0, 1.0]), family="matern", nu=0.5,
                theta=np.array([[1.0, 0.05, 0.02]]))


def small_case(seed, n, J=4, r=16, M=3, cluster=False, nu=0.5):
    """A small random problem for parity tests."""
    if cluster:
        x, y = mixture_locations(n, seed, k=4, sigma_range=(0.02, 0.2))
    else:
        x, y = uniform_locations(n, seed)
    rng = np.random.default_rng(seed + 7)
    z = rng.standard_normal(n)
    return dict(x=x, y=y, z=z, J=J, r=r, M=M, nu=nu)


# ---------------------------------------------------------------------------
# Surrogate network: initial parameters and the training design.
# ---------------------------------------------------------------------------

MLP_WIDTH = 128
MLP_LAYERS = [(128, 3), (128, 128), (128, 128), (128, 128), (1, 128)]  # (fan_out, fan_in)


def mlp_init(seed):
    """Initial parameters (float32, the library's order: W1, b1, ..., w5, b5):
    weights uniform in +-sqrt(6 / (fan_in + fan_out)), biases zero."""
    rng = np.random.default_rng(seed)
    parts = []
    for fo, fi in MLP_LAYERS:
        lim = np.sqrt(6.0 / (fi + fo))
        parts.append(rng.uniform(-lim, lim, size=fo * fi))
        parts.append(np.zeros(fo))
    return np.concatenate(parts).astype(np.float32)


def sobol_box(n, lo, hi, seed):
    """n scrambled Sobol points in the box [lo, hi] (per coordinate)."""
    from scipy.stats import qmc
    s = qmc.Sobol(d=len(lo), scramble=True, seed=seed).random(n)
    lo, hi = np.asarray(lo, dtype=np.float64), np.asarray(hi, dtype=np.float64)
    return lo + s * (hi - lo)


# Config 5: the surrogate's log-parameter box (log alpha, log beta, log tau).
# The sill range reaches 16 so that the box holds the profiled sill at the
# maximum of the config-3 likelihood (about 8.6 at range 0.26).
SURROGATE_BOX_LO = np.log([0.25, 0.02, 1e-3])
SURROGATE_BOX_HI = np.log([16.0, 0.3, 1e-1])
