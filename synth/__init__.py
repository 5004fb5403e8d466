"""Seeded synthetic workloads for the hierarchical kernel solver.

This module only draws random inputs (points, right-hand sides, targets and
per-problem parameters) with numpy's PCG64.  It holds none of the method's
arithmetic, so both the oracle side and the GPU side may use it.

The paper measures on real datasets that are not available here; seeded
Gaussian mixtures of the same shape stand in for them.  Config k uses the
generator seed 170102324 + k and the method's own sampling seed 170102324 + k.
"""
from __future__ import annotations

import numpy as np

BASE_SEED = 170102324


def rng_for(k: int, salt: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(BASE_SEED + k + 1000 * salt))


def gaussian_mixture(rng, N, d, k, center_lo, center_hi, sigma_lo=1.0, sigma_hi=None):
    """N points from k isotropic Gaussians: centres ~ U[lo,hi]^d, labels uniform,
    x = c_z + sigma_z * eps with sigma_z ~ U[sigma_lo, sigma_hi] (fixed if hi is None)."""
    centers = rng.uniform(center_lo, center_hi, size=(k, d))
    if sigma_hi is None:
        sig = np.full(k, float(sigma_lo))
    else:
        sig = rng.uniform(sigma_lo, sigma_hi, size=k)
    z = rng.integers(0, k, size=N)
    X = centers[z] + sig[z, None] * rng.standard_normal((N, d))
    return np.ascontiguousarray(X, dtype=np.float64)


def config(k: int, N: int | None = None, nrhs: int | None = None):
    """Workload k (1, 2, 3 or 5); N / nrhs override the sizes for reduced runs.

    Returns a dict with X (N x d), B (N x nrhs), and h, lam, m, s, nsamp, seed."""
    rng = rng_for(k)
    if k == 1:
        N = N or 4096; nrhs = nrhs or 1
        X = rng.uniform(0.0, 1.0, size=(N, 3))
        p = dict(h=0.5, lam=1.0, m=64, s=32)
    elif k == 2:
        N = N or 65536; nrhs = nrhs or 16
        X = gaussian_mixture(rng, N, 8, 8, -5.0, 5.0, 1.0)
        p = dict(h=1.0, lam=0.1, m=256, s=128)
    elif k == 3:
        N = N or 1 << 20; nrhs = nrhs or 64
        X = gaussian_mixture(rng, N, 16, 32, -10.0, 10.0, 0.5, 2.0)
        p = dict(h=2.0, lam=0.01, m=512, s=256)
    elif k == 5:
        N = N or 1 << 18; nrhs = nrhs or 4
        X = gaussian_mixture(rng, N, 8, 8, -5.0, 5.0, 1.0)
        p = dict(h=1.0, lam=0.05, m=256, s=128)
    else:
        raise ValueError(f"no single-problem workload {k}")
    B = rng.standard_normal((N, nrhs))
    out = dict(X=np.ascontiguousarray(X, dtype=np.float64), B=np.ascontiguousarray(B), nsamp=4 * p["s"],
               seed=BASE_SEED + k, **p)
    if k == 5:
        out["Y"] = rng.standard_normal((N, nrhs))
    return out


def batched_problems(count: int = 256, nrhs: int = 8, nmin: int = 2048, nmax: int = 32768):
    """Many independent problems of uneven size: N_p = round(exp(U[ln nmin, ln nmax])),
    d = 8, 4 clusters with centres ~ U[-5,5]^8 and sigma = 1, h_p ~ U[0.5, 2],
    lambda_p = 10^U[-3, 0], m = 128, s = 64."""
    rng = rng_for(4)
    probs = []
    for p in range(count):
        N = int(np.rint(np.exp(rng.uniform(np.log(nmin), np.log(nmax)))))
        X = gaussian_mixture(rng, N, 8, 4, -5.0, 5.0, 1.0)
        h = float(rng.uniform(0.5, 2.0))
        lam = float(10.0 ** rng.uniform(-3.0, 0.0))
        B = rng.standard_normal((N, nrhs))
        probs.append(dict(X=X, B=B, h=h, lam=lam, m=128, s=64, nsamp=256, seed=BASE_SEED + 4, problem=p))
    return probs


def small(N: int, d: int, seed: int, nrhs: int = 1, kind: str = "uniform", scale: float = 1.0):
    """Small test inputs: uniform in [0, scale]^d or a 4-cluster mixture."""
    rng = np.random.Generator(np.random.PCG64(BASE_SEED + 7919 * seed))
    if kind == "uniform":
        X = rng.uniform(0.0, scale, size=(N, d))
    else:
        X = gaussian_mixture(rng, N, d, 4, -scale, scale, 1.0)
    B = rng.standard_normal((N, nrhs))
    return np.ascontiguousarray(X), np.ascontiguousarray(B)
