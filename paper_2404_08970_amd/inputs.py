"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module only draws random numbers and builds marginals / plans of the shapes
the paper's experiments use; it contains none of the method's arithmetic and it
is the one piece of code that both the HIP path and the CPU checker consume.

Workload recipes (the paper's datasets are not used):

* 1D random marginals: U[0,1] entries then normalised (Sec. 5.1 setup).
* 1D Gaussian mixtures: 3 components, means U[0.1, 0.9], sigma U[0.02, 0.1],
  equal weights, pdf sampled at x_i = i/(n-1), normalised.  Tail entries may
  underflow to exactly 0.
* 2D blobs: U{1..5} isotropic Gaussian blobs on an H x W grid over [0,1]^2,
  centres U[0.1, 0.9]^2, sigma U[0.02, 0.1], normalised, optional floor added
  then renormalised.
* Dirichlet(alpha=1) marginals.
* Random non-negative plans with unit mass for gradient tests.
* Request stream for the request loop: 70% 1D grids with n ~ U{128..8192},
  30% square 2D grids with side s ~ U{16..96} (L1POW), X and Y of the same
  size with independently drawn marginals (mixtures in 1D, blobs without
  floor in 2D), k ~ U{1,2}, eps ~ U[1e-3, 1e-2], Poisson arrivals.
"""
from __future__ import annotations

import numpy as np


def rng_for(*key: int) -> np.random.Generator:
    return np.random.default_rng(list(int(k) for k in key))


def uniform_marginal(n: int, rng: np.random.Generator) -> np.ndarray:
    v = rng.uniform(0.0, 1.0, size=n)
    return v / v.sum()


def gauss_mixture_1d(n: int, rng: np.random.Generator, ncomp: int = 3,
                     mean_range=(0.1, 0.9), sigma_range=(0.02, 0.1),
                     floor: float = 0.0) -> np.ndarray:
    x = np.arange(n, dtype=np.float64) / max(n - 1, 1)
    means = rng.uniform(*mean_range, size=ncomp)
    sig = rng.uniform(*sigma_range, size=ncomp)
    v = np.zeros(n)
    for m, s in zip(means, sig):
        v += np.exp(-0.5 * ((x - m) / s) ** 2) / (s * np.sqrt(2 * np.pi))
    v = v / v.sum()
    if floor > 0:
        v = (v + floor)
        v = v / v.sum()
    return v


def blobs_2d(H: int, W: int, rng: np.random.Generator, floor: float = 0.0,
             nblobs=None, mean_range=(0.1, 0.9), sigma_range=(0.02, 0.1)) -> np.ndarray:
    """Flattened row-major H*W image of Gaussian blobs, normalised."""
    if nblobs is None:
        nblobs = int(rng.integers(1, 6))
    r = np.arange(H, dtype=np.float64) / max(H - 1, 1)
    c = np.arange(W, dtype=np.float64) / max(W - 1, 1)
    R, Cc = np.meshgrid(r, c, indexing="ij")
    img = np.zeros((H, W))
    for _ in range(nblobs):
        mr, mc = rng.uniform(*mean_range, size=2)
        s = rng.uniform(*sigma_range)
        img += np.exp(-0.5 * (((R - mr) / s) ** 2 + ((Cc - mc) / s) ** 2))
    img = img / img.sum()
    if floor > 0:
        img = img + floor
        img = img / img.sum()
    return img.reshape(-1)


def blobs_3d(D: int, H: int, W: int, rng: np.random.Generator, floor: float = 0.0,
             nblobs=None, mean_range=(0.1, 0.9), sigma_range=(0.05, 0.2)) -> np.ndarray:
    """Flattened row-major D*H*W volume of isotropic Gaussian blobs, normalised."""
    if nblobs is None:
        nblobs = int(rng.integers(1, 6))
    axes = [np.arange(e, dtype=np.float64) / max(e - 1, 1) for e in (D, H, W)]
    Z, R, Cc = np.meshgrid(*axes, indexing="ij")
    vol = np.zeros((D, H, W))
    for _ in range(nblobs):
        mz, mr, mc = rng.uniform(*mean_range, size=3)
        s = rng.uniform(*sigma_range)
        vol += np.exp(-0.5 * (((Z - mz) / s) ** 2 + ((R - mr) / s) ** 2 + ((Cc - mc) / s) ** 2))
    vol = vol / vol.sum()
    if floor > 0:
        vol = vol + floor
        vol = vol / vol.sum()
    return vol.reshape(-1)


def dirichlet(n: int, rng: np.random.Generator, alpha: float = 1.0) -> np.ndarray:
    return rng.dirichlet(np.full(n, alpha))


def random_plan(M: int, N: int, rng: np.random.Generator) -> np.ndarray:
    T = rng.uniform(0.0, 1.0, size=(M, N))
    return T / T.sum()


def peaked_plan(M: int, N: int, rng: np.random.Generator, width: float = 0.02) -> np.ndarray:
    """A plan concentrated near a random monotone curve (the shape converged
    GW plans take), plus a tiny uniform background; unit mass."""
    i = np.arange(M)[:, None] / max(M - 1, 1)
    p = np.arange(N)[None, :] / max(N - 1, 1)
    shift = rng.uniform(-0.1, 0.1)
    T = np.exp(-0.5 * ((p - i - shift) / width) ** 2) + 1e-12
    return T / T.sum()


def integer_plan(M: int, N: int, rng: np.random.Generator, hi: int = 8) -> np.ndarray:
    """Integer-valued non-negative matrix (for bit-exact checks)."""
    return rng.integers(0, hi, size=(M, N)).astype(np.float64)


def serving_requests(count: int, seed: int = 5, n_range=(128, 8192), side_range=(16, 96),
                     frac_1d: float = 0.7, eps_range=(1e-3, 1e-2), rate: float = 1.0):
    """`count` request descriptors: dict(shape, k, eps, p, q, arrival) with
    Poisson arrivals of the given rate (exponential gaps, first at 0)."""
    rng = rng_for(seed)
    out = []
    t = 0.0
    for i in range(count):
        if i > 0:
            t += float(rng.exponential(1.0 / rate))
        k = int(rng.integers(1, 3))
        eps = float(rng.uniform(*eps_range))
        if rng.uniform() < frac_1d:
            n = int(rng.integers(n_range[0], n_range[1] + 1))
            shape = (n,)
            p, q = gauss_mixture_1d(n, rng), gauss_mixture_1d(n, rng)
        else:
            s = int(rng.integers(side_range[0], side_range[1] + 1))
            shape = (s, s)
            p, q = blobs_2d(s, s, rng), blobs_2d(s, s, rng)
        out.append({"shape": shape, "k": k, "eps": eps, "p": p, "q": q, "arrival": t})
    return out
