"""Seeded synthetic inputs for the kNN-graph workloads.

This module only draws numbers: it holds none of the kNN method's arithmetic,
and both the HIP path's tests/benchmarks and the CPU oracle's tests take their
inputs from it.  Every generator is a pure function of its seed (NumPy PCG64).

The workloads stand in for the paper's datasets (Fashion-MNIST 70K x 784 and
GloVe-Twitter up to 10M points, Benchmarks section), which are not used here:

* ``gmm_isotropic``  - small isotropic Gaussian mixture (5,000 x 50, 10 comps),
  means ~ N(0, 4I), unit-variance components, equal weights.
* ``pixel_like``     - 70,000 x 784 image-like data: 10 cluster prototypes on
  a 28x28 grid with ~50% background that stays exactly 0; foreground values
  round(255 * clip(p + N(0, 0.15^2), 0, 1)) / 255 with p in [0.2, 1].
* ``gmm_anisotropic`` - Gaussian mixture with covariances Q diag(lam) Q^T,
  Q Haar-random, lam log-uniform on [0.1, 10], means ~ N(0, 4I); equal or
  Zipf(s) component weights.
* small structured cases for closed-form checks: sorted line, integer
  lattice, duplicated points, well-separated clusters.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "gmm_isotropic", "pixel_like", "gmm_anisotropic", "line_1d", "lattice",
    "with_duplicates", "separated_clusters", "sample_queries", "uniform_cube",
]


def gmm_isotropic(n: int = 5000, d: int = 50, comps: int = 10, seed: int = 0,
                  mean_std: float = 2.0, dtype=np.float32) -> np.ndarray:
    """Equal-weight isotropic mixture: x = mu_c + N(0, I), mu_c ~ N(0, mean_std^2 I)."""
    rng = np.random.default_rng(seed)
    mu = rng.normal(0.0, mean_std, size=(comps, d))
    lab = rng.integers(0, comps, size=n)
    x = mu[lab] + rng.normal(0.0, 1.0, size=(n, d))
    return np.ascontiguousarray(x.astype(dtype))


def _smooth2d(a: np.ndarray, passes: int = 2) -> np.ndarray:
    """Cheap 3x3 box blur on a stack of 28x28 images (edge-replicated)."""
    for _ in range(passes):
        p = np.pad(a, ((0, 0), (1, 1), (1, 1)), mode="edge")
        a = sum(p[:, i:i + a.shape[1], j:j + a.shape[2]]
                for i in range(3) for j in range(3)) / 9.0
    return a


def pixel_like(n: int = 70000, side: int = 28, comps: int = 10, seed: int = 0,
               noise_std: float = 0.15, fg_frac: float = 0.5,
               chunk: int = 8192) -> np.ndarray:
    """Quantised image-like clusters (values are multiples of 1/255, float32).

    Each prototype has a smooth random foreground mask covering ``fg_frac`` of
    the pixels; background pixels are exactly 0 in every sample.  Foreground
    intensities are a smoothed U(0.2, 1) field; a sample adds N(0, noise_std^2)
    per foreground pixel, clips to [0, 1] and rounds to the 1/255 grid.
    """
    rng = np.random.default_rng(seed)
    d = side * side
    field = _smooth2d(rng.random((comps, side, side)), passes=3)
    thr = np.quantile(field.reshape(comps, -1), 1.0 - fg_frac, axis=1)
    mask = (field.reshape(comps, -1) > thr[:, None])
    inten = _smooth2d(rng.uniform(0.2, 1.0, size=(comps, side, side)), 1).reshape(comps, d)
    proto = np.where(mask, inten, 0.0)
    lab = rng.integers(0, comps, size=n)
    out = np.empty((n, d), dtype=np.float32)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        p = proto[lab[s:e]]
        v = np.clip(p + rng.normal(0.0, noise_std, size=p.shape), 0.0, 1.0)
        q = np.rint(255.0 * v) / 255.0
        out[s:e] = np.where(mask[lab[s:e]], q, 0.0).astype(np.float32)
    return out


def gmm_anisotropic(n: int = 1_000_000, d: int = 50, comps: int = 50, seed: int = 0,
                    zipf: float | None = None, lam_lo: float = 0.1, lam_hi: float = 10.0,
                    mean_std: float = 2.0, dtype=np.float32,
                    chunk: int = 262144) -> np.ndarray:
    """Anisotropic Gaussian mixture (Haar rotations, log-uniform spectra).

    Component weights are equal, or proportional to c^-zipf (c = 1..comps) when
    ``zipf`` is given.  Sampling is chunked so 10M x 50 fits in host memory.
    """
    rng = np.random.default_rng(seed)
    mu = rng.normal(0.0, mean_std, size=(comps, d))
    rot = np.empty((comps, d, d))
    sq = np.empty((comps, d))
    for c in range(comps):
        g = rng.normal(size=(d, d))
        q, r = np.linalg.qr(g)
        q = q * np.sign(np.diag(r))[None, :]   # Haar measure
        rot[c] = q
        sq[c] = np.sqrt(np.exp(rng.uniform(np.log(lam_lo), np.log(lam_hi), size=d)))
    if zipf is None:
        w = np.full(comps, 1.0 / comps)
    else:
        w = np.arange(1, comps + 1, dtype=np.float64) ** (-zipf)
        w /= w.sum()
    lab = rng.choice(comps, size=n, p=w)
    out = np.empty((n, d), dtype=dtype)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        lb = lab[s:e]
        z = rng.normal(size=(e - s, d))
        x = np.empty((e - s, d))
        for c in np.unique(lb):
            m = lb == c
            x[m] = mu[c] + (z[m] * sq[c]) @ rot[c].T
        out[s:e] = x.astype(dtype)
    return out


def uniform_cube(n: int, d: int, seed: int = 0, dtype=np.float32) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.random((n, d)).astype(dtype)


def line_1d(n: int, seed: int = 0, dtype=np.float32) -> np.ndarray:
    """n distinct points on a line, in random order (n x 1).

    Gaps are distinct powers-free random values so that no two neighbours of a
    point are equidistant (the window property then fixes the kNN uniquely).
    """
    rng = np.random.default_rng(seed)
    gaps = rng.uniform(1.0, 2.0, size=n)
    pos = np.cumsum(gaps)
    perm = rng.permutation(n)
    return pos[perm].reshape(n, 1).astype(dtype)


def lattice(side: int, dim: int, seed: int | None = None, dtype=np.float32) -> np.ndarray:
    """All points of {0..side-1}^dim (integer coordinates), optionally shuffled."""
    grids = np.meshgrid(*[np.arange(side)] * dim, indexing="ij")
    pts = np.stack([g.reshape(-1) for g in grids], axis=1).astype(dtype)
    if seed is not None:
        pts = pts[np.random.default_rng(seed).permutation(len(pts))]
    return np.ascontiguousarray(pts)


def with_duplicates(n_unique: int, d: int, copies: int, seed: int = 0,
                    dtype=np.float32) -> np.ndarray:
    """n_unique random points, each repeated ``copies`` times, shuffled."""
    rng = np.random.default_rng(seed)
    base = rng.normal(size=(n_unique, d)).astype(dtype)
    x = np.repeat(base, copies, axis=0)
    return np.ascontiguousarray(x[rng.permutation(len(x))])


def separated_clusters(n_per: int, comps: int, d: int, sep: float = 1000.0,
                       seed: int = 0, dtype=np.float32):
    """Clusters of n_per points each, centres ``sep`` apart; returns (X, labels)."""
    rng = np.random.default_rng(seed)
    centres = np.zeros((comps, d))
    centres[:, 0] = sep * np.arange(comps)
    lab = np.repeat(np.arange(comps), n_per)
    x = centres[lab] + rng.normal(size=(comps * n_per, d))
    perm = rng.permutation(len(x))
    return np.ascontiguousarray(x[perm].astype(dtype)), lab[perm]


def sample_queries(n: int, m: int, seed: int = 2) -> np.ndarray:
    """m distinct row indices in [0, n), drawn without replacement, sorted."""
    rng = np.random.default_rng(seed)
    m = min(m, n)
    return np.sort(rng.choice(n, size=m, replace=False)).astype(np.int64)
