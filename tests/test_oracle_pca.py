"""Pins for the oracle's PCA (CPU only).

* Data built with a known covariance: X = mu + U S Q^T with U's columns
  centred and orthonormal, so the covariance is Q diag(S^2 / (n - 1)) Q^T
  exactly: the eigenvalues and (sign-fixed) eigenvectors are known.
* With all components kept the projection is a rotation: pairwise distances
  are preserved.
* Translating X changes only the mean.
"""
import numpy as np
import pytest


def _known(n=500, d=12, seed=0):
    rng = np.random.default_rng(seed)
    G = rng.normal(size=(n, d))
    G -= G.mean(axis=0)
    U, _ = np.linalg.qr(G)                      # centred (columns sum to ~0) and orthonormal
    U -= U.mean(axis=0)
    U, _ = np.linalg.qr(U)
    Q, _ = np.linalg.qr(rng.normal(size=(d, d)))
    S = np.linspace(10.0, 1.0, d)               # distinct singular values
    mu = rng.normal(size=d)
    return mu + (U * S) @ Q.T, Q, S, mu


def test_known_covariance(orc):
    n, d = 500, 12
    X, Q, S, mu = _known(n, d)
    Z, V, w, m = orc.pca(X, 5)
    np.testing.assert_allclose(w, (S[:5] ** 2) / (n - 1), rtol=1e-10)
    np.testing.assert_allclose(m, mu, atol=1e-12)
    for j in range(5):
        q = Q[:, j] * np.sign(Q[np.argmax(np.abs(Q[:, j])), j])
        np.testing.assert_allclose(V[:, j], q, atol=1e-10)
        assert V[np.argmax(np.abs(V[:, j])), j] > 0
    np.testing.assert_allclose(Z, (X - mu) @ V, atol=1e-10)


def test_all_components_preserve_distances(orc):
    rng = np.random.default_rng(3)
    X = rng.normal(size=(200, 7)) * np.arange(1, 8)
    Z, V, w, _ = orc.pca(X, 7)
    np.testing.assert_allclose(V.T @ V, np.eye(7), atol=1e-12)
    i, j = rng.integers(0, 200, size=(2, 300))
    np.testing.assert_allclose(np.linalg.norm(Z[i] - Z[j], axis=1), np.linalg.norm(X[i] - X[j], axis=1),
                               rtol=1e-12)
    assert np.all(np.diff(w) <= 0)


def test_translation_changes_only_the_mean(orc):
    X, _, _, _ = _known(300, 6, seed=2)
    Z1, V1, w1, m1 = orc.pca(X, 3)
    Z2, V2, w2, m2 = orc.pca(X + 100.0, 3)
    np.testing.assert_allclose(V1, V2, atol=1e-9)
    np.testing.assert_allclose(w1, w2, rtol=1e-9)
    np.testing.assert_allclose(Z1, Z2, atol=1e-8)
    np.testing.assert_allclose(m2 - m1, 100.0, atol=1e-12)
