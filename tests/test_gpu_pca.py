"""PCA on the GPU (knn_pca) against the oracle's FP64 eigh.

Mean and covariance-derived quantities are FP64 on both sides; the GPU's
Gram sums FP64 products in another order, so eigenvalues agree to 1e-10
relative, and eigenvectors to eps / gap (gap = relative distance to the
nearest other eigenvalue, which the cases keep above 1e-3): 1e-8.  The
projection is compared in FP32 (the output type): 1e-5 of the row norm.
Cases: a full decomposition (p = d = 12, no iteration), 200,000 rows of the
50-d anisotropic mixture reduced to 10 (subspace iteration), the 70,000 x
784 pixel-like set reduced to 50 (a covariance with a 392-dimensional null
space: its background pixels are always 0), a spectrum over 12 decades
(orthonormalisation after every product), a ragged n, and BF16 input."""
import numpy as np
import pytest
import torch

from paper_2603_04035_amd import datagen

pytestmark = pytest.mark.gpu


def _check(orc, Xnp, p, Xd=None, vec_tol=1e-8):
    import paper_2603_04035_amd as knn
    X = torch.from_numpy(Xnp).cuda() if Xd is None else Xd
    Z, V, w, mu = knn.pca(X, p)
    Z, V, w, mu = Z.cpu().numpy(), V.cpu().numpy(), w.cpu().numpy(), mu.cpu().numpy()
    Xv = Xnp if Xd is None else Xd.float().cpu().numpy()
    oZ, oV, ow, omu = orc.pca(Xv, p)
    np.testing.assert_allclose(mu, omu, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(w, ow, rtol=1e-10)
    err = np.abs(V - oV).max(axis=0)
    print("p", p, "eigenvalues", w[:4], "max vector error", err.max())
    assert np.all(err <= vec_tol), err
    scale = np.linalg.norm(oZ, axis=1, keepdims=True) + 1e-30
    assert np.all(np.abs(Z - oZ) <= 1e-5 * scale + 1e-6)


def test_pca_full_decomposition(orc):
    rng = np.random.default_rng(1)
    X = (rng.normal(size=(3001, 12)) * np.linspace(3, 0.5, 12) + 5.0).astype(np.float32)
    _check(orc, X, 12)


def test_pca_gmm_subspace(orc):
    X = datagen.gmm_anisotropic(n=200_000, d=50, comps=50, seed=0)
    _check(orc, X, 10)


def test_pca_pixel70k(orc):
    """Nine strong components (the ten cluster prototypes) over a near-flat
    noise spectrum: components 10-50 have relative gaps down to 1e-3, so
    only their eigenvalues and the span are compared (the vectors inside a
    near-degenerate bulk are not determined); the first nine are compared
    as vectors."""
    import paper_2603_04035_amd as knn
    X = datagen.pixel_like(n=70000, seed=0)
    Z, V, w, mu = knn.pca(torch.from_numpy(X).cuda(), 50)
    Z, V, w = Z.cpu().numpy(), V.cpu().numpy(), w.cpu().numpy()
    oZ, oV, ow, _ = orc.pca(X, 50)
    np.testing.assert_allclose(w, ow, rtol=1e-8)
    assert np.abs(V[:, :9] - oV[:, :9]).max() <= 1e-8
    assert np.abs(V.T @ V - np.eye(50)).max() <= 1e-10
    # the span: the oracle's top-50 basis projected on the GPU's
    resid = oV - V @ (V.T @ oV)
    print("pixel eigenvalues", w[:10], "span residual", np.abs(resid).max())
    assert np.abs(resid).max() <= 1e-4
    scale = np.linalg.norm(oZ[:, :9], axis=1, keepdims=True) + 1e-30
    assert np.all(np.abs(Z[:, :9] - oZ[:, :9]) <= 1e-5 * scale + 1e-6)


@pytest.mark.parametrize("p", [5, 20])
def test_pca_steep_spectrum(orc, p):
    """Singular values falling geometrically over 6 decades (eigenvalues
    over 12): the basis is badly conditioned after a few products, so the
    products between orthonormalisations must adapt (and the eigenvalues
    still match to 1e-10 relative)."""
    rng = np.random.default_rng(5)
    n, d = 6000, 40
    G = rng.normal(size=(n, d))
    G -= G.mean(axis=0)
    U, _ = np.linalg.qr(G)
    U -= U.mean(axis=0)
    U, _ = np.linalg.qr(U)
    Q, _ = np.linalg.qr(rng.normal(size=(d, d)))
    S = np.geomspace(1e3, 1e-3, d)
    X = (3.0 + (U * S) @ Q.T).astype(np.float32)
    _check(orc, X, p)


def test_pca_bf16_input(orc):
    X = datagen.gmm_anisotropic(n=20_001, d=40, comps=8, seed=3)
    Xb = torch.from_numpy(X).cuda().to(torch.bfloat16)
    _check(orc, X, 8, Xd=Xb)
