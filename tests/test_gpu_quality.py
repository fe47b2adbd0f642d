"""Embedding-quality metrics on the GPU (knn_quality) against the oracle.

The per-row terms (|N & L|, the trustworthiness and continuity rank sums)
are integers decided by distance comparisons; both sides take them in the
canonical FP32 precision (the oracle's canonical mode), so they must be
equal element for element, and the metrics built from them to 1e-12.  The
metrics are also compared with the oracle's FP64 definition to 1e-5: the
two differ only where two distances from one point tie within FP32
rounding, each such pair moving a rank sum by one.  Cases: a ragged
3,001-row mixture with a noisy 2-D projection as the embedding (k = 10 and
15), k = 1 and 16, points far from the origin (every pair re-decided
canonically), X in BF16 and FP16, an integer lattice (every rank decided by
index ties), the 70,000 x 784 pixel-like set on 64 sampled rows (its
metrics against the oracle's per-row sums are not available at full size;
the rows are), and 600,000 rows whose rank pass takes two launches."""
import numpy as np
import pytest
import torch

from paper_2603_04035_amd import datagen

pytestmark = pytest.mark.gpu


def _embed(X, seed):
    rng = np.random.default_rng(seed)
    R = rng.normal(size=(X.shape[1], 2)).astype(np.float32)
    return np.ascontiguousarray((X @ R + rng.normal(scale=0.5, size=(X.shape[0], 2))).astype(np.float32))


def _run(X, Y, k):
    import paper_2603_04035_amd as knn
    m, (h, t, c) = knn.quality(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(), k, per_row=True)
    return m, h.cpu().numpy(), t.cpu().numpy(), c.cpu().numpy()


@pytest.mark.parametrize("k", [1, 10, 15, 16])
def test_quality_mixture(orc, k):
    X = datagen.gmm_isotropic(n=3001, d=50, seed=8)
    Y = _embed(X, 1)
    m, h, t, c = _run(X, Y, k)
    oh, ot, oc = orc.quality_rows(X, Y, k, canonical=True)
    assert np.array_equal(h, oh) and np.array_equal(t, ot) and np.array_equal(c, oc)
    n = X.shape[0]
    z = 2.0 / (n * k * (2.0 * n - 3.0 * k - 1.0))
    canon = (oh.sum() / (n * k), 1.0 - z * ot.sum(), 1.0 - z * oc.sum())
    assert np.allclose(m, canon, rtol=0, atol=1e-12)
    # FP64 ranks differ only where two distances from a point tie within
    # FP32 rounding (common among 3,000 points in 2-D): each such pair moves
    # a rank sum by one unit of z
    exp = orc.quality(X, Y, k)
    print("k", k, "gpu", m, "oracle fp64", exp, "one rank unit", z)
    assert np.allclose(m, exp, rtol=0, atol=1e-5)


def test_quality_far_from_origin(orc):
    """Points far from the origin (a mixture shifted by 1000 in every
    coordinate): the Gram distance's error bound then exceeds every pair's
    separation, so the rank pass re-decides every pair canonically (full
    queues, many passes over each tile's rows)."""
    X = np.ascontiguousarray((datagen.gmm_isotropic(n=1500, d=40, seed=12) + 1000.0).astype(np.float32))
    Y = _embed(X - 1000.0, 3)
    m, h, t, c = _run(X, Y, 10)
    oh, ot, oc = orc.quality_rows(X, Y, 10, canonical=True)
    assert np.array_equal(h, oh) and np.array_equal(t, ot) and np.array_equal(c, oc)


@pytest.mark.parametrize("dt", [torch.bfloat16, torch.float16])
def test_quality_half_input(orc, dt):
    """X in BF16 / FP16 (the exact lists' re-rank reads X in its own type,
    widened exactly to FP32): the terms equal the oracle's on X's values."""
    import paper_2603_04035_amd as knn
    X = torch.from_numpy(datagen.gmm_isotropic(n=1201, d=40, seed=21)).to(dt)
    Xv = np.ascontiguousarray(X.float().numpy())
    Y = _embed(Xv, 5)
    m, (h, t, c) = knn.quality(X.cuda(), torch.from_numpy(Y).cuda(), 12, per_row=True)
    oh, ot, oc = orc.quality_rows(Xv, Y, 12, canonical=True)
    assert np.array_equal(h.cpu().numpy(), oh)
    assert np.array_equal(t.cpu().numpy(), ot) and np.array_equal(c.cpu().numpy(), oc)


def test_quality_lattice_ties(orc):
    X = datagen.lattice(14, 3, seed=2)                  # 2,744 points, shells of equal distances
    Y = np.ascontiguousarray(X[:, :2] + 0.01 * X[:, 2:3])
    m, h, t, c = _run(X, Y, 6)
    oh, ot, oc = orc.quality_rows(X, Y, 6, canonical=True)
    assert np.array_equal(h, oh) and np.array_equal(t, ot) and np.array_equal(c, oc)


def test_quality_identity_is_one():
    X = datagen.gmm_anisotropic(n=2000, d=20, comps=5, seed=3)
    m, _, _, _ = _run(X, X, 10)
    assert m == (1.0, 1.0, 1.0)


def test_quality_pixel70k_sampled(orc):
    X = datagen.pixel_like(n=70000, seed=0)
    Y = _embed(X, 2)
    m, h, t, c = _run(X, Y, 10)
    rows = datagen.sample_queries(70000, 64, seed=4)
    oh, ot, oc = orc.quality_rows(X, Y, 10, rows=rows, canonical=True)
    print("pixel70k quality", m)
    assert np.array_equal(h[rows], oh) and np.array_equal(t[rows], ot) and np.array_equal(c[rows], oc)
    assert 0.0 <= m[0] <= 1.0 and 0.0 < m[1] < 1.0 and 0.0 < m[2] < 1.0


def test_quality_two_rank_launches(orc):
    """600,000 x 24 rows: the X-space rank pass (which also keeps X's k-NN
    lists) runs as two launches of query blocks, each writing its counts and
    lists at its own offset; 64 sampled rows against the oracle."""
    X = datagen.gmm_isotropic(n=600_000, d=24, comps=30, seed=31)
    Y = _embed(X, 9)
    m, h, t, c = _run(X, Y, 10)
    rows = np.concatenate([datagen.sample_queries(600_000, 48, seed=6), [0, 524_287, 524_288, 599_999]])
    oh, ot, oc = orc.quality_rows(X, Y, 10, rows=rows, canonical=True)
    assert np.array_equal(h[rows], oh) and np.array_equal(t[rows], ot) and np.array_equal(c[rows], oc)


@pytest.mark.parametrize("n", [12, 50, 129])
def test_quality_small_sets(orc, n):
    """A partial tile (12 and 50 rows) and one row past a tile (129), 20-d
    (the fused rank pass), k = 3: every per-row term against the oracle."""
    X = datagen.gmm_isotropic(n=n, d=20, comps=3, seed=n)
    Y = _embed(X, n + 1)
    m, h, t, c = _run(X, Y, 3)
    oh, ot, oc = orc.quality_rows(X, Y, 3, canonical=True)
    assert np.array_equal(h, oh) and np.array_equal(t, ot) and np.array_equal(c, oc)
    z = 2.0 / (n * 3 * (2.0 * n - 3.0 * 3 - 1.0))
    assert np.allclose(m, (oh.sum() / (n * 3), 1.0 - z * ot.sum(), 1.0 - z * oc.sum()), rtol=0, atol=1e-12)


def test_quality_rejects_bad_k():
    import paper_2603_04035_amd as knn
    X = torch.zeros((30, 4), device="cuda")
    with pytest.raises(knn.KnnError):
        knn.quality(X, X, 17)
    with pytest.raises(knn.KnnError):
        knn.quality(X, X, 20)
