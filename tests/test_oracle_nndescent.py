"""Pins for the oracle's sequential NNDescent (CPU only).

The paper prints no recall or iteration count for its NNDescent, so the
oracle is pinned by invariants of the method (lists valid and sorted, stored
distances true, every approximate rank-r distance at least the exact one,
per-row monotone improvement across iterations), by special cases (k = n - 1
is exact from the start; zero iterations is the sorted random init), by the
early-termination rule delta * n * K, and by recall against the exact oracle.
"""
import numpy as np
import pytest

from paper_2603_04035_amd import datagen


def _check_lists(orc, X, idx, d2):
    n, K = idx.shape
    assert np.all((idx >= 0) & (idx < n))
    assert not np.any(idx == np.arange(n)[:, None])
    s = np.sort(idx, axis=1)
    assert not np.any(s[:, 1:] == s[:, :-1])
    # sorted by (dist, idx)
    dd = np.diff(d2, axis=1)
    assert np.all((dd > 0) | ((dd == 0) & (np.diff(idx, axis=1) > 0)))
    rec = orc.pair_d2(X, np.repeat(np.arange(n), K), idx.ravel()).reshape(n, K)
    assert np.array_equal(rec, d2)


def test_invariants_and_rank_bound(orc):
    X = datagen.gmm_isotropic(n=1200, d=10, seed=1)
    K = 12
    idx, d2, iters, upd = orc.nndescent(X, K, max_iters=6, rho=0.5, delta=0.0, seed=3)
    _check_lists(orc, X, idx, d2)
    assert iters == 6 and len(upd) == 6
    _, ed2 = orc.exact_knn(X, K)
    assert np.all(d2 >= ed2)            # approximate r-th >= exact r-th, every rank


def test_monotone_per_row(orc):
    """A longer run continues the shorter one: each sorted list only improves."""
    X = datagen.gmm_isotropic(n=800, d=8, seed=2)
    prev = None
    for t in range(0, 5):
        _, d2, iters, _ = orc.nndescent(X, 10, max_iters=t, rho=0.5, delta=0.0, seed=7)
        assert iters == t
        if prev is not None:
            assert np.all(d2 <= prev)
        prev = d2


def test_zero_iterations_is_sorted_random_init(orc):
    X = datagen.gmm_isotropic(n=300, d=5, seed=4)
    idx, d2, iters, upd = orc.nndescent(X, 8, max_iters=0, seed=5)
    assert iters == 0 and len(upd) == 0
    _check_lists(orc, X, idx, d2)
    # a random init is far from exact (recall near K/n)
    eidx, _ = orc.exact_knn(X, 8)
    assert orc.index_recall(idx, eidx, 8) < 0.2


def test_k_n_minus_one_exact_from_init(orc):
    X = datagen.gmm_isotropic(n=40, d=4, seed=6)
    idx, d2, _, upd = orc.nndescent(X, 39, max_iters=3, seed=1)
    eidx, ed2 = orc.exact_knn(X, 39)
    assert np.array_equal(idx, eidx) and np.array_equal(d2, ed2)
    assert np.all(upd == 0)            # nothing can improve an exact list


def test_seeded_init_exact_stays(orc):
    """Seeding with the exact graph: no update can ever succeed."""
    X = datagen.gmm_isotropic(n=500, d=6, seed=8)
    eidx, ed2 = orc.exact_knn(X, 10)
    idx, d2, iters, upd = orc.nndescent(X, 10, max_iters=3, delta=0.0, seed=2, init_idx=eidx)
    assert np.array_equal(idx, eidx) and np.array_equal(d2, ed2)
    assert np.all(upd == 0) and iters == 3


def test_seeded_init_completes_invalid_entries(orc):
    X = datagen.gmm_isotropic(n=200, d=4, seed=9)
    init = np.full((200, 6), -1, dtype=np.int64)
    init[:, 0] = (np.arange(200) + 1) % 200
    init[:, 1] = np.arange(200)          # self: must be dropped
    idx, d2, _, _ = orc.nndescent(X, 6, max_iters=0, init_idx=init)
    _check_lists(orc, X, idx, d2)
    assert np.all((idx == init[:, :1]).any(axis=1))


def test_early_termination_rule(orc):
    X = datagen.gmm_isotropic(n=2000, d=10, seed=3)
    K, delta = 10, 0.015
    _, _, iters, upd = orc.nndescent(X, K, max_iters=50, rho=0.5, delta=delta, seed=1)
    thr = delta * 2000 * K
    assert iters < 50
    assert upd[-1] < thr and np.all(upd[:-1] >= thr)
    assert upd[0] > upd[-1]


def test_recall_config1(orc):
    """5,000 x 50 isotropic mixture, K = 15, rho = 0.5, 8 iterations."""
    X = datagen.gmm_isotropic(n=5000, d=50, seed=0)
    idx, d2, iters, upd = orc.nndescent(X, 15, max_iters=8, rho=0.5, delta=0.015, seed=0)
    _check_lists(orc, X, idx, d2)
    eidx, ed2 = orc.exact_knn(X, 15)
    rows = np.arange(5000)
    r = orc.recall_at_k(X, rows, idx, np.sqrt(ed2[:, -1]), 15)
    assert r > 0.85, r
    assert orc.index_recall(idx, eidx, 15) <= r + 1e-12


def test_recall_clustered_full_sampling(orc):
    """Small separated clusters with rho = 1 and delta = 0 converge to exact."""
    X, _ = datagen.separated_clusters(25, 8, 3, seed=5)
    idx, d2, _, _ = orc.nndescent(X, 8, max_iters=15, rho=1.0, delta=0.0, seed=4)
    eidx, ed2 = orc.exact_knn(X, 8)
    r = orc.recall_at_k(X, np.arange(len(X)), idx, np.sqrt(ed2[:, -1]), 8)
    assert r > 0.99, r


def test_bad_args(orc):
    X = datagen.gmm_isotropic(n=10, d=3, seed=0)
    for kw in ({"K": 10}, {"K": 0}, {"K": 3, "rho": 0.0}, {"K": 3, "rho": 1.5},
               {"K": 3, "delta": -1.0}, {"K": 3, "max_iters": -1}):
        with pytest.raises(ValueError):
            orc.nndescent(X, **kw)
