"""The fuzzy graph on the GPU (UMAP membership strengths and their union)
against the oracle, both fed the same k-NN graph (the GPU exact path's).

Bars: rho equal (it is one of the given FP32 distances); sigma within one
FP32 rounding of the oracle's double root (rel 2^-23); weights within two
FP32 roundings (rel 2^-22); the CSR pattern (row_ptr, col) identical; the
union values within 1e-6 absolute (the GPU folds FP32-rounded weights in
double).  Cases: a ragged 3,001-row mixture, rows that hit the no-root limit
(duplicates, lattice ties), k = 1 and 32, rows listed by hundreds of others
(a hand-built graph), the 1,000,000-row graph on sampled rows, and graphs
with a self entry or a repeated entry (rejected).
"""
import numpy as np
import pytest
import torch

from paper_2603_04035_amd import datagen

pytestmark = pytest.mark.gpu


def _check(orc, G, D, rows=None):
    import paper_2603_04035_amd as knn
    rho, sig, w, rp, col, val = knn.fuzzy_graph(G, D)
    Gn, Dn = G.cpu().numpy(), D.cpu().numpy()
    n, k = Gn.shape
    rows = np.arange(n) if rows is None else rows
    orho, osig, ow = orc.fuzzy_rows(Dn[rows])
    rho, sig, w = rho.cpu().numpy()[rows], sig.cpu().numpy()[rows], w.cpu().numpy()[rows]
    assert np.array_equal(rho.astype(np.float64), orho)
    assert np.all(np.abs(sig - osig) <= 2.0 ** -23 * osig), np.max(np.abs(sig - osig) / np.maximum(osig, 1e-30))
    assert np.all(np.abs(w - ow) <= 2.0 ** -22 * ow + 1e-37), np.max(np.abs(w - ow))
    # union rows from the oracle's own weights: a sampled row needs its own
    # and those of the rows that list it
    need = np.isin(np.arange(n), rows) | np.isin(Gn, rows).any(axis=1)
    ow_all = np.full((n, k), np.nan)
    ow_all[need] = orc.fuzzy_rows(Dn[need])[2]
    urows = orc.fuzzy_union(Gn, ow_all, rows=rows)
    rp, col, val = rp.cpu().numpy(), col.cpu().numpy(), val.cpu().numpy()
    assert rp[0] == 0 and rp[-1] == len(col) and np.all(np.diff(rp) >= 1)
    for i, ur in zip(rows, urows):
        c = col[rp[i]:rp[i + 1]]
        v = val[rp[i]:rp[i + 1]]
        assert c.tolist() == [j for j, _ in ur], i
        np.testing.assert_allclose(v, [x for _, x in ur], rtol=0, atol=1e-6)
    return sig


def test_fuzzy_mixture_ragged(orc):
    import paper_2603_04035_amd as knn
    X = torch.from_numpy(datagen.gmm_isotropic(n=3001, d=50, seed=7)).cuda()
    G, D = knn.knn_exact(X, 15)
    sig = _check(orc, G, D)
    assert np.all(sig > 0)


def test_fuzzy_degenerate_rows(orc):
    """Four copies of each point: the three zero distances reach log2(15)
    only with a tie at rho; lattice points have shells of equal distance."""
    import paper_2603_04035_amd as knn
    X = torch.from_numpy(datagen.with_duplicates(500, 6, 5, seed=2)).cuda()
    G, D = knn.knn_exact(X, 15)
    sig = _check(orc, G, D)
    assert np.any(sig == 0)
    L = torch.from_numpy(datagen.lattice(12, 2, seed=1)).cuda()
    G, D = knn.knn_exact(L, 15)
    sig = _check(orc, G, D)
    assert np.any(sig == 0)


@pytest.mark.parametrize("k", [1, 2, 3, 32])
def test_fuzzy_k_extremes(orc, k):
    import paper_2603_04035_amd as knn
    X = torch.from_numpy(datagen.gmm_anisotropic(n=2000, d=20, comps=5, seed=3)).cuda()
    G, D = knn.knn_exact(X, k)
    _check(orc, G, D)


def test_fuzzy_hub_rows(orc):
    """Rows listed by hundreds of others (a transposed segment of several
    64-entry chunks), some of them listing those rows back: a hand-built
    graph of 700 rows, k = 6, where every row lists rows 0, 1 and 2 and
    three rows chosen at random (distinct, not itself, seed 11)."""
    n, k = 700, 6
    rng = np.random.default_rng(11)
    G = np.empty((n, k), dtype=np.int32)
    for i in range(n):
        hubs = [h for h in (0, 1, 2) if h != i]
        rest = rng.choice([j for j in range(3, n) if j != i], size=k - len(hubs), replace=False)
        G[i] = np.concatenate([hubs, rest])
    D = np.sort(rng.uniform(0.5, 2.0, size=(n, k)).astype(np.float32), axis=1)
    _check(orc, torch.from_numpy(G).cuda(), torch.from_numpy(D).cuda())


def test_fuzzy_1m_sampled(orc):
    import bench
    import paper_2603_04035_amd as knn
    X = torch.from_numpy(bench.make_data("gmm1m")).cuda()
    G, D = knn.knn_exact(X, 15)
    rows = datagen.sample_queries(X.shape[0], 200, seed=9)
    _check(orc, G, D, rows=rows)


def test_fuzzy_rejects_self_entry():
    import paper_2603_04035_amd as knn
    X = torch.from_numpy(datagen.gmm_isotropic(n=500, d=8, seed=1)).cuda()
    G, D = knn.knn_exact(X, 5)
    G[17, 2] = 17
    with pytest.raises(knn.KnnError) as e:
        knn.fuzzy_graph(G, D)
    assert e.value.status == -1
    G[17, 2] = G[17, 4]                                     # a column twice in one row
    with pytest.raises(knn.KnnError) as e:
        knn.fuzzy_graph(G, D)
    assert e.value.status == -1 and "twice" in str(e.value)
