"""Pins for the oracle's exact kNN (CPU only).

The oracle is checked against things other than itself: exact integer
arithmetic on tiny inputs, scikit-learn / SciPy brute force and k-d tree,
closed forms (a sorted line, integer lattices, duplicates, separated
clusters, k = n - 1) and invariants (symmetry, sortedness, triangle
inequality, translation and permutation behaviour).
"""
import itertools

import numpy as np
import pytest

from paper_2603_04035_amd import datagen


def _brute_int(P, k):
    """Exhaustive reference on integer points: exact integer D, full sort by (D, j)."""
    n = len(P)
    out = []
    for i in range(n):
        ds = []
        for j in range(n):
            if j == i:
                continue
            ds.append((sum((int(a) - int(b)) ** 2 for a, b in zip(P[i], P[j])), j))
        ds.sort()
        out.append(ds[:k])
    return out


@pytest.mark.parametrize("n", [2, 3, 5, 8, 12])
@pytest.mark.parametrize("d", [1, 2, 3])
def test_tiny_exhaustive_integer(orc, n, d):
    rng = np.random.default_rng(100 * n + d)
    P = rng.integers(0, 4, size=(n, d))          # small range: many exact ties
    for k in range(1, n):
        idx, d2 = orc.exact_knn(P.astype(np.float64), k)
        ref = _brute_int(P, k)
        for i in range(n):
            assert [j for _, j in ref[i]] == list(idx[i]), (n, d, k, i)
            assert [float(D) for D, _ in ref[i]] == list(d2[i])


def test_vs_sklearn_and_ckdtree(orc):
    from scipy.spatial import cKDTree
    from sklearn.neighbors import NearestNeighbors
    X = datagen.gmm_isotropic(n=2000, d=20, seed=3)
    k = 15
    idx, d2 = orc.exact_knn(X, k)
    X64 = X.astype(np.float64)
    nn = NearestNeighbors(n_neighbors=k + 1, algorithm="brute").fit(X64)
    sd, si = nn.kneighbors(X64)
    # drop self (the first column, distance 0; no duplicates in this data)
    assert np.all(si[:, 0] == np.arange(len(X)))
    np.testing.assert_allclose(np.sqrt(d2), sd[:, 1:], rtol=1e-10, atol=0)
    tree = cKDTree(X64)
    td, ti = tree.query(X64, k=k + 1)
    np.testing.assert_allclose(np.sqrt(d2), td[:, 1:], rtol=1e-10, atol=0)
    # indices must agree wherever neighbouring distances are separated
    dist = np.sqrt(d2)
    sep = np.ones_like(dist, dtype=bool)
    gap = np.diff(dist, axis=1) > 1e-9 * dist[:, 1:]
    sep[:, 1:] &= gap
    sep[:, :-1] &= gap
    assert np.array_equal(idx[sep], ti[:, 1:][sep])
    assert sep.mean() > 0.99


def test_line_window_closed_form(orc):
    """On a line the k nearest neighbours of a point form a window around it."""
    X = datagen.line_1d(300, seed=5)
    pos = X[:, 0].astype(np.float64)
    order = np.argsort(pos, kind="stable")
    rank = np.empty_like(order)
    rank[order] = np.arange(len(order))
    for k in (1, 4, 15, 60):
        idx, _ = orc.exact_knn(X, k)
        for i in range(len(X)):
            lo, hi = rank[i] - 1, rank[i] + 1
            exp = []
            while len(exp) < k:     # two-pointer merge outwards
                dl = pos[i] - pos[order[lo]] if lo >= 0 else np.inf
                dr = pos[order[hi]] - pos[i] if hi < len(X) else np.inf
                if dl <= dr:
                    exp.append(order[lo]); lo -= 1
                else:
                    exp.append(order[hi]); hi += 1
            assert list(idx[i]) == exp, (k, i)


def test_lattice_shells_and_tie_break(orc):
    """Z^2 grid: shells 1 (4 pts), sqrt2 (4), 2 (4), sqrt5 (8); ties by index."""
    side = 9
    X = datagen.lattice(side, 2, seed=11)
    idx, d2 = orc.exact_knn(X, 20)
    P = X.astype(np.int64)
    for i in range(len(X)):
        x, y = P[i]
        if not (2 <= x <= side - 3 and 2 <= y <= side - 3):
            continue                       # interior points have full shells
        assert list(d2[i]) == [1.0] * 4 + [2.0] * 4 + [4.0] * 4 + [5.0] * 8
        for a, b in ((0, 4), (4, 8), (8, 12), (12, 20)):
            shell = idx[i, a:b]
            assert list(shell) == sorted(shell)     # equal distances: ascending index
        exp1 = {(x + 1, y), (x - 1, y), (x, y + 1), (x, y - 1)}
        got1 = {tuple(P[j]) for j in idx[i, :4]}
        assert got1 == exp1
    X3 = datagen.lattice(5, 3, seed=12)
    idx3, d23 = orc.exact_knn(X3, 18)
    P3 = X3.astype(np.int64)
    for i in range(len(X3)):
        if np.all((P3[i] >= 1) & (P3[i] <= 3)):
            assert list(d23[i]) == [1.0] * 6 + [2.0] * 12


def test_duplicates_first_in_index_order(orc):
    copies = 4
    X = datagen.with_duplicates(50, 6, copies, seed=2)
    idx, d2 = orc.exact_knn(X, 6)
    for i in range(len(X)):
        twins = [j for j in range(len(X)) if j != i and np.array_equal(X[j], X[i])]
        assert len(twins) == copies - 1
        assert list(idx[i, :copies - 1]) == sorted(twins)
        assert np.all(d2[i, :copies - 1] == 0.0) and d2[i, copies - 1] > 0.0


def test_separated_clusters_stay_inside(orc):
    X, lab = datagen.separated_clusters(40, 5, 8, seed=4)
    idx, _ = orc.exact_knn(X, 39)
    assert np.all(lab[idx] == lab[:, None])


def test_k_equals_n_minus_one_is_permutation(orc):
    X = datagen.gmm_isotropic(n=37, d=5, seed=9)
    idx, d2 = orc.exact_knn(X, 36)
    for i in range(37):
        assert sorted(idx[i]) == [j for j in range(37) if j != i]
        assert np.all(np.diff(d2[i]) >= 0)


def test_invariants(orc):
    X = datagen.gmm_isotropic(n=600, d=12, seed=8)
    k = 10
    idx, d2 = orc.exact_knn(X, k)
    n = len(X)
    assert not np.any(idx == np.arange(n)[:, None])
    assert np.all(np.diff(d2, axis=1) >= 0)
    # stored distance equals the pair distance, and the pair distance is symmetric bitwise
    a = np.repeat(np.arange(n), k)
    b = idx.ravel()
    assert np.array_equal(orc.pair_d2(X, a, b), d2.ravel())
    assert np.array_equal(orc.pair_d2(X, b, a), d2.ravel())
    # triangle inequality through the first neighbour
    j = idx[:, 0]
    dij = np.sqrt(d2[:, 0])
    for r in range(k):
        dik = np.sqrt(d2[:, r])
        djk = np.sqrt(orc.pair_d2(X, j, idx[:, r]))
        assert np.all(dik <= dij + djk + 1e-12)
    # no non-neighbour is closer than the k-th neighbour (sampled columns)
    rng = np.random.default_rng(0)
    cols = rng.integers(0, n, size=(n, 30))
    dc = orc.pair_d2(X, np.repeat(np.arange(n), 30), cols.ravel()).reshape(n, 30)
    outside = ~(cols[:, :, None] == idx[:, None, :]).any(-1) & (cols != np.arange(n)[:, None])
    assert np.all(dc[outside] >= np.broadcast_to(d2[:, -1:], dc.shape)[outside])


def test_translation_exact_on_integer_data(orc):
    rng = np.random.default_rng(1)
    P = rng.integers(-20, 20, size=(200, 4)).astype(np.float64)
    i1, d1 = orc.exact_knn(P, 12)
    i2, d2 = orc.exact_knn(P + 1000.0, 12)
    assert np.array_equal(i1, i2) and np.array_equal(d1, d2)


def test_permutation_equivariance(orc):
    X = datagen.gmm_isotropic(n=300, d=7, seed=6)
    perm = np.random.default_rng(3).permutation(300)
    i1, d1 = orc.exact_knn(X, 9)
    i2, d2 = orc.exact_knn(X[perm], 9)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(300)
    # row r of the permuted problem is original row perm[r]; map its neighbours back
    assert np.array_equal(perm[i2], i1[perm])
    assert np.array_equal(d2, d1[perm])


def test_query_form_and_bad_args(orc):
    R = datagen.gmm_isotropic(n=100, d=3, seed=1)
    Q = datagen.gmm_isotropic(n=10, d=3, seed=2)
    idx, d2 = orc.exact_query(R, Q, 5)
    full = ((Q[:, None, :].astype(np.float64) - R[None].astype(np.float64)) ** 2).sum(-1)
    for i in range(10):
        order = sorted(range(100), key=lambda j: (full[i, j], j))[:5]
        assert list(idx[i]) == order
    with pytest.raises(ValueError):
        orc.exact_knn(R, 100)         # k > n - 1
    with pytest.raises(ValueError):
        orc.exact_knn(R, 0)


def test_comparator_rules(orc):
    """Hand-built rows: swaps inside a near-tie group pass, outside fail."""
    from oracle.compare import exact_parity, parity_ok
    X = np.array([[0.0], [1.0], [1.0 + 1e-7], [2.0], [3.0]])
    rows = np.array([0])
    O = np.array([[1, 2, 3]])
    od = np.array([[1.0, 1.0 + 1e-7, 2.0]])
    assert parity_ok(exact_parity(X, rows, O, od, O))
    swapped = np.array([[2, 1, 3]])
    sd = np.array([[1.0 + 1e-7, 1.0, 2.0]])
    r = exact_parity(X, rows, swapped, sd, O)
    assert parity_ok(r) and r["tie_swaps"] == 2
    bad = np.array([[1, 3, 2]])
    bd = np.array([[1.0, 2.0, 1.0 + 1e-7]])
    assert not parity_ok(exact_parity(X, rows, bad, bd, O))
    # boundary: index 4 instead of 3 at rank k is not a tie
    bnd = np.array([[1, 2, 4]])
    assert not parity_ok(exact_parity(X, rows, bnd, np.array([[1.0, 1.0 + 1e-7, 3.0]]), O))
    # a distance off by 1e-4 relative fails
    assert not parity_ok(exact_parity(X, rows, O, od * (1 + 1e-4), O))
    # self and duplicates fail
    assert not parity_ok(exact_parity(X, rows, np.array([[0, 2, 3]]), od, O))
    assert not parity_ok(exact_parity(X, rows, np.array([[1, 1, 3]]), od, O))
