"""Pins for the oracle's embedding-quality metrics (CPU only): k-NN
preservation, trustworthiness and continuity as the paper's section
"Embedding Quality" uses them (Venna & Kaski 2006).

* a six-point case counted by hand (every rank written out below);
* an embedding that preserves every rank (the identity, or any similarity
  transform) scores 1.0 on all three;
* swapping the roles of the two spaces swaps trustworthiness and
  continuity;
* ranking by the canonical FP32 distance gives the FP64 result where no two
  distances from a point are within FP32 error of each other;
* on lattices full of ties, the trust and continuity sums over L \ N (and
  N \ L) equal the sums of (rank - k)+ over all of L (and N), from
  brute-force ranks, and both equal the oracle's terms.
"""
import numpy as np
import pytest

from paper_2603_04035_amd import datagen


def test_hand_counted_six_points(orc):
    """X on a line at 0, 1, 3, 6, 10, 15; Y swaps points 0 and 5
    (15, 1, 3, 6, 10, 0); k = 1, so 2/(n k (2n - 3k - 1)) = 1/24.
    Nearest in X: 0->1, 1->0, 2->1, 3->2, 4->3, 5->4; in Y: 0->4, 1->5,
    2->1, 3->2, 4->3, 5->1.  Hits: rows 2, 3, 4, so P = 3/6.
    Trust: 0 lists 4 in Y, whose X-rank from 0 is 4 (distances 1, 3, 6, 10,
    15): +3; 1 lists 5, X-rank 5 from 1: +4; 5 lists 1, X-rank 4 from 5
    (distances 5, 9, 12, 14, 15): +3; T = 1 - 10/24.
    Cont: 0 lists 1 in X, Y-rank 4 from 0 (distances 5, 9, 12, 14, 15): +3;
    1 lists 0, Y-rank 5 from 1: +4; 5 lists 4, Y-rank 4 from 5 (1, 3, 6, 10,
    15): +3; C = 1 - 10/24."""
    X = np.array([0, 1, 3, 6, 10, 15], dtype=np.float64).reshape(6, 1)
    Y = np.array([15, 1, 3, 6, 10, 0], dtype=np.float64).reshape(6, 1)
    h, t, c = orc.quality_rows(X, Y, 1)
    assert h.tolist() == [0, 0, 1, 1, 1, 0]
    assert t.tolist() == [3, 4, 0, 0, 0, 3]
    assert c.tolist() == [3, 4, 0, 0, 0, 3]
    p, T, C = orc.quality(X, Y, 1)
    assert p == 0.5 and T == pytest.approx(1 - 10 / 24, abs=1e-15) and C == pytest.approx(1 - 10 / 24, abs=1e-15)


def test_rank_preserving_embeddings_score_one(orc):
    X = datagen.gmm_isotropic(n=400, d=12, seed=3)
    for Y in (X, 3.0 * X + 7.0, X @ np.linalg.qr(np.random.default_rng(1).normal(size=(12, 12)))[0]):
        for k in (1, 5, 15):
            assert orc.quality(X, Y, k) == (1.0, 1.0, 1.0)


def test_swapping_spaces_swaps_trust_and_continuity(orc):
    X = datagen.gmm_isotropic(n=300, d=8, seed=4)
    Y = np.random.default_rng(2).normal(size=(300, 2)) + X[:, :2]
    p1, t1, c1 = orc.quality(X, Y, 10)
    p2, t2, c2 = orc.quality(Y, X, 10)
    assert p1 == p2 and t1 == c2 and c1 == t2
    assert 0.0 < t1 < 1.0 and 0.0 < c1 < 1.0


def test_ties_break_by_index(orc):
    """Lattice: equal distances are ranked by index, so a point's 4 unit
    neighbours take ranks 1-4 in index order and k = 2 keeps the two lowest."""
    X = datagen.lattice(5, 2)          # index = 5 x + y
    Y = X.copy()
    Y[12] += 0.25                      # move the centre point slightly in the embedding only
    h, _, _ = orc.quality_rows(X, Y, 2, rows=[12])
    # centre 12 = (2, 2): unit neighbours 7, 11, 13, 17 -> N = {7, 11};
    # shifted to (2.25, 2.25): nearest are 13 (0.79) and 17 (0.79) -> L = {13, 17}
    assert h.tolist() == [0]


def test_canonical_fp32_equals_fp64_without_near_ties(orc):
    X = datagen.gmm_anisotropic(n=500, d=30, comps=5, seed=6)
    Y = datagen.gmm_isotropic(n=500, d=2, seed=7)
    for k in (5, 15):
        a = orc.quality_rows(X, Y, k)
        b = orc.quality_rows(X, Y, k, canonical=True)
        for u, v in zip(a, b):
            assert np.array_equal(u, v)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_trust_sum_over_all_of_l(orc, seed):
    """The identity the GPU's single X-space pass relies on: with ranks that
    break ties by index, the members of N(i) are exactly the rows of rank
    <= k, so sum over L(i) \\ N(i) of (r(i,j) - k) equals the sum over all of
    L(i) of max(r(i,j) - k, 0) (likewise for continuity).  Ranks here are
    brute force in FP64 with lexicographic (distance, index) order, on
    inputs with repeated points so that ties occur; both sums are checked
    against the oracle's per-row terms."""
    rng = np.random.default_rng(seed)
    n, k = 40, 4
    X = rng.integers(0, 4, size=(n, 3)).astype(np.float64)    # a small lattice: many equal distances
    Y = rng.integers(0, 5, size=(n, 2)).astype(np.float64)

    def ranks(Z):
        d = ((Z[:, None, :] - Z[None, :, :]) ** 2).sum(-1)
        r = np.zeros((n, n), dtype=np.int64)
        for i in range(n):
            order = sorted((j for j in range(n) if j != i), key=lambda j: (d[i, j], j))
            for pos, j in enumerate(order):
                r[i, j] = pos + 1
        return r

    rx, ry = ranks(X), ranks(Y)
    N = [set(np.nonzero((rx[i] >= 1) & (rx[i] <= k))[0]) for i in range(n)]
    L = [set(np.nonzero((ry[i] >= 1) & (ry[i] <= k))[0]) for i in range(n)]
    for i in range(n):
        assert len(N[i]) == k and len(L[i]) == k
    t_def = np.array([sum(rx[i, j] - k for j in L[i] - N[i]) for i in range(n)])
    t_all = np.array([sum(max(rx[i, j] - k, 0) for j in L[i]) for i in range(n)])
    c_def = np.array([sum(ry[i, j] - k for j in N[i] - L[i]) for i in range(n)])
    c_all = np.array([sum(max(ry[i, j] - k, 0) for j in N[i]) for i in range(n)])
    assert np.array_equal(t_def, t_all) and np.array_equal(c_def, c_all)
    h, t, c = orc.quality_rows(X, Y, k)
    assert np.array_equal(t, t_def) and np.array_equal(c, c_def)
    assert np.array_equal(h, np.array([len(N[i] & L[i]) for i in range(n)]))
