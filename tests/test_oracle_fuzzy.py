"""Pins for the oracle's UMAP membership strengths and fuzzy union (CPU only).

The UMAP definition (McInnes, Healy & Melville 2018) fixes sigma_i only
implicitly, through sum_r exp(-max(0, d_r - rho_i) / sigma_i) = log2(k); the
pins are cases where that equation has a closed form, its defining
identities, and hand-worked unions.
"""
import math

import numpy as np
import pytest


@pytest.mark.parametrize("rho,c", [(1.0, 1.0), (0.25, 3.0), (7.5, 0.01)])
def test_k3_quadratic_closed_form(orc, rho, c):
    """k = 3, distances (rho, rho + c, rho + 2c): with y = exp(-c / sigma)
    the equation is 1 + y + y^2 = log2 3, so y is the positive root of a
    quadratic and sigma = -c / ln y."""
    r, s, w = orc.fuzzy_rows(np.array([[rho, rho + c, rho + 2 * c]]))
    t = math.log2(3.0) - 1.0
    y = (-1.0 + math.sqrt(1.0 + 4.0 * t)) / 2.0
    assert r[0] == rho
    assert s[0] == pytest.approx(-c / math.log(y), rel=1e-13)
    np.testing.assert_allclose(w[0], [1.0, y, y * y], rtol=1e-13)


@pytest.mark.parametrize("k", [4, 15, 30])
def test_equal_far_neighbours_closed_form(orc, k):
    """Nearest at rho, the other k - 1 at rho + c: 1 + (k - 1) exp(-c/sigma)
    = log2 k gives sigma = c / ln((k - 1) / (log2 k - 1))."""
    rho, c = 2.0, 0.5
    d = np.array([[rho] + [rho + c] * (k - 1)])
    _, s, w = orc.fuzzy_rows(d)
    exp_s = c / math.log((k - 1) / (math.log2(k) - 1.0))
    assert s[0] == pytest.approx(exp_s, rel=1e-13)
    assert w[0, 0] == 1.0
    np.testing.assert_allclose(w[0, 1:], (math.log2(k) - 1.0) / (k - 1), rtol=1e-13)


def test_identities_on_random_rows(orc):
    """Every solvable row: weights sum to log2 k, the nearest positive
    distance has weight 1, weights fall with distance and lie in (0, 1];
    scaling all distances by s scales rho and sigma by s and keeps w."""
    rng = np.random.default_rng(3)
    k = 15
    d = np.sort(rng.gamma(2.0, 1.0, size=(500, k)), axis=1)
    rho, s, w = orc.fuzzy_rows(d)
    assert np.all(s > 0)
    np.testing.assert_allclose(w.sum(axis=1), math.log2(k), rtol=1e-12)
    np.testing.assert_array_equal(rho, d[:, 0])
    np.testing.assert_array_equal(w[:, 0], 1.0)
    assert np.all(np.diff(w, axis=1) <= 0) and np.all((w > 0) & (w <= 1))
    rho2, s2, w2 = orc.fuzzy_rows(d * 8.0)
    np.testing.assert_allclose(rho2, 8 * rho, rtol=1e-15)
    np.testing.assert_allclose(s2, 8 * s, rtol=1e-12)
    np.testing.assert_allclose(w2, w, rtol=1e-12, atol=1e-15)


def test_duplicates_and_degenerate_rows(orc):
    """Zero distances (duplicates) sit at or below rho, the smallest positive
    distance, so they get weight 1; rows whose count of distances <= rho
    reaches log2 k have no root and take the sigma -> 0 limit."""
    k = 8                                   # log2 k = 3
    d = np.array([[0.0, 0.0, 1.0, 2.0, 3.0, 4.0, 5.0, 6.0],     # c = 3 -> degenerate
                  [0.0, 1.0, 2.0, 3.0, 4.0, 5.0, 6.0, 7.0],     # c = 2 -> solvable
                  [3.0] * 8,                                   # all tied
                  [0.0] * 8])                                  # all duplicates
    rho, s, w = orc.fuzzy_rows(d)
    np.testing.assert_array_equal(rho, [1.0, 1.0, 3.0, 0.0])
    assert s[0] == 0 and s[2] == 0 and s[3] == 0 and s[1] > 0
    np.testing.assert_array_equal(w[0], [1, 1, 1, 0, 0, 0, 0, 0])
    np.testing.assert_array_equal(w[2], 1.0)
    np.testing.assert_array_equal(w[3], 1.0)
    assert w[1, 0] == 1.0 and w[1, 1] == 1.0 and w[1].sum() == pytest.approx(3.0, rel=1e-12)


def test_union_hand_worked(orc):
    """Four points, k = 2.  Lists: 0 -> (1, 2), 1 -> (0, 3), 2 -> (0, 1),
    3 -> (1, 2) with weights a..h.  W = A + A^T - A o A^T:
    (0,1): a + c - ac (mutual), (0,2): b + e - be (mutual), (1,2): f only,
    (1,3): d + g - dg (mutual), (2,3): h only; symmetric entries equal."""
    idx = np.array([[1, 2], [0, 3], [0, 1], [1, 2]])
    a, b, c, d, e, f, g, h = 0.9, 0.5, 0.8, 0.3, 0.7, 0.2, 0.6, 0.4
    w = np.array([[a, b], [c, d], [e, f], [g, h]])
    rows = orc.fuzzy_union(idx, w)
    u = lambda x, y: x + y - x * y
    assert rows[0] == [(1, pytest.approx(u(a, c))), (2, pytest.approx(u(b, e)))]
    assert rows[1] == [(0, pytest.approx(u(a, c))), (2, pytest.approx(f)), (3, pytest.approx(u(d, g)))]
    assert rows[2] == [(0, pytest.approx(u(b, e))), (1, pytest.approx(f)), (3, pytest.approx(h))]
    assert rows[3] == [(1, pytest.approx(u(d, g))), (2, pytest.approx(h))]


def test_union_symmetric_on_random_graph(orc):
    rng = np.random.default_rng(5)
    n, k = 60, 5
    idx = np.array([rng.choice([j for j in range(n) if j != i], k, replace=False) for i in range(n)])
    w = rng.random((n, k))
    rows = orc.fuzzy_union(idx, w)
    M = {}
    for i, row in enumerate(rows):
        cols = [j for j, _ in row]
        assert cols == sorted(cols) and len(set(cols)) == len(cols) and i not in cols
        for j, v in row:
            M[(i, j)] = v
    for (i, j), v in M.items():
        assert M[(j, i)] == v
    # the pattern is the union of the lists and their transpose
    pat = {(i, int(j)) for i in range(n) for j in idx[i]}
    assert set(M) == pat | {(j, i) for (i, j) in pat}
