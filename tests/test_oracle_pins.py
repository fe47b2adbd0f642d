"""Pins that tie the oracle's open parts to values fixed outside it (CPU only).

* NNDescent's sample and reverse steps (Dong, Charikar & Li; the paper's
  section "GPU-Native k-NN via NNDescent"): a six-point case worked out by hand
  (lists, samples, reverse unions and the update count of one iteration), and
  invariants of the traced samples on random data that a wrong step breaks
  (sampled entries left new, the old list sampled instead of taken whole, the
  reverse union dropped).
* Adam (Kingma & Ba 2015) beyond its first step: with a constant gradient the
  bias corrections make every step equal lr * g / (|g| + eps), so step t lands
  at w0 - t lr g / (|g| + eps) only if the corrections use beta^t; with a zero
  gradient then g the second step has the closed form lr * g / (1 + b1) /
  (|g| / sqrt(1 + b2) + eps), which tells the two moments apart.
* The sorted-projection order keys on integer data, where every FP32 sum and
  product is exact: the quantised codes are the exact rational floors
  (computed here with fractions) and the Z-order key is their bit interleave
  (built here from binary strings).
"""
from fractions import Fraction

import numpy as np
import pytest

from paper_2603_04035_amd import datagen


# ----------------------------------------------------------------- NNDescent

def test_nndescent_hand_worked_ring(orc):
    """Six points on a line, K = 1, rho = 1, lists seeded with a ring.

    x = [0, 5, 1, 9, 2, 20]; list(u) = {u+1 mod 6}: 0->1 (25), 1->2 (16),
    2->3 (64), 3->4 (49), 4->5 (324), 5->0 (400) in squared distance.

    Iteration 0.  Every entry is new, S = 1: new[v] = {v+1}, old[v] = {};
    the reverse new list of v is {v-1} (in-degree 1), so after the union
    new[v] = [v+1, v-1].  Points v = 0..5 join the one pair (v+1, v-1):
      v=0: (1,5) d=225: 1 keeps 2@16; 5 takes 1@225 (<400)        c=1
      v=1: (2,0) d=1:   2 takes 0@1; 0 takes 2@1                  c=3
      v=2: (3,1) d=16:  3 takes 1@16 (<49); 1 keeps 2@16 (tie, 2<3) c=4
      v=3: (4,2) d=1:   4 takes 2@1; 2 keeps 0@1 (tie, 0<4)       c=5
      v=4: (5,3) d=121: 5 takes 3@121 (<225); 3 keeps 1@16        c=6
      v=5: (0,4) d=4:   0 keeps 2@1; 4 keeps 2@1                  c=6
    Point 5 was updated twice, so c = 6 while 5 rows changed.

    Iteration 1 starts from 0:{2}, 1:{2}, 2:{0}, 3:{1}, 4:{2}, 5:{3}; every
    entry that changed is new, 1's entry (sampled in iteration 0) is old.
    Forward: new = {2},{},{0},{1},{2},{3}; old = {},{2},{},{},{},{}.
    Reverse new: 0<-{2}, 1<-{3}, 2<-{0,4} (one of the two is sampled),
    3<-{5}; reverse old: 2<-{1}.  Unions: new = {2},{3},{0}+pick,{1,5},{2},
    {3}; old = {},{2},{1},{},{},{}.
    """
    x = np.array([0, 5, 1, 9, 2, 20], dtype=np.float64).reshape(6, 1)
    init = np.array([[(u + 1) % 6] for u in range(6)], dtype=np.int64)
    idx, d2, iters, upd, tr = orc.nndescent_trace(x, 1, max_iters=2, rho=1.0, delta=0.0, seed=0,
                                                  init_idx=init, trace_iters=2)
    assert iters == 2
    sets = lambda a: [set(int(e) for e in row if e >= 0) for row in a]
    # iteration 0
    assert tr["lidx"][0].ravel().tolist() == [1, 2, 3, 4, 5, 0]
    assert np.all(tr["lflag"][0] == 1)
    assert sets(tr["newf"][0]) == [{1}, {2}, {3}, {4}, {5}, {0}]
    assert sets(tr["oldf"][0]) == [set()] * 6
    assert sets(tr["new"][0]) == [{1, 5}, {2, 0}, {3, 1}, {4, 2}, {5, 3}, {0, 4}]
    assert sets(tr["old"][0]) == [set()] * 6
    assert upd[0] == 6
    # iteration 1
    assert tr["lidx"][1].ravel().tolist() == [2, 2, 0, 1, 2, 3]
    assert tr["lflag"][1].ravel().tolist() == [1, 0, 1, 1, 1, 1]
    assert sets(tr["newf"][1]) == [{2}, set(), {0}, {1}, {2}, {3}]
    assert sets(tr["oldf"][1]) == [set(), {2}, set(), set(), set(), set()]
    new1 = sets(tr["new"][1])
    assert new1[:2] == [{2}, {3}] and new1[3:] == [{1, 5}, {2}, {3}]
    assert new1[2] in ({0}, {0, 4})
    assert sets(tr["old"][1]) == [set(), {2}, {1}, set(), set(), set()]
    # the one-iteration result: 1 keeps 2, the rest as worked out above
    idx1, d21, _, upd1 = orc.nndescent(x, 1, max_iters=1, rho=1.0, delta=0.0, seed=0, init_idx=init)
    assert idx1.ravel().tolist() == [2, 2, 0, 1, 2, 3]
    assert d21.ravel().tolist() == [1.0, 16.0, 1.0, 16.0, 1.0, 121.0]
    assert upd1.tolist() == [6]


@pytest.mark.parametrize("rho", [0.5, 1.0])
def test_nndescent_trace_invariants(orc, rho):
    """On random data, every traced iteration t and point v satisfy:
    the old list is every entry flagged old (not a sample of them); the new
    sample is min(S, #new) entries flagged new; a sampled entry still listed
    at t+1 is flagged old unless re-inserted (it cannot be: the update skips
    listed indices); the unions add only reverse entries, all of them when
    there are at most S; and the update count covers every entry that
    changed."""
    X = datagen.gmm_isotropic(n=400, d=6, seed=11)
    K, T = 8, 4
    S = int(np.ceil(rho * K))
    _, _, iters, upd, tr = orc.nndescent_trace(X, K, max_iters=T, rho=rho, delta=0.0, seed=5)
    assert iters == T
    n = X.shape[0]
    for t in range(T):
        L, F = tr["lidx"][t], tr["lflag"][t]
        newf = [set(int(e) for e in r if e >= 0) for r in tr["newf"][t]]
        oldf = [set(int(e) for e in r if e >= 0) for r in tr["oldf"][t]]
        new = [set(int(e) for e in r if e >= 0) for r in tr["new"][t]]
        old = [set(int(e) for e in r if e >= 0) for r in tr["old"][t]]
        rev_new = [set() for _ in range(n)]
        rev_old = [set() for _ in range(n)]
        for v in range(n):
            for u in newf[v]:
                rev_new[u].add(v)
            for u in oldf[v]:
                rev_old[u].add(v)
        changed = 0
        for v in range(n):
            flagged_new = {int(L[v, r]) for r in range(K) if F[v, r]}
            flagged_old = {int(L[v, r]) for r in range(K) if not F[v, r]}
            assert oldf[v] == flagged_old
            assert newf[v] <= flagged_new and len(newf[v]) == min(S, len(flagged_new))
            assert newf[v] <= new[v] and new[v] - newf[v] <= rev_new[v]
            assert oldf[v] <= old[v] and old[v] - oldf[v] <= rev_old[v]
            if len(rev_new[v]) <= S:
                assert rev_new[v] <= new[v]
            if len(rev_old[v]) <= S:
                assert rev_old[v] <= old[v]
            if t + 1 < T:
                L1, F1 = tr["lidx"][t + 1][v], tr["lflag"][t + 1][v]
                for r in range(K):
                    if int(L1[r]) in newf[v]:
                        assert F1[r] == 0
                changed += len(set(L1.tolist()) - set(L[v].tolist()))
        if t + 1 < T:
            assert upd[t] >= changed


def test_nndescent_trace_matches_untraced(orc):
    X = datagen.gmm_isotropic(n=300, d=5, seed=3)
    a = orc.nndescent(X, 6, max_iters=3, rho=0.5, delta=0.0, seed=9)
    b = orc.nndescent_trace(X, 6, max_iters=3, rho=0.5, delta=0.0, seed=9)
    for p, q in zip(a, b[:4]):
        assert np.array_equal(np.asarray(p), np.asarray(q))


# ---------------------------------------------------------------------- Adam

@pytest.mark.parametrize("lr,b1,b2", [(1e-3, 0.9, 0.999), (0.05, 0.5, 0.75)])
def test_adam_constant_gradient_steps(orc, lr, b1, b2):
    """m_t = (1 - b1^t) g and v_t = (1 - b2^t) g^2, so the corrected moments
    are g and g^2 at every step and w_t = w0 - t lr g / (|g| + eps)."""
    w0 = np.array([1.0, -2.0, 3.0, 0.25])
    g = np.array([0.5, -4.0, 1e-3, -0.125])
    w, m, v = w0.copy(), np.zeros(4), np.zeros(4)
    for t in range(1, 6):
        orc.adam_step(w, g, m, v, t=t, lr=lr, beta1=b1, beta2=b2)
        np.testing.assert_allclose(w, w0 - t * lr * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-13)
        np.testing.assert_allclose(m, (1 - b1 ** t) * g, rtol=1e-13, atol=0)
        np.testing.assert_allclose(v, (1 - b2 ** t) * g * g, rtol=1e-13, atol=0)


def test_adam_zero_then_gradient(orc):
    """Gradient 0 at t = 1, g at t = 2: m_2 = (1 - b1) g, v_2 = (1 - b2) g^2,
    the corrected moments are g / (1 + b1) and g^2 / (1 + b2), and the step is
    lr (g / (1 + b1)) / (|g| / sqrt(1 + b2) + eps).  Swapping the roles of
    the two moments changes the step (0.68955 lr instead of 0.74414 lr)."""
    lr, b1, b2 = 1e-2, 0.9, 0.999
    w0 = np.array([0.3, -0.7])
    g = np.array([2.0, -0.5])
    w, m, v = w0.copy(), np.zeros(2), np.zeros(2)
    orc.adam_step(w, np.zeros(2), m, v, t=1, lr=lr, beta1=b1, beta2=b2)
    np.testing.assert_array_equal(w, w0)
    orc.adam_step(w, g, m, v, t=2, lr=lr, beta1=b1, beta2=b2)
    step = lr * (g / (1 + b1)) / (np.abs(g) / np.sqrt(1 + b2) + 1e-8)
    np.testing.assert_allclose(w, w0 - step, rtol=0, atol=1e-15)
    np.testing.assert_allclose(np.abs(w0 - w), 0.744137 * lr, rtol=1e-5)


# ------------------------------------------------------- projection order keys

def _interleave(codes, bits):
    """Z-order key: the bit strings of the D codes, most significant level
    first, code 0 first within a level."""
    strs = [format(int(c), "0%db" % bits) for c in codes]
    return int("".join(s[l] for l in range(bits) for s in strs), 2)


@pytest.mark.parametrize("D,seed", [(2, 101), (4, 100), (8, 943)])
def test_proj_keys_exact_on_integers(orc, D, seed):
    """The seeds give every projection an odd range hi - lo, so q =
    (y - lo) 2^b / (hi - lo) is an integer only at the two endpoints; inside,
    q stays far enough from an integer that FP32 rounding cannot move its
    floor."""
    rng = np.random.default_rng(seed)
    n, m = 300, 32
    if D == 2:
        # 16-bit codes: a projection range below 64 keeps every non-integer
        # q at least 1/64 > 2^-22 q from an integer
        Z = rng.integers(-3, 4, size=(n, m)).astype(np.float32)
        dirs = np.zeros((D, m), np.float32)
        for j in range(D):
            sel = rng.choice(m, 8, replace=False)
            dirs[j, sel] = rng.choice([-1.0, 1.0], 8)
    else:
        Z = rng.integers(-9, 10, size=(n, m)).astype(np.float32)
        dirs = rng.integers(-3, 4, size=(D, m)).astype(np.float32)
    bits = 32 // D
    Zi = Z.astype(np.int64)
    Y = Zi @ dirs.astype(np.int64).T          # exact projections (|y| < 2^24)
    assert np.abs(Y).max() < 2 ** 24
    assert np.all((Y.max(0) - Y.min(0)) % 2 == 1)
    expect = np.empty(n, dtype=np.uint64)
    codes = np.empty((n, D), dtype=np.int64)
    for j in range(D):
        lo, hi = int(Y[:, j].min()), int(Y[:, j].max())
        for i in range(n):
            q = Fraction(int(Y[i, j]) - lo, 1) * (2 ** bits) / (hi - lo)
            # the FP32 product (two roundings, 2^-24 each) is within 2^-23
            # relative of q: the data stay 2^-22 q away from integer
            # boundaries other than the exact endpoints
            frac = q - (q.numerator // q.denominator)
            if Y[i, j] in (lo, hi):
                assert frac == 0
            else:
                assert 2 ** 22 * frac > q and 2 ** 22 * (1 - frac) > q, (i, j, q)
            codes[i, j] = min(q.numerator // q.denominator, 2 ** bits - 1)
    for i in range(n):
        expect[i] = _interleave(codes[i], bits)
    got = orc.proj_keys(Z, dirs, D=D)
    np.testing.assert_array_equal(got.astype(np.uint64), expect)


def test_proj_keys_single_direction_orders_by_projection(orc):
    """D = 1: the key orders points exactly as their (exact integer)
    projections, both zeros alike, negatives below positives."""
    rng = np.random.default_rng(7)
    Z = rng.integers(-20, 21, size=(500, 32)).astype(np.float32)
    r = rng.integers(-2, 3, size=(1, 32)).astype(np.float32)
    y = Z.astype(np.int64) @ r.astype(np.int64).ravel()
    keys = orc.proj_keys(Z, r, D=1).astype(np.int64)
    for a in range(0, 500, 7):
        for b in range(0, 500, 11):
            assert (keys[a] < keys[b]) == (y[a] < y[b])
            assert (keys[a] == keys[b]) == (y[a] == y[b])
