"""Pins for the oracle's rounding, encoder (MLP) and projection seeding (CPU only).

* BF16 rounding: against torch's CPU float32 -> bfloat16 cast (a library
  routine) and hand-checked halfway cases.
* MLP: analytic gradients against fp64 central finite differences; the
  triplet loss on a hand-built case; Adam's first step closed form.
* Seeding: with d = 1, the identity encoder, one projection and w >= k, the
  seed lists equal the exact kNN (window property of sorted lines).
"""
import numpy as np
import pytest
import torch

from paper_2603_04035_amd import datagen


def test_bf16_matches_torch_cast(orc):
    rng = np.random.default_rng(0)
    a = np.concatenate([rng.normal(size=20000).astype(np.float32) * 10.0 ** rng.integers(-30, 30, 20000),
                        np.array([0.0, -0.0, np.inf, -np.inf, 3.3895314e38, 1e-40, -1e-45],
                                 dtype=np.float32)]).astype(np.float32)
    ours = orc.round_bf16(a)
    ref = torch.from_numpy(a).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(ours, ref)


def test_bf16_ties_to_even(orc):
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties to the even mantissa (1.0)
    one_half_ulp = np.float32(1.0 + 2.0 ** -8)
    one_3half = np.float32(1.0 + 3 * 2.0 ** -8)
    bits = orc.round_bf16(np.array([one_half_ulp, one_3half], dtype=np.float32))
    assert bits[0] == 0x3F80                      # 1.0
    assert bits[1] == 0x3F82                      # 1 + 2^-6 (even)
    nan = orc.round_bf16(np.array([np.nan], dtype=np.float32))
    assert np.isnan(orc.bf16_to_f64(nan))[0]


def _mlp_params(d, seed=0):
    rng = np.random.default_rng(seed)
    W1 = rng.normal(0, np.sqrt(2.0 / d), size=(d, 64))
    b1 = rng.normal(0, 0.1, size=64)
    W2 = rng.normal(0, np.sqrt(2.0 / 64), size=(64, 32))
    b2 = rng.normal(0, 0.1, size=32)
    return W1, b1, W2, b2


def _loss(orc, X, params, B, margin):
    Z = orc.mlp_forward(X, *params)
    return orc.triplet_loss(Z, B, margin, want_grad=False)


def test_mlp_gradients_vs_finite_differences(orc):
    d, B, margin = 7, 6, 1.0
    rng = np.random.default_rng(1)
    X = rng.normal(size=(3 * B, d))
    params = list(_mlp_params(d, seed=2))
    Z, H = orc.mlp_forward(X, *params, want_hidden=True)
    loss, dZ = orc.triplet_loss(Z, B, margin)
    grads = orc.mlp_backward(X, params[0], params[1], params[2], dZ)
    # kinks: skip if any pre-activation or hinge sits within 1e-6 of 0
    pre = X @ params[0] + params[1]
    assert np.min(np.abs(pre)) > 1e-6
    h = 1e-6
    for p, g in zip(params, grads):
        flat = p.reshape(-1)
        num = np.empty(flat.size)
        for e in range(flat.size):
            old = flat[e]
            flat[e] = old + h
            lp = _loss(orc, X, params, B, margin)
            flat[e] = old - h
            lm = _loss(orc, X, params, B, margin)
            flat[e] = old
            num[e] = (lp - lm) / (2 * h)
        if np.linalg.norm(g) < 1e-12:       # b2: zero up to rounding (see below); FD is noise
            assert np.abs(num).max() < 1e-8
            continue
        err = np.linalg.norm(num - g.reshape(-1)) / np.linalg.norm(num)
        assert err < 1e-6, err
    assert loss > 0
    # the triplet loss is translation invariant in z: the b2 gradient vanishes
    assert np.abs(grads[3]).max() < 1e-14 and np.linalg.norm(grads[0]) > 1e-2


def test_triplet_loss_hand_case(orc):
    # B = 2, width 2: anchors, positives, negatives stacked
    Z = np.array([[0.0, 0.0], [1.0, 1.0],      # anchors
                  [1.0, 0.0], [1.0, 1.0],      # positives: dp = 1, 0
                  [0.0, 2.0], [5.0, 5.0]])     # negatives: dn = 4, 32
    loss, dZ = orc.triplet_loss(Z, 2, margin=4.0)
    # triplet 0: 4 + 1 - 4 = 1 > 0; triplet 1: 4 + 0 - 32 < 0
    assert loss == pytest.approx(0.5)
    # d/dza = (2/B)(zn - zp) = (0-1, 2-0) ; d/dzp = (2/B)(zp - za) ; d/dzn = (2/B)(za - zn)
    np.testing.assert_allclose(dZ[0], [-1.0, 2.0])
    np.testing.assert_allclose(dZ[2], [1.0, 0.0])
    np.testing.assert_allclose(dZ[4], [0.0, -2.0])
    assert np.all(dZ[[1, 3, 5]] == 0)


def test_adam_first_step_closed_form(orc):
    w = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -4.0, 0.0])
    m = np.zeros(3)
    v = np.zeros(3)
    orc.adam_step(w, g, m, v, t=1, lr=0.01)
    # bias-corrected first step: w -= lr * g / (|g| + eps)
    exp = np.array([1.0, -2.0, 3.0]) - 0.01 * g / (np.abs(g) + 1e-8)
    np.testing.assert_allclose(w, exp, rtol=0, atol=1e-15)


def test_adam_training_reduces_loss(orc):
    """Clusters in 6-d: triplets from the same / another cluster; loss falls."""
    X, lab = datagen.separated_clusters(20, 4, 6, sep=2.0, seed=1)
    rng = np.random.default_rng(3)
    params = [p.copy() for p in _mlp_params(6, seed=4)]
    moms = [np.zeros_like(p) for p in params]
    vels = [np.zeros_like(p) for p in params]
    B = 32
    def batch():
        a = rng.integers(0, len(X), B)
        p = np.array([rng.choice(np.flatnonzero((lab == lab[i]) & (np.arange(len(X)) != i))) for i in a])
        q = np.array([rng.choice(np.flatnonzero(lab != lab[i])) for i in a])
        return np.concatenate([a, p, q])
    fixed = batch()
    first = _loss(orc, X[fixed], params, B, 1.0)
    for t in range(1, 201):
        rows = batch()
        Z = orc.mlp_forward(X[rows], *params)
        _, dZ = orc.triplet_loss(Z, B, 1.0)
        grads = orc.mlp_backward(X[rows], params[0], params[1], params[2], dZ)
        for p, g, m, v in zip(params, grads, moms, vels):
            orc.adam_step(p, g, m, v, t, lr=1e-2)
    last = _loss(orc, X[fixed], params, B, 1.0)
    assert first > 1.0 and last < 0.1 * first, (first, last)


def test_proj_seed_line_equals_exact(orc):
    X = datagen.line_1d(400, seed=3)
    Z = X.astype(np.float64)            # identity encoder, m = 1
    dirs = np.array([[1.0]])
    for k in (1, 5, 15):
        idx, d2 = orc.proj_seed(X, Z, dirs, w=k, K=k)
        eidx, ed2 = orc.exact_knn(X, k)
        assert np.array_equal(idx, eidx) and np.array_equal(d2, ed2)


def test_proj_seed_invariants(orc):
    X = datagen.gmm_isotropic(n=500, d=8, seed=2)
    rng = np.random.default_rng(0)
    Z = rng.normal(size=(500, 4))
    dirs = rng.normal(size=(3, 4))
    idx, d2 = orc.proj_seed(X, Z, dirs, w=2, K=20)
    n = 500
    valid = idx >= 0
    assert np.all(valid.sum(1) >= 4)               # at least the two nearest in one order
    assert np.all(valid.sum(1) <= 12)              # 2 * w * P distinct candidates at most
    assert not np.any(idx == np.arange(n)[:, None])
    assert np.all(np.isinf(d2[~valid]))
    # every kept candidate is a window neighbour in some order
    for p in range(3):
        order = np.lexsort((np.arange(n), Z @ dirs[p]))
        rank = np.empty(n, dtype=np.int64)
        rank[order] = np.arange(n)
        for i in range(0, n, 50):
            win = set(order[max(0, rank[i] - 2): rank[i] + 3]) - {i}
            assert win <= set(idx[i][valid[i]]) or len(win | set(idx[i][valid[i]])) > 0


def test_zorder_keys_visit_quadrants_recursively(orc):
    """Z-order (D = 2): on a 16 x 16 grid whose coordinate range is exactly 16
    (one extra point at (16, 16) makes (hi - lo) * scale exact), the sorted
    order visits aligned 2^l x 2^l squares one after another at every level,
    the defining property of the curve."""
    g = np.array([(x, y) for x in range(16) for y in range(16)] + [(16, 16)], dtype=np.float32)
    keys = orc.proj_keys(g, np.eye(2, dtype=np.float32), D=2)
    order = np.lexsort((np.arange(len(g)), keys))[:256]
    pts = g[order].astype(int)
    assert sorted(map(tuple, pts)) == [(x, y) for x in range(16) for y in range(16)]
    for lvl in (1, 2, 3):
        side = 2 ** lvl
        blocks = pts.reshape(-1, side * side, 2)
        for b in blocks:
            assert (b[:, 0] // side).min() == (b[:, 0] // side).max()
            assert (b[:, 1] // side).min() == (b[:, 1] // side).max()
    # D = 1: keys order like the projections themselves
    z = np.random.default_rng(0).normal(size=(1000, 3)).astype(np.float32)
    k1 = orc.proj_keys(z, np.array([[1.0, 0.0, 0.0]], np.float32), D=1)
    assert np.array_equal(np.argsort(k1, kind="stable"), np.argsort(z[:, 0], kind="stable"))


def test_proj_seed_zorder_windows(orc):
    """Seeds from Z-order windows contain only window members and the best
    of them by true distance."""
    rng = np.random.default_rng(1)
    X = rng.normal(size=(400, 6))
    Z = X[:, :4].astype(np.float32)
    dirs = rng.normal(size=(2 * 4, 4)).astype(np.float32)     # P = 2 curves, D = 4
    idx, d2 = orc.proj_seed(X, Z, dirs, w=3, K=12, D=4)
    members = [set() for _ in range(400)]
    for p in range(2):
        keys = orc.proj_keys(Z, dirs[4 * p:4 * p + 4], D=4)
        order = np.lexsort((np.arange(400), keys))
        rank = np.empty(400, np.int64)
        rank[order] = np.arange(400)
        for i in range(400):
            members[i] |= set(order[max(0, rank[i] - 3): rank[i] + 4].tolist()) - {i}
    for i in range(400):
        cand = sorted(members[i], key=lambda j: (((X[i] - X[j]) ** 2).sum(), j))
        got = [j for j in idx[i] if j >= 0]
        assert got == cand[:12]


def _exact_mlp_case(rng, m=40, d=50):
    """Inputs on which every BF16 rounding of the BF16 mode is exact: small
    integers and quarters, so products, sums and hidden values keep at most
    8 significant bits."""
    X = rng.integers(-2, 3, size=(m, d)).astype(np.float64)
    W1 = rng.integers(-1, 2, size=(d, 64)) / 4.0
    b1 = rng.integers(-4, 5, size=64) / 4.0
    W2 = rng.integers(-1, 2, size=(64, 32)) / 4.0
    b2 = rng.integers(-4, 5, size=32) / 4.0
    return X, W1, b1, W2, b2


def test_mlp_bf16_mode_equals_fp64_when_rounding_is_exact(orc):
    rng = np.random.default_rng(3)
    X, W1, b1, W2, b2 = _exact_mlp_case(rng)
    Zb, Hb = orc.mlp_forward_bf16(X, W1, b1, W2, b2, want_hidden=True)
    Z, H = orc.mlp_forward(X, W1, b1, W2, b2, want_hidden=True)
    assert np.array_equal(Zb, Z) and np.array_equal(Hb, H)
    dZ = rng.integers(-3, 4, size=Z.shape) / 4.0
    for gb, g in zip(orc.mlp_backward_bf16(X, W1, b1, W2, dZ), orc.mlp_backward(X, W1, b1, W2, dZ)):
        assert np.array_equal(gb, g)


@pytest.mark.parametrize("which", ["X", "W1", "W2"])
def test_mlp_bf16_mode_rounds_each_factor(orc, which):
    """Perturb one factor off the BF16 grid: the BF16 mode equals the FP64
    forward of the same inputs with that factor rounded, and only that one."""
    rng = np.random.default_rng(4)
    X, W1, b1, W2, b2 = _exact_mlp_case(rng)
    args = {"X": X, "W1": W1, "W2": W2}
    off = args[which] * (1.0 + 2.0 ** -10)   # below BF16 resolution, above FP32's: rounds back
    args[which] = off
    Zb = orc.mlp_forward_bf16(args["X"], args["W1"], b1, args["W2"], b2)
    rounded = dict(args)
    rounded[which] = orc.bf16_values(off)
    Zr = orc.mlp_forward(rounded["X"], rounded["W1"], b1, rounded["W2"], b2)
    assert np.array_equal(Zb, Zr)
    assert not np.array_equal(orc.mlp_forward(args["X"], args["W1"], b1, args["W2"], b2), Zr)


def test_mlp_bf16_mode_close_to_fp64_on_generic_inputs(orc):
    """On generic data the BF16 mode differs from FP64 by the BF16 rounding:
    the embedding and gW2 by a nonzero amount within 3e-2 relative (tensor
    norm).  gW1 and gb1 also depend on the ReLU mask, which flips for hidden
    units within rounding of zero, and their batch sums cancel, so they are
    held to 1e-1."""
    rng = np.random.default_rng(5)
    X = datagen.gmm_isotropic(n=500, d=50, seed=5).astype(np.float64)
    W1 = rng.normal(0, 0.2, size=(50, 64))
    b1 = rng.normal(0, 0.1, size=64)
    W2 = rng.normal(0, 0.2, size=(64, 32))
    b2 = rng.normal(0, 0.1, size=32)
    Zb = orc.mlp_forward_bf16(X, W1, b1, W2, b2)
    Z = orc.mlp_forward(X, W1, b1, W2, b2)
    rel = np.linalg.norm(Zb - Z) / np.linalg.norm(Z)
    assert 0 < rel < 3e-2, rel
    dZ = rng.normal(size=Z.shape)
    for name, gb, g in zip(("gW1", "gb1", "gW2", "gb2"), orc.mlp_backward_bf16(X, W1, b1, W2, dZ),
                           orc.mlp_backward(X, W1, b1, W2, dZ)):
        rel = np.linalg.norm(gb - g) / np.linalg.norm(g)
        assert rel < (1e-1 if name in ("gW1", "gb1") else 3e-2), (name, rel)
