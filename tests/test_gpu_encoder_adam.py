"""The encoder's optimiser on the GPU against the oracle (Adam of Kingma & Ba,
the learned-initialisation form's training).

For three consecutive training steps, in both product precisions: the rows
``knn_encoder_train`` draws are those ``knn_encoder_triplets`` reports for
that step, every positive is one of its anchor's listed neighbours, and the
weights and both Adam moments after the step equal the oracle's Adam step
(FP64) applied to the GPU's own gradient of those rows at the weights before
the step.  The oracle takes the settings as the FP32 values the call
carries (lr, beta1 = fl(0.9), beta2 = fl(0.999)).  The GPU computes the
update in FP32, so the bars are a few FP32 ulps: of each weight plus a 1e-6
share of the step size, and of the two terms of each moment update (the
terms of the first moment can cancel, so its relative error is not small).
"""
import numpy as np
import pytest
import torch

from paper_2603_04035_amd import datagen

pytestmark = pytest.mark.gpu


def F(x):
    """The FP32 value a float setting carries, as a double."""
    return float(np.float32(x))


def _flat(enc):
    return np.concatenate([a.ravel() for a in enc.get_weights()]).astype(np.float64)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_train_steps_match_oracle_adam(orc, precision):
    import paper_2603_04035_amd as knn
    from paper_2603_04035_amd import Encoder
    from paper_2603_04035_amd.encoder import triplets
    n, d, k, B = 3000, 50, 15, 512
    lr, seed = 2e-3, 17
    X = torch.from_numpy(datagen.gmm_anisotropic(n=n, d=d, comps=10, seed=4)).cuda()
    gidx, _ = knn.knn_exact(X, k)
    G = gidx.cpu().numpy()
    enc = Encoder(d, seed=2)
    m_o = np.zeros(enc.n_params)
    v_o = np.zeros(enc.n_params)
    for step in range(3):
        w0 = _flat(enc)
        m_g, v_g, t = enc.adam_state()
        assert t == step
        rows = triplets(gidx, B, seed, t)
        r = rows.cpu().numpy()
        a, p, q = r[:B], r[B:2 * B], r[2 * B:]
        assert np.all((a >= 0) & (a < n)) and np.all((q >= 0) & (q < n))
        assert np.all((G[a] == p[:, None]).any(axis=1)), "a positive is not a listed neighbour"
        _, g = enc.grads(X, rows, B, margin=1.0, precision=precision)
        g = g.cpu().numpy().astype(np.float64)
        enc.train(X, gidx, steps=1, batch=B, lr=lr, margin=1.0, seed=seed, precision=precision)
        w1 = _flat(enc)
        m1, v1, t1 = enc.adam_state()
        assert t1 == step + 1
        w = w0.copy()
        # FP32 rounding of each moment update: a few ulps of its two terms
        # (they can cancel in the first moment)
        eps = np.finfo(np.float32).eps
        bar_m = 4 * eps * (F(0.9) * np.abs(m_o) + (1 - F(0.9)) * np.abs(g)) + 1e-30
        bar_v = 4 * eps * (F(0.999) * v_o + (1 - F(0.999)) * g * g) + 1e-38
        orc.adam_step(w, g, m_o, v_o, t=step + 1, lr=F(lr), beta1=F(0.9), beta2=F(0.999))
        bar = 4 * eps * np.abs(w0) + 1e-6 * lr
        assert np.all(np.abs(w1 - w) <= bar), np.max(np.abs(w1 - w) - bar)
        assert np.all(np.abs(m1 - m_o) <= bar_m), np.max(np.abs(m1 - m_o) / bar_m)
        assert np.all(np.abs(v1 - v_o) <= bar_v), np.max(np.abs(v1 - v_o) / bar_v)
        # the oracle continues from the GPU's moments (FP32-rounded)
        m_o[:] = m1
        v_o[:] = v1


def test_step_on_given_rows_equals_train(orc):
    """knn_encoder_step on the reported triplets is the training step, bit for
    bit; on arbitrary rows it is the oracle's Adam step on the GPU gradient."""
    import paper_2603_04035_amd as knn
    from paper_2603_04035_amd import Encoder
    from paper_2603_04035_amd.encoder import triplets
    n, d, k, B = 2000, 50, 10, 300
    X = torch.from_numpy(datagen.gmm_isotropic(n=n, d=d, seed=6)).cuda()
    gidx, _ = knn.knn_exact(X, k)
    a, b = Encoder(d, seed=9), Encoder(d, seed=9)
    a.train(X, gidx, steps=1, batch=B, lr=1e-3, seed=4)
    b.step(X, triplets(gidx, B, 4, 0), B, lr=1e-3)
    for wa, wb in zip(a.get_weights(), b.get_weights()):
        assert np.array_equal(wa, wb)
    rng = np.random.default_rng(1)
    rows = torch.from_numpy(rng.integers(0, n, size=3 * B).astype(np.int32))
    w0 = _flat(b)
    m0, v0, t0 = b.adam_state()
    _, g = b.grads(X, rows, B)
    b.step(X, rows, B, lr=1e-3)
    w = w0.copy()
    m, v = m0.astype(np.float64), v0.astype(np.float64)
    orc.adam_step(w, g.cpu().numpy().astype(np.float64), m, v, t=t0 + 1, lr=F(1e-3), beta1=F(0.9),
                  beta2=F(0.999))
    eps = np.finfo(np.float32).eps
    gg = g.cpu().numpy().astype(np.float64)
    bar_m = 4 * eps * (F(0.9) * np.abs(m0) + (1 - F(0.9)) * np.abs(gg)) + 1e-30
    bar_v = 4 * eps * (F(0.999) * v0 + (1 - F(0.999)) * gg * gg) + 1e-38
    bar = 4 * eps * np.abs(w0) + 1e-9
    assert np.all(np.abs(b.adam_state()[0] - m) <= bar_m)
    assert np.all(np.abs(b.adam_state()[1] - v) <= bar_v)
    assert np.all(np.abs(_flat(b) - w) <= bar)
