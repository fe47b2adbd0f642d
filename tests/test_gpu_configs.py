"""The larger workloads at full size, as GPU parity cases.

* 70,000 x 784 pixel-like data, plain FP32 NNDescent, recall against the
  oracle's exact lists on sampled rows; the bar is set from the sequential
  oracle NNDescent's own recall at the same K_b, rho and delta
  (tests/golden/pixel70k_nnd.json, written by make_pixel70k_nnd.py).
* The same data stored in BF16: exact path with BF16 MFMA candidates and an
  FP32 re-rank of the top 30 (parity with the oracle on the stored values),
  and the NNDescent BF16 form (K_b = 30), whose working-list distances come
  from the BF16 MFMA join: their error against FP64 distances is reported,
  both of the stored (rounded) values and of the original FP32 values.
* 10,000,000 x 50 FP16 (200-component mixture, Zipf(1.1) weights), BF16
  form seeded by a trained encoder; recall on 10,000 sampled rows against the
  GPU exact path, which is itself checked against the oracle on 20 of them.
"""
import json
import os

import numpy as np
import pytest
import torch

from paper_2603_04035_amd import datagen
from oracle.compare import exact_parity, parity_ok

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows_ok(orc, X, rows, G, D, rel=1e-5):
    """Invariants of returned rows: valid, distinct, not self, sorted, and the
    returned distances equal the FP64 distances of the returned pairs."""
    n = X.shape[0]
    k = G.shape[1]
    assert np.all((G >= 0) & (G < n))
    assert not np.any(G == rows[:, None])
    s = np.sort(G, axis=1)
    assert not np.any(s[:, 1:] == s[:, :-1])
    assert np.all(np.diff(D, axis=1) >= 0)
    true = np.sqrt(orc.pair_d2(X, np.repeat(rows, k), G.ravel()).reshape(-1, k))
    err = np.abs(D - true) / np.maximum(true, 1e-30)
    assert np.all((err <= rel) | (true == 0)), err.max()


def _rel_err_stats(approx_d2, true_d2):
    m = true_d2 > 0
    e = np.abs(approx_d2[m] - true_d2[m]) / true_d2[m]
    return {"max": float(e.max()), "p50": float(np.percentile(e, 50)), "p99": float(np.percentile(e, 99))}


def test_pixel70k_fp32_nndescent(orc):
    import paper_2603_04035_amd as knn
    gold = json.load(open(os.path.join(GOLDEN, "pixel70k_nnd.json")))
    X = datagen.pixel_like(n=70000, seed=0)
    rows = datagen.sample_queries(70000, 300, seed=2)
    G, D, st = knn.nndescent_build(torch.from_numpy(X).cuda(), 15, build_k=32, sample_rate=1.0,
                                   max_iters=30, delta=0.015)
    G, D = G.cpu().numpy()[rows], D.cpu().numpy()[rows]
    _rows_ok(orc, X, rows, G, D)
    _, O2 = orc.exact_knn(X, 15, rows=rows)
    r = orc.recall_at_k(X, rows, G, np.sqrt(O2[:, -1]), 15)
    print("pixel70k fp32 recall", r, "oracle", gold["oracle_recall_at_15"], "iters", st["iters"])
    # the GPU's approximations (at most join_cap = 4 partners per member
    # and join list, join lists cut at 64 members: list_dropped counts them,
    # hashed candidate slots) cost 0.023 here (0.810 against 0.833)
    assert r >= gold["oracle_recall_at_15"] - 0.03, (r, gold)


def test_pixel70k_bf16_storage_precision_form(orc):
    import paper_2603_04035_amd as knn
    X32 = datagen.pixel_like(n=70000, seed=0)
    bits = orc.round_bf16(X32)
    Xs = orc.bf16_to_f64(bits).astype(np.float32)   # the stored values, exactly
    Xb = torch.from_numpy(Xs).cuda().to(torch.bfloat16)
    rows = datagen.sample_queries(70000, 150, seed=2)
    O, O2 = orc.exact_knn(Xs, 15, rows=rows)

    # exact path: BF16 MFMA candidates, FP32 re-rank of the top 30
    idx, dist = knn.knn_exact(Xb, 15, precision="bf16", rerank_k=30)
    idx, dist = idx.cpu().numpy()[rows], dist.cpu().numpy()[rows]
    res = exact_parity(Xs, rows, idx, dist, O)
    print("pixel70k bf16 exact", res)
    assert res["dist_err"] == 0 and res["self"] == 0 and res["dup"] == 0, res
    r_exact = orc.recall_at_k(Xs, rows, idx, np.sqrt(O2[:, -1]), 15)
    assert r_exact >= 0.99, r_exact

    # NNDescent BF16 form: K_b = 30, FP32 re-rank of the final lists
    G, D, st, (si, sd, _) = knn.nndescent_build(Xb, 15, precision="bf16", build_k=30, sample_rate=1.0,
                                                max_iters=30, delta=0.015, return_state=True)
    G, D = G.cpu().numpy()[rows], D.cpu().numpy()[rows]
    _rows_ok(orc, Xs, rows, G, D)
    r = orc.recall_at_k(Xs, rows, G, np.sqrt(O2[:, -1]), 15)
    # working-list distances (BF16 MFMA join, norm expansion) against FP64
    si, sd = si.cpu().numpy()[rows], sd.cpu().numpy()[rows]
    ok = si >= 0
    a = np.repeat(rows, si.shape[1]).reshape(si.shape)[ok]
    b = si[ok]
    vs_stored = _rel_err_stats(sd[ok].astype(np.float64), orc.pair_d2(Xs, a, b))
    vs_orig = _rel_err_stats(sd[ok].astype(np.float64), orc.pair_d2(X32, a, b))
    print("pixel70k bf16 form recall", r, "iters", st["iters"], "err vs stored", vs_stored,
          "err vs original", vs_orig)
    assert r >= 0.76, r   # measured 0.788
    assert vs_stored["p99"] <= 1e-3, vs_stored
    assert vs_orig["p99"] <= 5e-2, vs_orig


def test_scale_10m_fp16_learned_bf16(orc):
    import bench
    import paper_2603_04035_amd as knn
    X = torch.from_numpy(bench.make_data("scale10m")).cuda()
    assert X.dtype == torch.float16 and X.shape == (10_000_000, 50)
    enc, info = bench.train_encoder("scale10m")
    assert info["loss_last"] < info["loss_first"], info
    p = dict(bench.FORMS["bf16-learned"], encoder=enc)
    G, D, st = knn.nndescent_build(X, 15, seed=0, **p)
    rows = datagen.sample_queries(10_000_000, 10_000, seed=2)
    rows_t = torch.as_tensor(rows, device="cuda")
    eidx, edist = knn.knn_exact_query(X[rows_t].contiguous(), X, 15, q_self=rows_t.to(torch.int32))
    # the exact path at this size, pinned to the oracle on 20 rows
    few = np.arange(20)
    Xh = X.cpu().numpy()
    O, _ = orc.exact_query(Xh, Xh[rows[few]], 15, q_self=rows[few])
    res = exact_parity(Xh, rows[few], eidx.cpu().numpy()[few], edist.cpu().numpy()[few], O)
    assert parity_ok(res), res
    r = bench.recall_gpu(X, G, D, rows, 15)
    Gs, Ds = G[rows_t].cpu().numpy(), D[rows_t].cpu().numpy()
    _rows_ok(orc, Xh, rows[:200], Gs[:200], Ds[:200])
    print("scale10m recall", r, "iters", st["iters"], "ms", st["ms_total"])
    assert r >= 0.9, (r, st)


def test_benchmark_forms_meet_recall(orc):
    """Both benchmark forms, with exactly the settings bench.py times, on the
    1,000,000 x 50 mixture: recall@15 >= 0.98 over 10,000 sampled rows (the
    metric's condition; the exact lists come from the exact path, pinned to
    the oracle on 20 of the rows), valid rows and oracle-exact distances on
    300 of them."""
    import bench
    import paper_2603_04035_amd as knn
    Xn = bench.make_data("gmm1m")
    X = torch.from_numpy(Xn).cuda()
    enc, _ = bench.train_encoder("gmm1m")
    rows = datagen.sample_queries(X.shape[0], 10_000, seed=2)
    rows_t = torch.as_tensor(rows, device="cuda")
    eidx, edist = knn.knn_exact_query(X[rows_t].contiguous(), X, 15, q_self=rows_t.to(torch.int32))
    few = np.arange(20)
    O, _ = orc.exact_query(Xn, Xn[rows[few]], 15, q_self=rows[few])
    res = exact_parity(Xn, rows[few], eidx.cpu().numpy()[few], edist.cpu().numpy()[few], O)
    assert parity_ok(res), res
    for form in ("bf16-learned", "fp32"):
        p = dict(bench.FORMS[form])
        if p.get("init_kind") == "encoder":
            p["encoder"] = enc
        G, D, st = knn.nndescent_build(X, 15, seed=0, **p)
        r = bench.recall_gpu(X, G, D, rows, 15)
        print(form, "recall", r, "iters", st["iters"])
        assert r >= 0.98, (form, r)
        _rows_ok(orc, Xn, rows[:300], G[rows_t[:300]].cpu().numpy(), D[rows_t[:300]].cpu().numpy())
