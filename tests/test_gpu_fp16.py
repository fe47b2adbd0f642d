"""FP16 MFMA distances (precision "fp16") for FP16-stored data.

FP16 data are exact as FP16 MFMA operands, so the candidates' squared
distances carry only the FP32 accumulation error of the norm expansion,
where the BF16 form first rounds every coordinate to 8 significant bits.
Checks: the exact path in the FP16 form has parity with the oracle on the
stored values (like the FP32 form, after the FP32 re-rank); NNDescent's FP16
form keeps working-list distances within 1e-4 (p99) of FP64, far tighter
than the BF16 form on the same data, and reaches the same recall; the
encoder-seeded FP16 form runs end to end.
"""
import numpy as np
import pytest
import torch

from paper_2603_04035_amd import datagen
from oracle.compare import exact_parity

pytestmark = pytest.mark.gpu


def _fp16_data(n, seed):
    X = datagen.gmm_anisotropic(n=n, d=50, comps=40, zipf=1.1, seed=seed, dtype=np.float16)
    return X, X.astype(np.float32)


def test_exact_fp16_form_parity(orc):
    import paper_2603_04035_amd as knn
    X16, X32 = _fp16_data(20_011, 1)
    Xd = torch.from_numpy(X16).cuda()
    idx, dist = knn.knn_exact(Xd, 15, precision="fp16")
    rows = datagen.sample_queries(20_011, 400, seed=3)
    O, O2 = orc.exact_knn(X32, 15, rows=rows)
    res = exact_parity(X32, rows, idx.cpu().numpy()[rows], dist.cpu().numpy()[rows], O)
    assert res["dist_err"] == 0 and res["self"] == 0 and res["dup"] == 0 and res["bad_index"] == 0, res
    r = orc.recall_at_k(X32, rows, idx.cpu().numpy()[rows], np.sqrt(O2[:, -1]), 15)
    assert r >= 0.999, r
    # FP32-stored input rounded to FP16 by the form: valid rows, distances of the FP32 values
    Xf = torch.from_numpy(X32).cuda()
    idx2, dist2 = knn.knn_exact(Xf, 15, precision="fp16")
    res2 = exact_parity(X32, rows, idx2.cpu().numpy()[rows], dist2.cpu().numpy()[rows], O)
    assert res2["dist_err"] == 0 and res2["self"] == 0 and res2["dup"] == 0, res2


def _list_error(orc, X32, rows, si, sd):
    si, sd = si.cpu().numpy()[rows], sd.cpu().numpy()[rows]
    ok = si >= 0
    a = np.repeat(rows, si.shape[1]).reshape(si.shape)[ok]
    true = orc.pair_d2(X32, a, si[ok])
    m = true > 0
    e = np.abs(sd[ok][m].astype(np.float64) - true[m]) / true[m]
    return float(np.percentile(e, 99))


def test_nndescent_fp16_form(orc):
    import paper_2603_04035_amd as knn
    X16, X32 = _fp16_data(200_000, 2)
    Xd = torch.from_numpy(X16).cuda()
    rows = datagen.sample_queries(200_000, 1000, seed=4)
    _, O2 = orc.exact_knn(X32, 15, rows=rows)
    out = {}
    for prec in ("fp16", "bf16"):
        G, D, st, (si, sd, _) = knn.nndescent_build(Xd, 15, precision=prec, build_k=30, sample_rate=1.0,
                                                    max_iters=30, delta=0.015, return_state=True)
        r = orc.recall_at_k(X32, rows, G.cpu().numpy()[rows], np.sqrt(O2[:, -1]), 15)
        out[prec] = (r, _list_error(orc, X32, rows, si, sd), st["iters"])
    print("fp16 / bf16 forms (recall, p99 list-distance error, iterations)", out)
    assert out["fp16"][1] <= 1e-4 and out["fp16"][1] < out["bf16"][1] / 10
    assert out["fp16"][0] >= out["bf16"][0] - 0.01 and out["fp16"][0] >= 0.95


def test_nndescent_fp16_encoder_seeded(orc):
    import paper_2603_04035_amd as knn
    X16, X32 = _fp16_data(50_000, 5)
    Xd = torch.from_numpy(X16).cuda()
    enc = knn.Encoder(50, seed=1)
    G, D, st = knn.nndescent_build(Xd, 15, precision="fp16", init_kind="encoder", encoder=enc, sample_rate=1.0,
                                   max_iters=30)
    rows = datagen.sample_queries(50_000, 300, seed=6)
    _, O2 = orc.exact_knn(X32, 15, rows=rows)
    r = orc.recall_at_k(X32, rows, G.cpu().numpy()[rows], np.sqrt(O2[:, -1]), 15)
    assert r >= 0.95, (r, st["iters"])
