"""knn_exact_noalloc (the entry point for callers that cannot allocate device
memory) against knn_exact, the entry point it mirrors: identical indices and
distances on two calls in a row, the first large enough that the queries run
in several chunks of the static array, the second smaller (the array keeps
the first call's contents, which must not leak into the second).  A few rows
of each are also checked against the oracle, and an input whose staged copy
cannot fit the array is refused with KNN_ENOMEM before any work."""
import numpy as np
import pytest
import torch

from paper_2603_04035_amd import datagen

pytestmark = pytest.mark.gpu


def _same(a, b):
    return torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


@pytest.mark.parametrize("precision,d", [("fp32", 50), ("bf16", 50), ("fp32", 2)])
def test_noalloc_matches_knn_exact_twice(orc, precision, d):
    """d = 50: the GEMM path (part lists alone: 150K x 2 x 256 B > 64 MiB);
    d = 2 in FP32: the direct path (split lists 150K x 4 x 256 B > 64 MiB)."""
    import paper_2603_04035_amd as knn
    from oracle.compare import exact_parity, parity_ok
    big = datagen.gmm_isotropic(n=150_000, d=d, seed=3)
    small = datagen.gmm_isotropic(n=3_001, d=d, seed=4)
    for X in (big, small):
        print("noalloc case", X.shape, precision, flush=True)
        Xd = torch.from_numpy(X).cuda()
        ref = knn.knn_exact(Xd, 15, precision=precision)
        got = knn.knn_exact_noalloc(Xd, 15, precision=precision)
        torch.cuda.synchronize()
        assert _same(ref, got)
        rows = datagen.sample_queries(X.shape[0], 40, seed=5)
        O, _ = orc.exact_knn(X, 15, rows=rows)
        res = exact_parity(X, rows, got[0].cpu().numpy()[rows], got[1].cpu().numpy()[rows], O)
        if precision == "fp32":
            assert parity_ok(res), res
        else:
            assert res["dist_err"] == 0 and res["self"] == 0 and res["dup"] == 0, res


def test_noalloc_into_given_outputs_and_limit():
    import paper_2603_04035_amd as knn
    from paper_2603_04035_amd._lib import KNN_ENOMEM, KnnError
    X = torch.from_numpy(datagen.gmm_isotropic(n=4000, d=50, seed=6)).cuda()
    oi = torch.full((4000, 10), -7, dtype=torch.int32, device="cuda")
    od = torch.zeros((4000, 10), dtype=torch.float32, device="cuda")
    knn.knn_exact_noalloc(X, 10, out_idx=oi, out_dist=od)
    ref = knn.knn_exact(X, 10)
    assert torch.equal(oi, ref[0]) and torch.equal(od, ref[1])
    # 300,000 x 50 FP32 stages 76.8 MB: more than the 64 MiB array
    Y = torch.zeros((300_000, 50), dtype=torch.float32, device="cuda")
    with pytest.raises(KnnError) as e:
        knn.knn_exact_noalloc(Y, 5)
    assert e.value.status == KNN_ENOMEM
