"""bench.recall_gpu's scoring (CPU tensors, exact lists from the oracle):
an entry counts only if its index is valid, not the row itself and not a
repeat within the row, and only by its recomputed distance, never the one
the graph reports."""
import numpy as np
import torch

from paper_2603_04035_amd import datagen


def test_recall_ignores_reported_distances_and_bad_entries(orc):
    import bench
    X = datagen.gmm_isotropic(n=400, d=6, seed=5)
    k = 5
    rows = np.arange(0, 400, 7)
    O, O2 = orc.exact_knn(X, k, rows=rows)
    kth = torch.from_numpy(np.sqrt(O2[:, -1]))
    ex = (torch.from_numpy(rows), kth)
    Xt = torch.from_numpy(X)
    G = torch.full((400, k), -1, dtype=torch.int32)
    G[torch.from_numpy(rows)] = torch.from_numpy(O.astype(np.int32))
    D = torch.zeros((400, k))
    assert bench.recall_gpu(Xt, G, D, rows, k, exact=ex) == 1.0
    bad = G.clone()
    r0, r1, r2, r3 = rows[:4]
    bad[r0, 0] = int(r0)                    # the row itself
    bad[r1, 1] = bad[r1, 0]                 # a repeat
    bad[r2, 2] = 400                        # out of range
    far = int(np.argmax(((X - X[r3]) ** 2).sum(1)))
    bad[r3, 3] = far                        # a valid but distant point
    lost = 4
    assert bench.recall_gpu(Xt, bad, D, rows, k, exact=ex) == (len(rows) * k - lost) / (len(rows) * k)
    # reported distances play no part: zeros everywhere above, huge here
    assert bench.recall_gpu(Xt, G, D + 1e9, rows, k, exact=ex) == 1.0


def test_bench_refuses_several_gpus():
    """The bench measures one GPU: --gpus 2 exits with status 2 and says so,
    before touching any device."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    p = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2 and "one GPU" in p.stderr, (p.returncode, p.stderr)


def test_cpu_baseline_leg_fields():
    """The CPU leg's record: the oracle's sequential NNDescent rate on the
    sample (one core) with its recall, the exact oracle's query rate, and the
    subset caveat only when the sample is a subset."""
    import bench
    X = datagen.gmm_anisotropic(n=2500, d=50, comps=50, seed=0)
    part = bench.cpu_baseline(X, 15, "fp32", 1200, exact_queries=40)
    assert part["kind"] == "oracle" and part["cores"] == 1 and part["unit"] == "points/s"
    assert part["value"] > 0 and 0.0 <= part["recall_at_15"] <= 1.0
    assert "overstates" in part["sample"] and "first 1200 of the 2500 rows" in part["sample"]
    assert part["exact_oracle"]["queries"] == 40 and part["exact_oracle"]["queries_per_s"] > 0
    full = bench.cpu_baseline(X[:1200], 15, "fp32", 1200, exact_queries=40)
    assert "overstates" not in full["sample"]
