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
