"""Writes config1_nnd.json: the CPU oracle's sequential NNDescent recall@15 on
the 5,000 x 50 isotropic mixture (datagen.gmm_isotropic(n=5000, d=50,
seed=0)) at K_b = 15, rho = 0.5, delta = 0.015 and at most 8 iterations, for
algorithm seeds 0-4, against the oracle's exact kNN on all rows.  Calls only
the oracle and the seeded input generator; seconds on one core."""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2603_04035_amd import datagen  # noqa: E402


def main():
    n, K, rho, delta, iters = 5000, 15, 0.5, 0.015, 8
    X = datagen.gmm_isotropic(n=n, d=50, seed=0)
    rows = np.arange(n)
    _, O2 = oracle.exact_knn(X, 15)
    rec, its = [], []
    for seed in range(5):
        idx, _, it, _ = oracle.nndescent(X, K, max_iters=iters, rho=rho, delta=delta, seed=seed)
        rec.append(float(oracle.recall_at_k(X, rows, idx[:, :15], np.sqrt(O2[:, -1]), 15)))
        its.append(int(it))
    out = {"workload": "gmm_isotropic(n=5000, d=50, seed=0)", "k": 15, "build_k": K, "rho": rho,
           "delta": delta, "max_iters": iters, "seeds": list(range(5)), "rows": "all",
           "oracle_recall_at_15": rec, "oracle_iters": its,
           "oracle_recall_mean": float(np.mean(rec)), "oracle_recall_sd": float(np.std(rec))}
    with open(os.path.join(HERE, "config1_nnd.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(out)


if __name__ == "__main__":
    main()
