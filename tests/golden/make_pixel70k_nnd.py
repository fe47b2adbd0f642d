"""Writes pixel70k_nnd.json: the CPU oracle's sequential NNDescent recall@15 on
the 70,000 x 784 pixel-like workload (K_b = 32, rho = 1, delta = 0.015, seed 0),
measured on 300 sampled rows against the oracle's exact kNN.  Calls only the
oracle and the seeded input generator.  Takes a few minutes on one core."""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2603_04035_amd import datagen  # noqa: E402


def main():
    n, K, rho, delta = 70000, 32, 1.0, 0.015
    X = datagen.pixel_like(n=n, seed=0)
    rows = datagen.sample_queries(n, 300, seed=2)
    _, O2 = oracle.exact_knn(X, 15, rows=rows)
    idx, _, iters, _ = oracle.nndescent(X, K, max_iters=30, rho=rho, delta=delta, seed=0)
    r = oracle.recall_at_k(X, rows, idx[rows, :15], np.sqrt(O2[:, -1]), 15)
    out = {"workload": "pixel_like(n=70000, seed=0)", "k": 15, "build_k": K, "rho": rho, "delta": delta,
           "seed": 0, "rows": "sample_queries(70000, 300, seed=2)", "oracle_recall_at_15": float(r),
           "oracle_iters": int(iters)}
    with open(os.path.join(HERE, "pixel70k_nnd.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(out)


if __name__ == "__main__":
    main()
