"""Comparators: tie-aware recall and the exact-path parity rule (test infrastructure).

Distances here are Euclidean (square roots of fp64 squared distances computed
from the stored input values).

* near tie: two distances a, b are tied when |a - b| <= rel * max(a, b)
  (equal zeros are tied); rel = 1e-5.
* exact-path parity, per row i and rank r, with O the oracle's list and G the
  list under test:
    - G[i] holds k distinct indices, none equal to i, all in range;
    - the returned distance of G[i][r] agrees with the fp64 distance of that
      pair to ``rel`` relative;
    - G[i][r] == O[i][r] unless their fp64 distances are near-tied;
    - the fp64 distance of G[i][r] is near-tied with (or equal to) that of
      O[i][r] rank by rank, so a swap across the rank-k boundary is only
      allowed inside a near-tie group.
* recall@k (tie-aware): (1/(n k)) sum_i min(k, #{j in G(i) : D(i, j) <=
  D*_k(i) (1 + rel)}) with D*_k the exact k-th distance.
"""
from __future__ import annotations

import numpy as np

REL = 1e-5


def near_tie(a, b, rel: float = REL):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.abs(a - b) <= rel * np.maximum(np.abs(a), np.abs(b))


def _row_dist(X, rows, G):
    """fp64 Euclidean distances between X[rows[i]] and X[G[i, r]] (G may hold -1)."""
    X = np.asarray(X, dtype=np.float64)
    Gc = np.where(G < 0, 0, G)
    diff = X[np.asarray(rows)][:, None, :] - X[Gc]
    out = np.sqrt(np.einsum("ijk,ijk->ij", diff, diff))
    return np.where(G < 0, np.inf, out)


def exact_parity(X, rows, G, gdist, O, odist2=None, rel: float = REL,
                 squared: bool = False) -> dict:
    """Check a k-NN result (G, gdist) against the oracle list O for query rows.

    ``gdist`` is what the path returned (Euclidean, or squared when
    ``squared``).  Returns counts of violations (all zero means parity) plus
    the number of index mismatches that were excused as near ties.
    """
    rows = np.asarray(rows, dtype=np.int64)
    G = np.asarray(G, dtype=np.int64)
    O = np.asarray(O, dtype=np.int64)
    n = np.asarray(X).shape[0]
    k = O.shape[1]
    res = {"rows": int(len(rows)), "k": int(k), "bad_shape": 0, "bad_index": 0, "self": 0,
           "dup": 0, "dist_err": 0, "order_err": 0, "rank_dist_err": 0, "tie_swaps": 0,
           "max_dist_rel": 0.0}
    if G.shape != O.shape:
        res["bad_shape"] = 1
        return res
    oob = (G < 0) | (G >= n)
    res["bad_index"] = int(oob.sum())
    res["self"] = int((G == rows[:, None]).sum())
    srt = np.sort(G, axis=1)
    res["dup"] = int((srt[:, 1:] == srt[:, :-1]).sum())
    if res["bad_index"]:
        return res
    dg = _row_dist(X, rows, G)            # fp64 distance of the returned pair
    do = _row_dist(X, rows, O)            # fp64 distance of the oracle's pair
    ret = np.asarray(gdist, dtype=np.float64)
    if squared:
        ret = np.sqrt(np.maximum(ret, 0.0))
    ok = near_tie(ret, dg, rel) | ((ret == 0) & (dg == 0))
    res["dist_err"] = int((~ok).sum())
    with np.errstate(invalid="ignore", divide="ignore"):
        relerr = np.abs(ret - dg) / np.where(dg > 0, dg, 1.0)
    res["max_dist_rel"] = float(np.max(relerr)) if relerr.size else 0.0
    mism = G != O
    tied = near_tie(dg, do, rel) | ((dg == 0) & (do == 0))
    res["order_err"] = int((mism & ~tied).sum())
    res["tie_swaps"] = int((mism & tied).sum())
    res["rank_dist_err"] = int((~tied).sum())
    return res


def parity_ok(res: dict) -> bool:
    return all(res[k] == 0 for k in ("bad_shape", "bad_index", "self", "dup", "dist_err",
                                     "order_err", "rank_dist_err"))


def recall_at_k(X, rows, G, exact_kth, k: int, rel: float = REL) -> float:
    """Tie-aware recall of the first k columns of G for the query rows.

    ``exact_kth`` holds the exact (oracle or validated exact path) k-th
    Euclidean distance of each query row.
    """
    rows = np.asarray(rows, dtype=np.int64)
    G = np.asarray(G, dtype=np.int64)[:, :k]
    dg = _row_dist(X, rows, G)
    thr = np.asarray(exact_kth, dtype=np.float64)[:, None] * (1.0 + rel)
    valid = (G >= 0) & (G != rows[:, None])
    order = np.argsort(G, axis=1, kind="stable")
    srt = np.take_along_axis(G, order, axis=1)
    first = np.ones_like(valid)
    first[:, 1:] = srt[:, 1:] != srt[:, :-1]          # later copies of an index do not count
    uniq = np.empty_like(first)
    np.put_along_axis(uniq, order, first, axis=1)
    hit = ((dg <= thr) & valid & uniq).sum(axis=1)
    return float(np.minimum(hit, k).sum() / (len(rows) * k))


def index_recall(G, O, k: int) -> float:
    """Plain index-intersection recall of the first k columns."""
    G = np.asarray(G)[:, :k]
    O = np.asarray(O)[:, :k]
    hits = sum(len(np.intersect1d(g, o)) for g, o in zip(G, O))
    return hits / (G.shape[0] * k)
