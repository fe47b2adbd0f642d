"""CPU oracle for the kNN-graph path -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg use
this package.  The library never imports it, and it imports nothing from the
library (inputs come from ``paper_2603_04035_amd.datagen`` in the callers).

What it computes (the C part lives in ``knn_oracle.c``):

* ``exact_knn`` / ``exact_query`` - the definition of the exact k nearest
  neighbours (the paper ranks neighbours by exact pairwise Euclidean distance
  in its embedding-quality section): fp64 direct-difference squared distances,
  ordered by (distance, index), self excluded.
* ``nndescent`` - sequential NNDescent of Dong, Charikar & Li (WWW 2011), the
  algorithm of the paper's GPU-native k-NN section, with its delta = 0.015
  early-termination rule; ``nndescent_trace`` also returns the per-iteration
  lists, samples and reverse unions.
* ``round_bf16`` - FP32 -> BF16 round-to-nearest-even by bit definition.
* ``mlp_forward`` / ``triplet_loss`` / ``mlp_backward`` / ``adam_step`` - the
  seeding encoder (d -> 64 -> 32, ReLU) in fp64.
* ``proj_seed`` - seed lists from sorted projections of an embedding.
* ``recall_at_k`` / ``exact_parity`` - the comparators (``compare.py``).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

from .compare import recall_at_k, index_recall, exact_parity, near_tie  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "knn_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")


def build(verbose: bool = False) -> str:
    """Compile knn_oracle.c with gcc (no fast-math: evaluation order is kept)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
           "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", _LIB_PATH + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build()
    lib = C.CDLL(_LIB_PATH)
    i64, i32, f64, u64 = C.c_int64, C.c_int, C.c_double, C.c_uint64
    lib.oracle_exact_query.argtypes = [_dp, i64, i64, i32, _dp, i64, i64, C.c_void_p, i32, _ip, _dp]
    lib.oracle_exact_query.restype = i32
    lib.oracle_pair_d2.argtypes = [_dp, i64, i32, _ip, _ip, i64, _dp]
    lib.oracle_pair_d2.restype = None
    lib.oracle_nndescent.argtypes = [_dp, i64, i64, i32, i32, i32, f64, f64, u64, C.c_void_p,
                                     _ip, _dp, C.POINTER(C.c_int), _ip]
    lib.oracle_nndescent.restype = i32
    _u8 = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
    lib.oracle_nndescent_traced.argtypes = [_dp, i64, i64, i32, i32, i32, f64, f64, u64, C.c_void_p,
                                            _ip, _dp, C.POINTER(C.c_int), _ip, i32,
                                            _ip, _u8, _ip, _ip, _ip, _ip]
    lib.oracle_nndescent_traced.restype = i32
    lib.oracle_round_bf16.argtypes = [np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS"),
                                      np.ctypeslib.ndpointer(dtype=np.uint16, flags="C_CONTIGUOUS"), i64]
    lib.oracle_round_bf16.restype = None
    lib.oracle_mlp_forward.argtypes = [_dp, i64, i64, i32, _dp, _dp, i32, _dp, _dp, i32, C.c_void_p, _dp]
    lib.oracle_mlp_forward.restype = None
    lib.oracle_triplet_loss.argtypes = [_dp, i64, i32, f64, C.c_void_p]
    lib.oracle_triplet_loss.restype = f64
    lib.oracle_mlp_backward.argtypes = [_dp, i64, i64, i32, _dp, _dp, i32, _dp, i32, _dp,
                                        _dp, _dp, _dp, _dp]
    lib.oracle_mlp_backward.restype = None
    lib.oracle_adam_step.argtypes = [_dp, _dp, _dp, _dp, i64, f64, f64, f64, f64, i32]
    lib.oracle_adam_step.restype = None
    _fp = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
    lib.oracle_proj_seed.argtypes = [_dp, i64, i64, i32, _fp, i32, _fp, i32, i32, i32, i32, _ip, _dp]
    lib.oracle_proj_seed.restype = i32
    lib.oracle_proj_keys.argtypes = [_fp, i64, i32, _fp, i32,
                                     np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS"), _fp]
    lib.oracle_proj_keys.restype = i32
    lib.oracle_fuzzy_rows.argtypes = [_dp, i64, i32, _dp, _dp, _dp]
    lib.oracle_fuzzy_rows.restype = None
    lib.oracle_quality_rows.argtypes = [_dp, i32, _dp, i32, i64, i32, _ip, i64, i32, _ip, _ip, _ip]
    lib.oracle_quality_rows.restype = i32
    _lib = lib
    return lib


def _f64(a) -> np.ndarray:
    """Exact upcast of the stored values (f16/bf16-as-f32/f32 -> f64)."""
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def exact_query(R, Q, k: int, q_self=None):
    """k nearest rows of R for every row of Q: (idx int64, squared dist f64).

    q_self[i] (optional) names a row of R that query i must not return.
    """
    R = _f64(R)
    Q = _f64(Q)
    if R.ndim != 2 or Q.ndim != 2 or R.shape[1] != Q.shape[1]:
        raise ValueError("shape mismatch")
    nq = Q.shape[0]
    idx = np.empty((nq, k), dtype=np.int64)
    d2 = np.empty((nq, k), dtype=np.float64)
    qs = None
    if q_self is not None:
        qs_arr = np.ascontiguousarray(np.asarray(q_self, dtype=np.int64))
        qs = qs_arr.ctypes.data_as(C.c_void_p)
    rc = _load().oracle_exact_query(R, R.shape[0], R.shape[1], R.shape[1], Q, nq, Q.shape[1],
                                    qs, k, idx, d2)
    if rc != 0:
        raise ValueError("oracle_exact_query: bad arguments")
    return idx, d2


def exact_knn(X, k: int, rows=None):
    """Exact kNN of the rows of X among X itself (self excluded).

    ``rows`` restricts the queries to a subset (sampled checks at full size).
    """
    X = _f64(X)
    rows = np.arange(X.shape[0], dtype=np.int64) if rows is None else np.asarray(rows, np.int64)
    return exact_query(X, X[rows], k, q_self=rows)


def pair_d2(X, a, b) -> np.ndarray:
    X = _f64(X)
    a = np.ascontiguousarray(np.asarray(a, np.int64).ravel())
    b = np.ascontiguousarray(np.asarray(b, np.int64).ravel())
    out = np.empty(a.shape[0], dtype=np.float64)
    _load().oracle_pair_d2(X, X.shape[1], X.shape[1], a, b, a.shape[0], out)
    return out


def nndescent(X, K: int, max_iters: int = 10, rho: float = 0.5, delta: float = 0.015,
              seed: int = 0, init_idx=None):
    """Sequential NNDescent; returns (idx n x K, squared dist, iters, updates)."""
    X = _f64(X)
    n, d = X.shape
    idx = np.empty((n, K), dtype=np.int64)
    d2 = np.empty((n, K), dtype=np.float64)
    iters = C.c_int(0)
    upd = np.zeros(max(1, max_iters), dtype=np.int64)
    ini = None
    if init_idx is not None:
        ini_arr = np.ascontiguousarray(np.asarray(init_idx, dtype=np.int64))
        if ini_arr.shape != (n, K):
            raise ValueError("init_idx must be n x K")
        ini = ini_arr.ctypes.data_as(C.c_void_p)
    rc = _load().oracle_nndescent(X, n, d, d, K, max_iters, float(rho), float(delta),
                                  int(seed) & ((1 << 64) - 1), ini, idx, d2,
                                  C.byref(iters), upd)
    if rc != 0:
        raise ValueError("oracle_nndescent: bad arguments")
    return idx, d2, iters.value, upd[:iters.value].copy()


def nndescent_trace(X, K: int, max_iters: int, rho: float = 0.5, delta: float = 0.0,
                    seed: int = 0, init_idx=None, trace_iters: int | None = None):
    """Sequential NNDescent with a trace of its first ``trace_iters`` iterations.

    Returns (idx, squared dist, iters, updates, trace) where trace holds, per
    iteration t and point v (-1 pads every list): ``lidx`` / ``lflag`` (T x n x
    K) the list and its new-flags as iteration t starts; ``newf`` (T x n x S)
    and ``oldf`` (T x n x K) the forward samples; ``new`` (T x n x 2S) and
    ``old`` (T x n x (K+S)) the lists after the reverse union.
    """
    X = _f64(X)
    n, d = X.shape
    T = max_iters if trace_iters is None else trace_iters
    S = int(np.ceil(rho * K))
    idx = np.empty((n, K), dtype=np.int64)
    d2 = np.empty((n, K), dtype=np.float64)
    iters = C.c_int(0)
    upd = np.zeros(max(1, max_iters), dtype=np.int64)
    T1 = max(T, 1)
    tr = {"lidx": np.full((T1, n, K), -1, np.int64), "lflag": np.zeros((T1, n, K), np.uint8),
          "newf": np.full((T1, n, S), -1, np.int64), "oldf": np.full((T1, n, K), -1, np.int64),
          "new": np.full((T1, n, 2 * S), -1, np.int64), "old": np.full((T1, n, K + S), -1, np.int64)}
    ini = None
    if init_idx is not None:
        ini_arr = np.ascontiguousarray(np.asarray(init_idx, dtype=np.int64))
        if ini_arr.shape != (n, K):
            raise ValueError("init_idx must be n x K")
        ini = ini_arr.ctypes.data_as(C.c_void_p)
    rc = _load().oracle_nndescent_traced(X, n, d, d, K, max_iters, float(rho), float(delta),
                                         int(seed) & ((1 << 64) - 1), ini, idx, d2, C.byref(iters), upd,
                                         T, tr["lidx"], tr["lflag"], tr["newf"], tr["oldf"],
                                         tr["new"], tr["old"])
    if rc != 0:
        raise ValueError("oracle_nndescent: bad arguments")
    tr = {key: val[:min(T, iters.value)] for key, val in tr.items()}
    return idx, d2, iters.value, upd[:iters.value].copy(), tr


def round_bf16(a) -> np.ndarray:
    """FP32 -> BF16 (RNE) bit patterns as uint16."""
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    out = np.empty(a.shape, dtype=np.uint16)
    _load().oracle_round_bf16(a.ravel(), out.ravel(), a.size)
    return out


def bf16_to_f64(bits) -> np.ndarray:
    b = np.asarray(bits, dtype=np.uint16).astype(np.uint32) << 16
    return b.view(np.float32).astype(np.float64)


def mlp_forward(X, W1, b1, W2, b2, want_hidden: bool = False):
    X, W1, b1, W2, b2 = map(_f64, (X, W1, b1, W2, b2))
    m, d = X.shape
    h1, h2 = W1.shape[1], W2.shape[1]
    Z = np.empty((m, h2))
    H = np.empty((m, h1)) if want_hidden else None
    _load().oracle_mlp_forward(X, m, d, d, W1, b1, h1, W2, b2, h2,
                               H.ctypes.data_as(C.c_void_p) if H is not None else None, Z)
    return (Z, H) if want_hidden else Z


def bf16_values(a) -> np.ndarray:
    """a rounded FP32 -> BF16 (RNE), as float64 values."""
    return bf16_to_f64(round_bf16(a))


def mlp_forward_bf16(X, W1, b1, W2, b2, want_hidden: bool = False):
    """The encoder's BF16 mode: every factor of a product is rounded to BF16
    (x, W1, the post-ReLU hidden values, W2), the sums are exact (FP64) and
    the biases are not rounded.  Returns Z (and the rounded hidden layer)."""
    Xr, W1r, W2r = bf16_values(X), bf16_values(W1), bf16_values(W2)
    b2 = _f64(b2)
    _, H = mlp_forward(Xr, W1r, b1, W2r, np.zeros_like(b2), want_hidden=True)
    Hr = bf16_values(H)
    Z = Hr @ W2r + b2
    return (Z, Hr) if want_hidden else Z


def mlp_backward_bf16(X, W1, b1, W2, dZ):
    """Gradients of the BF16 mode: dH = round(dZ) round(W2)^T masked by the
    hidden layer's sign; gW1 = round(X)^T round(dH), gW2 = round(H)^T round(dZ)
    with H the rounded hidden layer; gb1, gb2 are plain sums of dH, dZ."""
    Xr, W2r = bf16_values(X), bf16_values(W2)
    _, Hr = mlp_forward_bf16(X, W1, b1, W2, np.zeros(W2.shape[1]), want_hidden=True)
    dZ = _f64(dZ)
    dZr = bf16_values(dZ)
    dH = (dZr @ W2r.T) * (Hr > 0)
    return Xr.T @ bf16_values(dH), dH.sum(axis=0), Hr.T @ dZr, dZ.sum(axis=0)


def triplet_loss(Z, B: int, margin: float = 1.0, want_grad: bool = True):
    Z = _f64(Z)
    dZ = np.zeros_like(Z) if want_grad else None
    loss = _load().oracle_triplet_loss(Z, B, Z.shape[1], float(margin),
                                       dZ.ctypes.data_as(C.c_void_p) if dZ is not None else None)
    return (loss, dZ) if want_grad else loss


def mlp_backward(X, W1, b1, W2, dZ):
    X, W1, b1, W2, dZ = map(_f64, (X, W1, b1, W2, dZ))
    m, d = X.shape
    h1, h2 = W1.shape[1], W2.shape[1]
    gW1, gb1 = np.empty((d, h1)), np.empty(h1)
    gW2, gb2 = np.empty((h1, h2)), np.empty(h2)
    _load().oracle_mlp_backward(X, m, d, d, W1, b1, h1, W2, h2, dZ, gW1, gb1, gW2, gb2)
    return gW1, gb1, gW2, gb2


def adam_step(w, g, m, v, t: int, lr: float = 1e-3, beta1: float = 0.9,
              beta2: float = 0.999, eps: float = 1e-8):
    """In-place Adam step on fp64 arrays w, m, v given gradient g."""
    for a in (w, m, v):
        if a.dtype != np.float64 or not a.flags.c_contiguous:
            raise ValueError("w, m, v must be C-contiguous float64")
    g = _f64(g)
    _load().oracle_adam_step(w.reshape(-1), g.reshape(-1), m.reshape(-1), v.reshape(-1),
                             w.size, lr, beta1, beta2, eps, int(t))


def proj_seed(X, Z, dirs, w: int, K: int, D: int = 1):
    """Sorted-projection seed lists: (idx n x K with -1 pads, squared dist).

    Z and dirs are taken as FP32 (the projections decide an order, so they are
    computed in the kernel's precision); dirs has P*D rows, D per curve.
    """
    X = _f64(X)
    Z = np.ascontiguousarray(np.asarray(Z, dtype=np.float32))
    dirs = np.ascontiguousarray(np.asarray(dirs, dtype=np.float32))
    n, d = X.shape
    if dirs.shape[0] % D:
        raise ValueError("dirs must hold P*D rows")
    P = dirs.shape[0] // D
    idx = np.empty((n, K), dtype=np.int64)
    d2 = np.empty((n, K), dtype=np.float64)
    rc = _load().oracle_proj_seed(X, n, d, d, Z, Z.shape[1], dirs, P, D, w, K, idx, d2)
    if rc != 0:
        raise ValueError("oracle_proj_seed: bad arguments")
    return idx, d2


def proj_keys(Z, dirs, D: int = 1) -> np.ndarray:
    """Order keys of one curve (dirs: D x m): ordered projection or Z-order code."""
    Z = np.ascontiguousarray(np.asarray(Z, dtype=np.float32))
    dirs = np.ascontiguousarray(np.asarray(dirs, dtype=np.float32))
    n = Z.shape[0]
    keys = np.empty(n, dtype=np.uint32)
    y = np.empty(n * D, dtype=np.float32)
    if _load().oracle_proj_keys(Z, n, Z.shape[1], dirs, D, keys, y) != 0:
        raise ValueError("oracle_proj_keys: bad D")
    return keys


def fuzzy_rows(dist):
    """Per-row UMAP membership strengths of a k-NN graph's edges.

    dist: n x k Euclidean neighbour distances (self excluded).  Returns
    (rho n, sigma n, w n x k) in fp64 (see oracle_fuzzy_rows)."""
    d = _f64(dist)
    n, k = d.shape
    rho, sigma, w = np.empty(n), np.empty(n), np.empty((n, k))
    _load().oracle_fuzzy_rows(d, n, k, rho, sigma, w)
    return rho, sigma, w


def fuzzy_union(idx, w, rows=None):
    """Fuzzy union W = A + A^T - A o A^T of the directed memberships A
    (A[i, idx[i, r]] = w[i, r]), as sorted rows: for each requested row i a
    list of (column, value) pairs sorted by column.  The row's columns are
    its k neighbours and every j that lists i.  Rows default to all."""
    idx = np.asarray(idx, dtype=np.int64)
    w = np.asarray(w, dtype=np.float64)
    n, k = idx.shape
    rows = range(n) if rows is None else rows
    # who lists whom: edge numbers grouped by target
    flat = idx.ravel()
    order = np.argsort(flat, kind="stable")
    tgt = flat[order]
    out = []
    for i in rows:
        a = {}
        for r in range(k):
            a[int(idx[i, r])] = float(w[i, r])
        # reverse edges j -> i
        lo, hi = np.searchsorted(tgt, i, "left"), np.searchsorted(tgt, i, "right")
        b = {int(e // k): float(w[e // k, e % k]) for e in order[lo:hi]}
        cols = sorted(set(a) | set(b))
        out.append([(j, a.get(j, 0.0) + b.get(j, 0.0) - a.get(j, 0.0) * b.get(j, 0.0)) for j in cols])
    return out


def quality_rows(X, Y, k: int, rows=None, canonical: bool = False):
    """Per-row terms (hits, trust, cont) of k-NN preservation,
    trustworthiness and continuity for the requested rows (default all);
    canonical=True ranks by the canonical FP32 distance instead of FP64."""
    X, Y = _f64(X), _f64(Y)
    n = X.shape[0]
    rows = np.arange(n, dtype=np.int64) if rows is None else np.ascontiguousarray(np.asarray(rows, np.int64))
    h, t, c = (np.empty(len(rows), np.int64) for _ in range(3))
    if _load().oracle_quality_rows(X, X.shape[1], Y, Y.shape[1], n, k, rows, len(rows), int(canonical),
                                   h, t, c) != 0:
        raise ValueError("oracle_quality_rows: bad arguments")
    return h, t, c


def quality(X, Y, k: int, canonical: bool = False):
    """(k-NN preservation, trustworthiness, continuity) over all rows:
    P = sum hits / (n k); T = 1 - 2 / (n k (2n - 3k - 1)) sum trust;
    C likewise with cont."""
    n = np.asarray(X).shape[0]
    h, t, c = quality_rows(X, Y, k, canonical=canonical)
    z = 2.0 / (n * k * (2.0 * n - 3.0 * k - 1.0))
    return float(h.sum()) / (n * k), 1.0 - z * float(t.sum()), 1.0 - z * float(c.sum())


def pca(X, p: int):
    """Principal components of the rows of X (the paper's PCA preprocessing
    to pca_dim, section "Scaling Behavior"): mean mu, covariance
    C = (X - mu)^T (X - mu) / (n - 1) in FP64, its eigenpairs by
    numpy.linalg.eigh, the p largest eigenvalues in descending order with
    their eigenvectors, each eigenvector's sign fixed so that its entry of
    largest magnitude (the first such) is positive, and the projection
    Z = (X - mu) V.  Returns (Z n x p, V d x p, eigenvalues p, mu d)."""
    X = _f64(X)
    n = X.shape[0]
    mu = X.mean(axis=0)
    Xc = X - mu
    C = (Xc.T @ Xc) / (n - 1)
    w, V = np.linalg.eigh(C)
    order = np.argsort(-w, kind="stable")[:p]
    w, V = w[order], V[:, order]
    piv = np.argmax(np.abs(V), axis=0)
    V = V * np.sign(V[piv, np.arange(V.shape[1])])
    return Xc @ V, V, w, mu
