"""ctypes binding of libknn.so (argument marshalling only).

Every computation runs in the HIP library; this module allocates output
tensors with torch, passes device pointers and the current HIP stream, and
turns status codes into exceptions.  Importing it on a machine where
libknn.so is missing raises immediately: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libknn.so")

KNN_OK, KNN_EINVAL, KNN_ENOMEM, KNN_EDEVICE, KNN_ENOTSUP = 0, -1, -2, -3, -4
KNN_F32, KNN_BF16, KNN_F16 = 0, 1, 2
KNN_PREC_FP32, KNN_PREC_BF16, KNN_PREC_FP16 = 0, 1, 2
KNN_OUT_L2, KNN_OUT_SQL2 = 0, 1
KNN_INIT_RANDOM, KNN_INIT_ENCODER = 0, 1
KNN_MAX_K = 32
ENC_H1, ENC_H2 = 64, 32
MAX_ITERS_LOGGED = 64

_DTYPES = {torch.float32: KNN_F32, torch.bfloat16: KNN_BF16, torch.float16: KNN_F16}
_PREC = {"fp32": KNN_PREC_FP32, "bf16": KNN_PREC_BF16, "fp16": KNN_PREC_FP16}
_OUT = {"l2": KNN_OUT_L2, "sql2": KNN_OUT_SQL2}


class KnnError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_status_name(status)}: {msg}")
        self.status = status


class knn_matrix(C.Structure):
    _fields_ = [("data", C.c_void_p), ("n", C.c_int64), ("d", C.c_int32),
                ("ld", C.c_int64), ("dtype", C.c_int32)]


class knn_nnd_params(C.Structure):
    _fields_ = [("k", C.c_int32), ("build_k", C.c_int32), ("max_iters", C.c_int32),
                ("sample_rate", C.c_float), ("delta", C.c_float), ("seed", C.c_uint64),
                ("precision", C.c_int32), ("out_kind", C.c_int32), ("init_kind", C.c_int32),
                ("encoder", C.c_void_p), ("proj_count", C.c_int32), ("proj_window", C.c_int32),
                ("proj_dims", C.c_int32),
                ("cand_slots", C.c_int32), ("join_cap", C.c_int32),
                ("workspace_limit_bytes", C.c_int64), ("rev_slots", C.c_int32), ("ensemble", C.c_int32)]


class knn_nnd_stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("build_k", C.c_int32),
                ("updates", C.c_int64 * MAX_ITERS_LOGGED), ("emitted", C.c_int64 * MAX_ITERS_LOGGED),
                ("bytes_gathered", C.c_uint64),
                ("ms_total", C.c_double), ("ms_init", C.c_double), ("ms_sample", C.c_double),
                ("ms_join", C.c_double), ("ms_merge", C.c_double), ("ms_final", C.c_double),
                ("ms_join_iter", C.c_float * MAX_ITERS_LOGGED),
                ("slot_collisions", C.c_int64 * MAX_ITERS_LOGGED),
                ("list_dropped", C.c_int64 * MAX_ITERS_LOGGED),
                ("pairs_joined", C.c_uint64)]

    def as_dict(self) -> dict:
        it = self.iters
        return {"iters": it, "build_k": self.build_k,
                "updates": list(self.updates[:min(it, MAX_ITERS_LOGGED)]),
                "emitted": list(self.emitted[:min(it, MAX_ITERS_LOGGED)]),
                "bytes_gathered": int(self.bytes_gathered),
                "ms_total": self.ms_total, "ms_init": self.ms_init, "ms_sample": self.ms_sample,
                "ms_join": self.ms_join, "ms_merge": self.ms_merge, "ms_final": self.ms_final,
                "ms_join_iter": [round(x, 4) for x in self.ms_join_iter[:min(it, MAX_ITERS_LOGGED)]],
                "slot_collisions": list(self.slot_collisions[:min(it, MAX_ITERS_LOGGED)]),
                "list_dropped": list(self.list_dropped[:min(it, MAX_ITERS_LOGGED)]),
                "pairs_joined": int(self.pairs_joined)}


class knn_train_params(C.Structure):
    _fields_ = [("steps", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float),
                ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("margin", C.c_float), ("seed", C.c_uint64), ("precision", C.c_int32)]


EXPORTS = [
    "knn_status_str", "knn_last_error", "knn_exact", "knn_exact_query",
    "knn_nnd_default_params", "nndescent_build", "nndescent_refine",
    "knn_encoder_create", "knn_encoder_destroy", "knn_encoder_set_weights",
    "knn_encoder_get_weights", "knn_encoder_embed", "knn_encoder_grads",
    "knn_train_default_params", "knn_encoder_train", "knn_proj_seed",
    "knn_encoder_triplets", "knn_encoder_step", "knn_encoder_get_adam",
    "knn_exact_query_limited", "knn_exact_noalloc", "knn_fuzzy_graph", "knn_quality", "knn_pca",
]
NOALLOC_SCRATCH_BYTES = 64 << 20

_lib = None


def load() -> C.CDLL:
    """Load libknn.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2603_04035_amd.build.build()")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, f32, u64 = C.c_void_p, C.c_int32, C.c_int64, C.c_float, C.c_uint64
    lib.knn_status_str.restype = C.c_char_p
    lib.knn_status_str.argtypes = [i32]
    lib.knn_last_error.restype = C.c_char_p
    lib.knn_last_error.argtypes = []
    lib.knn_exact.restype = i32
    lib.knn_exact.argtypes = [knn_matrix, i32, i32, i32, i32, vp, vp, vp]
    lib.knn_exact_query.restype = i32
    lib.knn_exact_query.argtypes = [knn_matrix, knn_matrix, vp, i32, i32, i32, i32, vp, vp, vp]
    lib.knn_exact_query_limited.restype = i32
    lib.knn_exact_query_limited.argtypes = [knn_matrix, knn_matrix, vp, i32, i32, i32, i32, i64, vp, vp, vp]
    lib.knn_exact_noalloc.restype = i32
    lib.knn_exact_noalloc.argtypes = [knn_matrix, i32, i32, i32, i32, vp, vp, vp]
    lib.knn_pca.restype = i32
    lib.knn_pca.argtypes = [knn_matrix, i32, i32, vp, vp, vp, vp, vp]
    lib.knn_quality.restype = i32
    lib.knn_quality.argtypes = [knn_matrix, knn_matrix, i32, vp, vp, vp, C.POINTER(C.c_double), vp]
    lib.knn_fuzzy_graph.restype = i32
    lib.knn_fuzzy_graph.argtypes = [vp, vp, i64, i32, vp, vp, vp, vp, vp, vp, C.POINTER(C.c_int64), vp]
    lib.knn_nnd_default_params.restype = None
    lib.knn_nnd_default_params.argtypes = [i32, C.POINTER(knn_nnd_params)]
    lib.nndescent_build.restype = i32
    lib.nndescent_build.argtypes = [knn_matrix, C.POINTER(knn_nnd_params), vp, vp, vp, vp, vp,
                                    C.POINTER(knn_nnd_stats), vp]
    lib.nndescent_refine.restype = i32
    lib.nndescent_refine.argtypes = [knn_matrix, C.POINTER(knn_nnd_params), vp, vp, vp, i32, i32,
                                     vp, vp, vp, vp, vp, C.POINTER(knn_nnd_stats), vp]
    lib.knn_encoder_create.restype = i32
    lib.knn_encoder_create.argtypes = [i32, u64, C.POINTER(vp)]
    lib.knn_encoder_destroy.restype = None
    lib.knn_encoder_destroy.argtypes = [vp]
    lib.knn_encoder_set_weights.restype = i32
    lib.knn_encoder_set_weights.argtypes = [vp, vp, vp, vp, vp]
    lib.knn_encoder_get_weights.restype = i32
    lib.knn_encoder_get_weights.argtypes = [vp, vp, vp, vp, vp]
    lib.knn_encoder_embed.restype = i32
    lib.knn_encoder_embed.argtypes = [vp, knn_matrix, i32, vp, vp]
    lib.knn_encoder_grads.restype = i32
    lib.knn_encoder_grads.argtypes = [vp, knn_matrix, vp, i32, f32, i32, C.POINTER(C.c_float), vp, vp]
    lib.knn_train_default_params.restype = None
    lib.knn_train_default_params.argtypes = [C.POINTER(knn_train_params)]
    lib.knn_encoder_train.restype = i32
    lib.knn_encoder_train.argtypes = [vp, knn_matrix, vp, i32, C.POINTER(knn_train_params), vp, vp]
    lib.knn_encoder_triplets.restype = i32
    lib.knn_encoder_triplets.argtypes = [i64, vp, i32, i32, u64, i32, vp, vp]
    lib.knn_encoder_step.restype = i32
    lib.knn_encoder_step.argtypes = [vp, knn_matrix, vp, i32, C.POINTER(knn_train_params),
                                     C.POINTER(C.c_float), vp]
    lib.knn_encoder_get_adam.restype = i32
    lib.knn_encoder_get_adam.argtypes = [vp, vp, vp, C.POINTER(C.c_int32)]
    lib.knn_proj_seed.restype = i32
    lib.knn_proj_seed.argtypes = [knn_matrix, vp, i32, vp, i32, i32, i32, i32, vp, vp, vp]
    _lib = lib
    return lib


def _status_name(s: int) -> str:
    try:
        return load().knn_status_str(s).decode()
    except Exception:
        return str(s)


def _check(status: int):
    if status != KNN_OK:
        raise KnnError(status, load().knn_last_error().decode())


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _ptr(t):
    return None if t is None else t.data_ptr()


def matrix(X: torch.Tensor) -> knn_matrix:
    """Describe a 2-D CUDA tensor (rows may be strided, elements contiguous)."""
    if X.dim() != 2:
        raise ValueError("expected a 2-D tensor")
    if not X.is_cuda:
        raise ValueError("expected a device tensor")
    if X.dtype not in _DTYPES:
        raise ValueError(f"unsupported dtype {X.dtype}")
    if X.stride(1) != 1:
        raise ValueError("rows must be contiguous")
    return knn_matrix(X.data_ptr(), X.shape[0], X.shape[1], X.stride(0), _DTYPES[X.dtype])


def knn_exact(X: torch.Tensor, k: int, precision: str = "fp32", rerank_k: int = 0,
              out: str = "l2"):
    """Exact kNN of the rows of X among themselves -> (idx int32 n x k, dist f32 n x k)."""
    lib = load()
    n = X.shape[0]
    idx = torch.empty((n, k), dtype=torch.int32, device=X.device)
    dist = torch.empty((n, k), dtype=torch.float32, device=X.device)
    _check(lib.knn_exact(matrix(X), k, _PREC[precision], rerank_k, _OUT[out],
                         idx.data_ptr(), dist.data_ptr(), _stream()))
    return idx, dist


def knn_exact_noalloc(X: torch.Tensor, k: int, precision: str = "fp32", rerank_k: int = 0,
                      out: str = "l2", out_idx: torch.Tensor | None = None,
                      out_dist: torch.Tensor | None = None):
    """knn_exact working in the library's static device array (no device
    allocation inside the call); outputs may be passed in preallocated."""
    lib = load()
    n = X.shape[0]
    idx = out_idx if out_idx is not None else torch.empty((n, k), dtype=torch.int32, device=X.device)
    dist = out_dist if out_dist is not None else torch.empty((n, k), dtype=torch.float32, device=X.device)
    if idx.shape != (n, k) or dist.shape != (n, k) or not idx.is_contiguous() or not dist.is_contiguous():
        raise ValueError("outputs must be contiguous n x k")
    _check(lib.knn_exact_noalloc(matrix(X), k, _PREC[precision], rerank_k, _OUT[out],
                                 idx.data_ptr(), dist.data_ptr(), _stream()))
    return idx, dist


def knn_exact_query(Q: torch.Tensor, R: torch.Tensor, k: int, q_self=None,
                    precision: str = "fp32", rerank_k: int = 0, out: str = "l2",
                    workspace_limit: int = 0):
    """Exact kNN of the rows of Q among the rows of R (q_self: rows to exclude).

    workspace_limit > 0 bounds the call's scratch bytes (queries are then
    processed in chunks, each a pass over R)."""
    lib = load()
    nq = Q.shape[0]
    idx = torch.empty((nq, k), dtype=torch.int32, device=Q.device)
    dist = torch.empty((nq, k), dtype=torch.float32, device=Q.device)
    qs = None
    if q_self is not None:
        qs = torch.as_tensor(q_self, dtype=torch.int32, device=Q.device).contiguous()
    if workspace_limit:
        _check(lib.knn_exact_query_limited(matrix(Q), matrix(R), _ptr(qs), k, _PREC[precision], rerank_k,
                                           _OUT[out], int(workspace_limit), idx.data_ptr(), dist.data_ptr(),
                                           _stream()))
    else:
        _check(lib.knn_exact_query(matrix(Q), matrix(R), _ptr(qs), k, _PREC[precision], rerank_k,
                                   _OUT[out], idx.data_ptr(), dist.data_ptr(), _stream()))
    return idx, dist


def nnd_params(k: int, **kw) -> knn_nnd_params:
    p = knn_nnd_params()
    load().knn_nnd_default_params(k, C.byref(p))
    for key, val in kw.items():
        if key == "precision":
            val = _PREC[val] if isinstance(val, str) else val
        elif key == "out_kind":
            val = _OUT[val] if isinstance(val, str) else val
        elif key == "init_kind":
            val = {"random": KNN_INIT_RANDOM, "encoder": KNN_INIT_ENCODER}.get(val, val)
        elif key == "encoder":
            val = val.handle if val is not None else None
        if not hasattr(p, key):
            raise TypeError(f"unknown NNDescent parameter {key}")
        setattr(p, key, val)
    return p


def _state_tensors(n, K, device, want):
    if not want:
        return None, None, None
    return (torch.empty((n, K), dtype=torch.int32, device=device),
            torch.empty((n, K), dtype=torch.float32, device=device),
            torch.empty((n, K), dtype=torch.uint8, device=device))


def _build_k(p: knn_nnd_params, n: int) -> int:
    K = p.build_k
    if K == 0:
        K = min(2 * p.k, KNN_MAX_K) if p.precision != KNN_PREC_FP32 else p.k
    return min(K, n - 1)


def nndescent_build(X: torch.Tensor, k: int, return_state: bool = False, **kw):
    """NNDescent graph -> (idx, dist, stats dict[, (state_idx, state_d2, state_flags)])."""
    lib = load()
    p = nnd_params(k, **kw)
    n = X.shape[0]
    idx = torch.empty((n, k), dtype=torch.int32, device=X.device)
    dist = torch.empty((n, k), dtype=torch.float32, device=X.device)
    si, sd, sf = _state_tensors(n, _build_k(p, n), X.device, return_state)
    st = knn_nnd_stats()
    _check(lib.nndescent_build(matrix(X), C.byref(p), idx.data_ptr(), dist.data_ptr(),
                               _ptr(si), _ptr(sd), _ptr(sf), C.byref(st), _stream()))
    if return_state:
        return idx, dist, st.as_dict(), (si, sd, sf)
    return idx, dist, st.as_dict()


def nndescent_refine(X: torch.Tensor, k: int, init_idx: torch.Tensor, init_dist=None,
                     init_flags=None, iter_offset: int = 0, return_state: bool = False, **kw):
    """Continue NNDescent from given lists (init_idx: n x init_k int32)."""
    lib = load()
    p = nnd_params(k, **kw)
    n = X.shape[0]
    init_idx = init_idx.to(torch.int32).contiguous()
    if init_dist is not None:
        init_dist = init_dist.to(torch.float32).contiguous()
    if init_flags is not None:
        init_flags = init_flags.to(torch.uint8).contiguous()
    idx = torch.empty((n, k), dtype=torch.int32, device=X.device)
    dist = torch.empty((n, k), dtype=torch.float32, device=X.device)
    si, sd, sf = _state_tensors(n, _build_k(p, n), X.device, return_state)
    st = knn_nnd_stats()
    _check(lib.nndescent_refine(matrix(X), C.byref(p), init_idx.data_ptr(), _ptr(init_dist),
                                _ptr(init_flags), init_idx.shape[1], iter_offset,
                                idx.data_ptr(), dist.data_ptr(), _ptr(si), _ptr(sd), _ptr(sf),
                                C.byref(st), _stream()))
    if return_state:
        return idx, dist, st.as_dict(), (si, sd, sf)
    return idx, dist, st.as_dict()


def fuzzy_graph(idx: torch.Tensor, dist: torch.Tensor):
    """UMAP membership strengths and fuzzy union of a k-NN graph.

    Returns (rho n, sigma n, weights n x k, row_ptr n+1 int64, col int32,
    val float32) with col / val cut to the nonzero count."""
    lib = load()
    idx = idx.to(torch.int32).contiguous()
    dist = dist.to(torch.float32).contiguous()
    n, k = idx.shape
    dev = idx.device
    rho = torch.empty(n, dtype=torch.float32, device=dev)
    sigma = torch.empty(n, dtype=torch.float32, device=dev)
    w = torch.empty((n, k), dtype=torch.float32, device=dev)
    row_ptr = torch.empty(n + 1, dtype=torch.int64, device=dev)
    col = torch.empty(2 * n * k, dtype=torch.int32, device=dev)
    val = torch.empty(2 * n * k, dtype=torch.float32, device=dev)
    nnz = C.c_int64()
    _check(lib.knn_fuzzy_graph(idx.data_ptr(), dist.data_ptr(), n, k, rho.data_ptr(), sigma.data_ptr(),
                               w.data_ptr(), row_ptr.data_ptr(), col.data_ptr(), val.data_ptr(),
                               C.byref(nnz), _stream()))
    return rho, sigma, w, row_ptr, col[:nnz.value], val[:nnz.value]


def quality(X: torch.Tensor, Y: torch.Tensor, k: int = 10, per_row: bool = False):
    """(k-NN preservation, trustworthiness, continuity) of embedding Y of X;
    with per_row also the per-row terms (hits, trust, cont) as tensors."""
    lib = load()
    n = X.shape[0]
    m = (C.c_double * 3)()
    h = t = c = None
    if per_row:
        h = torch.empty(n, dtype=torch.int32, device=X.device)
        t = torch.empty(n, dtype=torch.int64, device=X.device)
        c = torch.empty(n, dtype=torch.int64, device=X.device)
    _check(lib.knn_quality(matrix(X), matrix(Y), k, _ptr(h), _ptr(t), _ptr(c), m, _stream()))
    out = (m[0], m[1], m[2])
    return (out, (h, t, c)) if per_row else out


def pca(X: torch.Tensor, p: int, iters: int = 0):
    """PCA of the rows of X: (Z n x p float32, components d x p float64,
    eigenvalues p float64, mean d float64)."""
    lib = load()
    n, d = X.shape
    dev = X.device
    Z = torch.empty((n, p), dtype=torch.float32, device=dev)
    V = torch.empty((d, p), dtype=torch.float64, device=dev)
    w = torch.empty(p, dtype=torch.float64, device=dev)
    mu = torch.empty(d, dtype=torch.float64, device=dev)
    _check(lib.knn_pca(matrix(X), p, iters, Z.data_ptr(), V.data_ptr(), w.data_ptr(), mu.data_ptr(), _stream()))
    return Z, V, w, mu
