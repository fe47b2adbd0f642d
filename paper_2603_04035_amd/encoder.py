"""Binding of the learned-seeding entry points (argument marshalling only)."""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import ENC_H1, ENC_H2, _check, _stream, load, matrix


class Encoder:
    """MLP encoder d -> 64 -> 32 living on the current device (knn_encoder)."""

    def __init__(self, d: int, seed: int = 0):
        self._lib = load()
        h = C.c_void_p()
        _check(self._lib.knn_encoder_create(d, seed, C.byref(h)))
        self.handle = h.value
        self.d = d

    def close(self):
        if getattr(self, "handle", None):
            self._lib.knn_encoder_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def n_params(self) -> int:
        return self.d * ENC_H1 + ENC_H1 + ENC_H1 * ENC_H2 + ENC_H2

    def get_weights(self):
        W1 = np.empty((self.d, ENC_H1), np.float32)
        b1 = np.empty(ENC_H1, np.float32)
        W2 = np.empty((ENC_H1, ENC_H2), np.float32)
        b2 = np.empty(ENC_H2, np.float32)
        _check(self._lib.knn_encoder_get_weights(self.handle, W1.ctypes.data, b1.ctypes.data,
                                                 W2.ctypes.data, b2.ctypes.data))
        return W1, b1, W2, b2

    def set_weights(self, W1, b1, W2, b2):
        arrs = [np.ascontiguousarray(np.asarray(a, np.float32)) for a in (W1, b1, W2, b2)]
        if arrs[0].shape != (self.d, ENC_H1) or arrs[2].shape != (ENC_H1, ENC_H2):
            raise ValueError("weight shapes")
        _check(self._lib.knn_encoder_set_weights(self.handle, *[a.ctypes.data for a in arrs]))

    def embed(self, X: torch.Tensor, precision: str = "fp32") -> torch.Tensor:
        Z = torch.empty((X.shape[0], ENC_H2), dtype=torch.float32, device=X.device)
        _check(self._lib.knn_encoder_embed(self.handle, matrix(X), _lib._PREC[precision],
                                           Z.data_ptr(), _stream()))
        return Z

    def grads(self, X: torch.Tensor, rows: torch.Tensor, B: int, margin: float = 1.0,
              precision: str = "fp32"):
        """Loss and flat gradient (gW1, gb1, gW2, gb2) of one triplet batch."""
        rows = rows.to(device=X.device, dtype=torch.int32).contiguous()
        if rows.numel() != 3 * B:
            raise ValueError("rows must hold 3B entries")
        g = torch.empty(self.n_params, dtype=torch.float32, device=X.device)
        loss = C.c_float()
        _check(self._lib.knn_encoder_grads(self.handle, matrix(X), rows.data_ptr(), B, margin,
                                           _lib._PREC[precision], C.byref(loss), g.data_ptr(), _stream()))
        return loss.value, g

    @staticmethod
    def _train_params(steps, batch, lr, margin, seed, precision):
        t = _lib.knn_train_params()
        load().knn_train_default_params(C.byref(t))
        t.steps, t.batch, t.lr, t.margin, t.seed = steps, batch, lr, margin, seed
        t.precision = _lib._PREC[precision]
        return t

    def adam_state(self):
        """(first moments, second moments, steps taken) as flat float32 arrays."""
        m = np.empty(self.n_params, np.float32)
        v = np.empty(self.n_params, np.float32)
        t = C.c_int32()
        _check(self._lib.knn_encoder_get_adam(self.handle, m.ctypes.data, v.ctypes.data, C.byref(t)))
        return m, v, t.value

    def step(self, X: torch.Tensor, rows: torch.Tensor, B: int, lr: float = 1e-3, margin: float = 1.0,
             precision: str = "fp32") -> float:
        """One Adam step on the given triplet rows (3B); returns the batch loss."""
        rows = rows.to(device=X.device, dtype=torch.int32).contiguous()
        if rows.numel() != 3 * B:
            raise ValueError("rows must hold 3B entries")
        t = self._train_params(1, B, lr, margin, 0, precision)
        loss = C.c_float()
        _check(self._lib.knn_encoder_step(self.handle, matrix(X), rows.data_ptr(), B, C.byref(t),
                                          C.byref(loss), _stream()))
        return loss.value

    def train(self, X: torch.Tensor, knn_idx: torch.Tensor, steps: int = 2000, batch: int = 4096,
              lr: float = 1e-3, margin: float = 1.0, seed: int = 0, precision: str = "fp32") -> np.ndarray:
        t = self._train_params(steps, batch, lr, margin, seed, precision)
        knn_idx = knn_idx.to(torch.int32).contiguous()
        log = np.zeros(max(steps, 1), np.float32)
        _check(self._lib.knn_encoder_train(self.handle, matrix(X), knn_idx.data_ptr(), knn_idx.shape[1],
                                           C.byref(t), log.ctypes.data, _stream()))
        return log[:steps]


def triplets(knn_idx: torch.Tensor, B: int, seed: int, step: int) -> torch.Tensor:
    """The 3B triplet rows that training step `step` draws from the graph knn_idx."""
    knn_idx = knn_idx.to(torch.int32).contiguous()
    rows = torch.empty(3 * B, dtype=torch.int32, device=knn_idx.device)
    _check(load().knn_encoder_triplets(knn_idx.shape[0], knn_idx.data_ptr(), knn_idx.shape[1], B, seed, step,
                                       rows.data_ptr(), _stream()))
    return rows


def knn_proj_seed(X: torch.Tensor, Z: torch.Tensor, dirs: torch.Tensor, w: int, K: int, D: int = 1):
    """Seed lists from sorted projections: (idx int32 n x K, squared dist n x K).

    dirs holds P*D rows; order p sorts by the Z-order code of its D projections
    (D = 1: the projection itself).
    """
    lib = load()
    Z = Z.to(torch.float32).contiguous()
    dirs = dirs.to(device=X.device, dtype=torch.float32).contiguous()
    if dirs.shape[0] % D:
        raise ValueError("dirs must hold P*D rows")
    n = X.shape[0]
    idx = torch.empty((n, K), dtype=torch.int32, device=X.device)
    d2 = torch.empty((n, K), dtype=torch.float32, device=X.device)
    _check(lib.knn_proj_seed(matrix(X), Z.data_ptr(), Z.shape[1], dirs.data_ptr(), dirs.shape[0] // D, D,
                             w, K, idx.data_ptr(), d2.data_ptr(), _stream()))
    return idx, d2
