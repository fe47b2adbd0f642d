"""MI355X (gfx950) k-nearest-neighbour graph construction.

The compute lives in ``libknn.so`` (hand-written HIP kernels behind a C ABI,
declared in ``include/knn.h``); this package is a thin binding.  Importing
the package does not load the library; the first call does, and raises if it
has not been built (``paper_2603_04035_amd.build.build()``).
"""
from __future__ import annotations

__all__ = ["knn_exact", "knn_exact_query", "knn_exact_noalloc", "nndescent_build", "nndescent_refine",
           "Encoder", "knn_proj_seed", "fuzzy_graph", "quality", "pca", "load"]


def __getattr__(name):
    if name in __all__ or name in ("KnnError", "nnd_params"):
        if name == "Encoder" or name == "knn_proj_seed":
            from . import encoder as _enc
            return getattr(_enc, name)
        from . import _lib
        return getattr(_lib, name)
    raise AttributeError(name)
