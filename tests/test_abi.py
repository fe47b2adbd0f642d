"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/knn.h, and rejects bad arguments before touching the
device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "knn.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([a-z_][a-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_2603_04035_amd import _lib
    return _lib.load()


def test_header_declares_the_boundary():
    names = _declared()
    for fn in ("knn_exact", "knn_exact_query", "nndescent_build", "nndescent_refine"):
        assert fn in names
    assert len(names) >= 16


def test_every_declared_symbol_is_exported(lib):
    from paper_2603_04035_amd import _lib
    names = _declared()
    for fn in names:
        assert hasattr(lib, fn), fn
    assert sorted(_lib.EXPORTS) == names


def test_status_strings(lib):
    assert lib.knn_status_str(0) == b"KNN_OK"
    assert lib.knn_status_str(-1) == b"KNN_EINVAL"
    assert lib.knn_status_str(-4) == b"KNN_ENOTSUP"


def test_default_params(lib):
    from paper_2603_04035_amd import _lib
    p = _lib.knn_nnd_params()
    lib.knn_nnd_default_params(15, C.byref(p))
    assert p.k == 15 and p.max_iters == 20 and p.build_k == 0
    assert abs(p.sample_rate - 0.5) < 1e-7 and abs(p.delta - 0.015) < 1e-7
    t = _lib.knn_train_params()
    lib.knn_train_default_params(C.byref(t))
    assert t.steps > 0 and t.batch > 0 and t.lr > 0


def _fake(n=100, d=8, dtype=0, ld=None):
    from paper_2603_04035_amd import _lib
    # a non-null pointer that is never dereferenced: every call below fails validation first
    return _lib.knn_matrix(0x1000, n, d, d if ld is None else ld, dtype)


@pytest.mark.parametrize("case", ["null", "n1", "d0", "ld", "dtype", "k0", "kbig", "prec", "out", "rerank"])
def test_exact_rejects_bad_arguments(lib, case):
    from paper_2603_04035_amd import _lib
    X = _fake()
    k, prec, rer, out = 5, 0, 0, 0
    outp = 0x2000
    if case == "null":
        X.data = None
    elif case == "n1":
        X.n = 1
    elif case == "d0":
        X.d = 0
    elif case == "ld":
        X.ld = 4
    elif case == "dtype":
        X.dtype = 7
    elif case == "k0":
        k = 0
    elif case == "kbig":
        k = 100
    elif case == "prec":
        prec = 9
    elif case == "out":
        out = 9
    elif case == "rerank":
        rer = 3
    rc = lib.knn_exact(X, k, prec, rer, out, outp, outp, None)
    assert rc == _lib.KNN_EINVAL
    assert len(lib.knn_last_error()) > 0


def test_exact_rejects_unsupported_width(lib):
    from paper_2603_04035_amd import _lib
    rc = lib.knn_exact(_fake(), 5, 0, 40, 0, 0x2000, 0x2000, None)
    assert rc == _lib.KNN_ENOTSUP


@pytest.mark.parametrize("field,val", [("k", 0), ("k", 100), ("build_k", 3), ("sample_rate", 0.0),
                                       ("sample_rate", 1.5), ("delta", -1.0), ("max_iters", -1),
                                       ("precision", 5), ("init_kind", 1), ("out_kind", 4)])
def test_nndescent_rejects_bad_params(lib, field, val):
    from paper_2603_04035_amd import _lib
    p = _lib.knn_nnd_params()
    lib.knn_nnd_default_params(5, C.byref(p))
    setattr(p, field, val)
    st = _lib.knn_nnd_stats()
    rc = lib.nndescent_build(_fake(), C.byref(p), 0x2000, 0x2000, None, None, None, C.byref(st), None)
    assert rc == _lib.KNN_EINVAL


def test_nndescent_rejects_wide_lists(lib):
    from paper_2603_04035_amd import _lib
    p = _lib.knn_nnd_params()
    lib.knn_nnd_default_params(5, C.byref(p))
    p.build_k = 40
    rc = lib.nndescent_build(_fake(), C.byref(p), 0x2000, 0x2000, None, None, None, None, None)
    assert rc == _lib.KNN_ENOTSUP


def test_refine_rejects_null_init(lib):
    from paper_2603_04035_amd import _lib
    p = _lib.knn_nnd_params()
    lib.knn_nnd_default_params(5, C.byref(p))
    rc = lib.nndescent_refine(_fake(), C.byref(p), None, None, None, 5, 0, 0x2000, 0x2000,
                              None, None, None, None, None)
    assert rc == _lib.KNN_EINVAL
