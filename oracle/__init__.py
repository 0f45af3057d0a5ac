"""CPU oracle for the all-points minimax path distance -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library
(``paper_2407_07058_amd``) never imports it and shares no code with it.

The arithmetic lives in ``appd_oracle.c`` (plain C, built with gcc without
floating-point contraction); this module only builds it and marshals numpy
arrays.  See the header of ``appd_oracle.c`` for what each function computes and
which passage of arXiv 2407.07058 it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "appd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


_FLAGS = ["-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math", "-Wall"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O3, no FMA contraction) into liboracle.so.
    Portable code: the library also runs on hosts other than the build host."""
    if not force and os.path.exists(_LIB):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.run(["gcc", "-O3", *_FLAGS, "-o", tmp, _SRC, "-lm"], check=True)
    os.replace(tmp, _LIB)
    return _LIB


_SIGS = [
    ("oracle_appd_alg4", ["P", "I64", "P", "P"]),
    ("oracle_appd_alg4_f64", ["P", "I64", "P", "P"]),
    ("oracle_appd_widest", ["P", "I64", "P", "P"]),
    ("oracle_appd_alg4_rows", ["P", "I64", "P", "I64", "I", "P", "P"]),
    ("oracle_mst_prim", ["P", "I64", "I", "P", "P", "P", "P"]),
    ("oracle_linkage", ["P", "I64", "I", "P"]),
    ("oracle_appd_fw", ["P", "I64", "I", "P", "P"]),
    ("oracle_pairwise_euclidean_f32", ["P", "I64", "I64", "P"]),
    ("oracle_pairwise_euclidean_f64", ["P", "I64", "I64", "P"]),
    ("oracle_grad_points", ["P", "I64", "I64", "P", "P", "P", "P"]),
]


def _bind(path):
    lib = ctypes.CDLL(path)
    T = {"P": ctypes.c_void_p, "I64": ctypes.c_int64, "I": ctypes.c_int}
    for name, args in _SIGS:
        f = getattr(lib, name)
        f.argtypes = [T[a] for a in args]
        f.restype = ctypes.c_int
    lib.oracle_loss_f64.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
    lib.oracle_loss_f64.restype = ctypes.c_double
    return lib


def _load():
    global _lib
    if _lib is not None:
        return _lib
    other = os.environ.get("APPD_ORACLE_LIB")  # another build (the sanitizer test's)
    if other:
        _lib = _bind(other)
        return _lib
    if not os.path.exists(_LIB):
        build()
    _lib = _bind(_LIB)
    return _lib


_native = None


def native_build():
    """The oracle compiled for this host with -O3 -march=native (the CPU
    timing reference), built at run time into a temporary directory, since a
    library tuned for one host's instruction set must not travel to another."""
    global _native
    if _native is None:
        import tempfile
        d = tempfile.mkdtemp(prefix="appd_oracle_")
        path = os.path.join(d, "liboracle_native.so")
        subprocess.run(["gcc", "-O3", "-march=native", *_FLAGS, "-o", path, _SRC, "-lm"],
                       check=True)
        _native = _bind(path)
    return _native


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _chk(rc: int, what: str):
    if rc != 0:
        raise RuntimeError("%s failed with code %d" % (what, rc))


def _sq(W, dtype):
    W = np.ascontiguousarray(W, dtype=dtype)
    if W.ndim != 2 or W.shape[0] != W.shape[1]:
        raise ValueError("W must be square")
    return W


def appd(W: np.ndarray, lib=None, out=None):
    """Algorithm 4 on a float32 weight matrix -> (M float32, idx int32).
    lib: a library from native_build() instead of the portable one; out:
    optional (M, idx) arrays to write into."""
    W = _sq(W, np.float32)
    n = W.shape[0]
    if out is None:
        M = np.empty((n, n), np.float32)
        idx = np.empty((n, n), np.int32)
    else:
        M, idx = out
        assert M.shape == (n, n) and M.dtype == np.float32 and M.flags.c_contiguous
        assert idx.shape == (n, n) and idx.dtype == np.int32 and idx.flags.c_contiguous
    _chk((lib or _load()).oracle_appd_alg4(_p(W), n, _p(M), _p(idx)), "oracle_appd_alg4")
    return M, idx


def appd_f64(W: np.ndarray):
    """Algorithm 4 on a float64 weight matrix -> (M float64, idx int32)."""
    W = _sq(W, np.float64)
    n = W.shape[0]
    M = np.empty((n, n), np.float64)
    idx = np.empty((n, n), np.int32)
    _chk(_load().oracle_appd_alg4_f64(_p(W), n, _p(M), _p(idx)), "oracle_appd_alg4_f64")
    return M, idx


def appd_widest(W: np.ndarray):
    """Widest-path variant of Algorithm 4 (maximum spanning tree, ascending removal)."""
    W = _sq(W, np.float32)
    n = W.shape[0]
    M = np.empty((n, n), np.float32)
    idx = np.empty((n, n), np.int32)
    _chk(_load().oracle_appd_widest(_p(W), n, _p(M), _p(idx)), "oracle_appd_widest")
    return M, idx


def appd_rows(W: np.ndarray, rows, widest: bool = False):
    """Algorithm 4, only the given rows: (M[len(rows), n], idx[len(rows), n])."""
    W = _sq(W, np.float32)
    n = W.shape[0]
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    M = np.empty((len(rows), n), np.float32)
    idx = np.empty((len(rows), n), np.int32)
    _chk(_load().oracle_appd_alg4_rows(_p(W), n, _p(rows), len(rows), int(widest), _p(M),
                                       _p(idx)), "oracle_appd_alg4_rows")
    return M, idx


def mst_prim(W: np.ndarray, widest: bool = False):
    """Prim from vertex 0 -> (order, parent, attach_w, attach_f)."""
    W = _sq(W, np.float32)
    n = W.shape[0]
    order = np.empty(n, np.int64)
    parent = np.empty(n, np.int64)
    aw = np.empty(n, np.float32)
    af = np.empty(n, np.int64)
    _chk(_load().oracle_mst_prim(_p(W), n, int(widest), _p(order), _p(parent), _p(aw), _p(af)),
         "oracle_mst_prim")
    return order, parent, aw, af


def linkage(W: np.ndarray, widest: bool = False) -> np.ndarray:
    """Single-linkage dendrogram, (n-1) x 4 float64: clusters a < b joined, weight,
    size of the new cluster (ids >= n are earlier merges)."""
    W = _sq(W, np.float32)
    n = W.shape[0]
    Z = np.zeros((max(n - 1, 0), 4), np.float64)
    _chk(_load().oracle_linkage(_p(W), n, int(widest), _p(Z)), "oracle_linkage")
    return Z


def appd_fw(W: np.ndarray, widest: bool = False):
    """Minimax (or widest) Floyd-Warshall over the edge total order, O(n^3)."""
    W = _sq(W, np.float32)
    n = W.shape[0]
    M = np.empty((n, n), np.float32)
    idx = np.empty((n, n), np.int32)
    _chk(_load().oracle_appd_fw(_p(W), n, int(widest), _p(M), _p(idx)), "oracle_appd_fw")
    return M, idx


def pairwise_euclidean_f32(X: np.ndarray, lib=None) -> np.ndarray:
    X = np.ascontiguousarray(X, dtype=np.float32)
    n, d = X.shape
    W = np.empty((n, n), np.float32)
    _chk((lib or _load()).oracle_pairwise_euclidean_f32(_p(X), n, d, _p(W)),
         "pairwise_euclidean_f32")
    return W


def pairwise_euclidean_f64(X: np.ndarray) -> np.ndarray:
    X = np.ascontiguousarray(X, dtype=np.float64)
    n, d = X.shape
    W = np.empty((n, n), np.float64)
    _chk(_load().oracle_pairwise_euclidean_f64(_p(X), n, d, _p(W)), "pairwise_euclidean_f64")
    return W


def grad_points(X: np.ndarray, G: np.ndarray, idx: np.ndarray, with_edges: bool = False,
                lib=None):
    """dL/dX (float64) of L = sum_{i!=j} G_ij M_ij through the bottleneck edges idx."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    G = np.ascontiguousarray(G, dtype=np.float64)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    n, d = X.shape
    dX = np.empty((n, d), np.float64)
    ge = np.empty((n, n), np.float64) if with_edges else None
    _chk((lib or _load()).oracle_grad_points(_p(X), n, d, _p(G), _p(idx), _p(dX),
                                    _p(ge) if with_edges else None), "oracle_grad_points")
    return (dX, ge) if with_edges else dX


def loss_f64(G: np.ndarray, M: np.ndarray) -> float:
    G = np.ascontiguousarray(G, dtype=np.float64)
    M = np.ascontiguousarray(M, dtype=np.float64)
    return float(_load().oracle_loss_f64(_p(G), _p(M), G.shape[0]))
