"""CPU oracle for the neighbourhood-graph step (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  The HIP library never does,
and this package imports nothing from it.

The arithmetic lives in ``oracle.c`` (float64, brute force, compiled with
``-ffp-contract=off``); this module only builds it with gcc and marshals
numpy arrays.  ``mlp.py`` holds the float64 reference of the partition
router's network, ``partition.py`` the k-means partitions and the routed
form's candidate sets, ``edistance.py`` the group-pair distance sums and
energy distances, ``pca.py`` the sparse PCA that produces the embedding,
``umap.py`` the UMAP layout of the graph, ``leiden.py`` Leiden communities
of the graph (arithmetic in ``leiden.c``).
"""

from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "leiden.c")]
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` and ``leiden.c`` into ``liboracle.so`` with gcc (OpenMP, no contraction)."""
    if (not force and os.path.exists(_LIB)
            and all(os.path.getmtime(_LIB) >= os.path.getmtime(src) for src in _SRCS)):
        return _LIB
    tmp = _LIB + f".tmp{os.getpid()}"
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wextra", "-o", tmp, *_SRCS, "-lquadmath", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build(force=False)
            lib = ctypes.CDLL(_LIB)
            P = ctypes.c_void_p
            i64 = ctypes.c_int64
            i32 = ctypes.c_int
            lib.oracle_knn.argtypes = [P, i64, P, P, i64, i32, i32, P, P, P]
            lib.oracle_knn.restype = i32
            lib.oracle_pair_d2.argtypes = [P, i64, i32, P, P, i64, P]
            lib.oracle_pair_d2.restype = i32
            lib.oracle_smooth_knn.argtypes = [P, P, i64, i32, P, P, P]
            lib.oracle_smooth_knn.restype = i64
            lib.oracle_fuzzy_union.argtypes = [P, P, i64, i32, P, P, P, i64]
            lib.oracle_fuzzy_union.restype = i64
            lib.oracle_max_threads.restype = i32
            lib.oracle_knn_cosine.argtypes = [P, i64, P, P, i64, i32, i32, P, P, P]
            lib.oracle_knn_cosine.restype = i32
            lib.oracle_knn_subset.argtypes = [P, i64, i32, i32, P, i64, P, P, P, P, P]
            lib.oracle_knn_subset.restype = i32
            lib.oracle_edistance_sums.argtypes = [P, i64, i32, P, i64, P, P, i64, P]
            lib.oracle_edistance_sums.restype = i32
            lib.oracle_umap_layout.argtypes = [P, P, P, i64, i32, P, i32, ctypes.c_double, ctypes.c_double,
                                               ctypes.c_double, ctypes.c_double, i32, ctypes.c_uint64]
            lib.oracle_umap_layout.restype = i32
            lib.oracle_splitmix64_next.argtypes = [ctypes.c_uint64]
            lib.oracle_splitmix64_next.restype = ctypes.c_uint64
            lib.oracle_umap_negative.argtypes = [ctypes.c_uint64, i32, i64, i32, i64]
            lib.oracle_umap_negative.restype = i64
            lib.oracle_leiden.argtypes = [P, P, P, i64, ctypes.c_double, P, P, P]
            lib.oracle_leiden.restype = i32
            lib.oracle_leiden_refine.argtypes = [P, P, P, i64, ctypes.c_double, P, P]
            lib.oracle_leiden_refine.restype = i32
            lib.oracle_leiden_scale.argtypes = [i64, ctypes.c_double]
            lib.oracle_leiden_scale.restype = i32
            _lib = lib
    return _lib


def _p(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def knn(R: np.ndarray, k: int, Q: np.ndarray | None = None, self_ids: np.ndarray | None = None,
        metric: str = "euclidean"):
    """Exact kNN (float64 brute force, lowest index first on ties).

    ``knn(X, k)``: every row of ``X`` against ``X``, self forced into slot 0.
    ``knn(R, k, Q=Q, self_ids=ids)``: queries ``Q`` against ``R``; ``ids``
    (or ``None``) names the reference row that is each query itself.
    Returns ``(idx int32, d2 float64, dist float32)``, each ``nq x k``.
    ``metric="cosine"``: the cosine distance 1 - cos (float64 in the second
    array, float32 in the third); rows of zero norm are at distance 1.
    """
    R = np.ascontiguousarray(R, dtype=np.float32)
    if Q is None:
        Q = R
        self_ids = np.arange(R.shape[0], dtype=np.int64)
    Q = np.ascontiguousarray(Q, dtype=np.float32)
    if self_ids is not None:
        self_ids = np.ascontiguousarray(self_ids, dtype=np.int64)
        assert self_ids.shape == (Q.shape[0],)
    nq, d = Q.shape
    nr = R.shape[0]
    assert R.shape[1] == d
    idx = np.empty((nq, k), dtype=np.int32)
    d2 = np.empty((nq, k), dtype=np.float64)
    dist = np.empty((nq, k), dtype=np.float32)
    if metric not in ("euclidean", "cosine"):
        raise ValueError(f"unknown metric {metric!r}")
    fn = _load().oracle_knn if metric == "euclidean" else _load().oracle_knn_cosine
    rc = fn(_p(Q), nq, _p(self_ids), _p(R), nr, d, k, _p(idx), _p(d2), _p(dist))
    if rc != 0:
        raise ValueError("oracle_knn: invalid arguments")
    return idx, d2, dist


def knn_subset(X: np.ndarray, k: int, cand_off: np.ndarray, cand_ids: np.ndarray, rows: np.ndarray | None = None):
    """Exact kNN of rows of ``X`` among their own candidate rows.

    Query ``i`` is row ``rows[i]`` (row ``i`` when ``rows`` is None); its
    candidates are ``cand_ids[cand_off[i]:cand_off[i+1]]``; the query's row
    sits in slot 0, empty slots hold index -1.  Returns ``(idx, d2, dist)``.
    """
    X = np.ascontiguousarray(X, dtype=np.float32)
    cand_off = np.ascontiguousarray(cand_off, dtype=np.int64)
    cand_ids = np.ascontiguousarray(cand_ids, dtype=np.int64)
    n, d = X.shape
    qrows = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    nq = n if qrows is None else qrows.shape[0]
    assert cand_off.shape == (nq + 1,) and cand_off[0] == 0 and cand_off[-1] == cand_ids.shape[0]
    idx = np.empty((nq, k), dtype=np.int32)
    d2 = np.empty((nq, k), dtype=np.float64)
    dist = np.empty((nq, k), dtype=np.float32)
    rc = _load().oracle_knn_subset(_p(X), n, d, k, _p(qrows), nq, _p(cand_off), _p(cand_ids), _p(idx), _p(d2),
                                   _p(dist))
    if rc != 0:
        raise ValueError("oracle_knn_subset: invalid arguments")
    return idx, d2, dist


def knn_rows(X: np.ndarray, rows: np.ndarray, k: int, metric: str = "euclidean"):
    """Exact kNN of the selected rows of ``X`` against all of ``X`` (self in slot 0)."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    return knn(X, k, Q=X[rows], self_ids=rows, metric=metric)


def pair_d2(X: np.ndarray, ii: np.ndarray, jj: np.ndarray) -> np.ndarray:
    """Exact float64 squared distances of row pairs ``(ii[p], jj[p])``."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    ii = np.ascontiguousarray(ii, dtype=np.int64).ravel()
    jj = np.ascontiguousarray(jj, dtype=np.int64).ravel()
    out = np.empty(ii.shape[0], dtype=np.float64)
    rc = _load().oracle_pair_d2(_p(X), X.shape[0], X.shape[1], _p(ii), _p(jj), ii.shape[0], _p(out))
    if rc != 0:
        raise ValueError("oracle_pair_d2: index out of range")
    return out


def smooth_knn(idx: np.ndarray, dist: np.ndarray):
    """``(rho, sigma, a, n_degenerate)`` from a kNN result (self in slot 0)."""
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    dist = np.ascontiguousarray(dist, dtype=np.float32)
    n, k = idx.shape
    rho = np.empty(n, dtype=np.float64)
    sigma = np.empty(n, dtype=np.float64)
    a = np.empty((n, max(k - 1, 0)), dtype=np.float64)
    deg = _load().oracle_smooth_knn(_p(idx), _p(dist), n, k, _p(rho), _p(sigma), _p(a))
    if deg < 0:
        raise ValueError("oracle_smooth_knn: invalid arguments")
    return rho, sigma, a, int(deg)


def fuzzy_union(idx: np.ndarray, a: np.ndarray):
    """CSR ``(indptr int64, indices int32, data float32)`` of A + A^T - A o A^T."""
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    n, k = idx.shape
    a = np.ascontiguousarray(a, dtype=np.float64)
    assert a.shape == (n, k - 1)
    cap = max(1, 2 * n * (k - 1))
    indptr = np.empty(n + 1, dtype=np.int64)
    indices = np.empty(cap, dtype=np.int32)
    data = np.empty(cap, dtype=np.float32)
    nnz = _load().oracle_fuzzy_union(_p(idx), _p(a), n, k, _p(indptr), _p(indices), _p(data), cap)
    if nnz < 0:
        raise ValueError("oracle_fuzzy_union: invalid kNN lists")
    return indptr, indices[:nnz].copy(), data[:nnz].copy()


def connectivities(idx: np.ndarray, dist: np.ndarray):
    """Smooth-kNN weights then fuzzy union: ``(indptr, indices, data, rho, sigma)``."""
    rho, sigma, a, _ = smooth_knn(idx, dist)
    indptr, indices, data = fuzzy_union(idx, a)
    return indptr, indices, data, rho, sigma


def knn_graph(X: np.ndarray, k: int, metric: str = "euclidean"):
    """The whole step on the CPU: exact kNN, then connectivities."""
    idx, _, dist = knn(X, k, metric=metric)
    indptr, indices, data, rho, sigma = connectivities(idx, dist)
    return dict(idx=idx, dist=dist, indptr=indptr, indices=indices, data=data, rho=rho, sigma=sigma)
