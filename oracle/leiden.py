"""Leiden communities of the connectivities graph (test infrastructure only).

The arithmetic is ``oracle_leiden`` in leiden.c, whose header spells out the
reading of the algorithm; this module marshals arrays and holds the plain
modularity of a labelling by its definition.
"""

from __future__ import annotations

import ctypes

import numpy as np

from . import _load, _p


def leiden(indptr, indices, weights, gamma: float = 1.0):
    """``(labels int32, modularity, levels)`` of a symmetric CSR graph."""
    lib = _load()
    indptr = np.ascontiguousarray(indptr, dtype=np.int64)
    indices = np.ascontiguousarray(indices, dtype=np.int32)
    weights = np.ascontiguousarray(weights, dtype=np.float32)
    n = len(indptr) - 1
    labels = np.empty(n, dtype=np.int32)
    q = ctypes.c_double(0.0)
    lv = ctypes.c_int32(0)
    st = lib.oracle_leiden(_p(indptr), _p(indices), _p(weights), n, gamma, _p(labels), ctypes.byref(q),
                           ctypes.byref(lv))
    if st != 0:
        raise ValueError("oracle_leiden: invalid graph or resolution")
    return labels, float(q.value), int(lv.value)


def refine(indptr, indices, weights, labels, gamma: float = 1.0):
    """The refinement step alone: refined labels inside the communities ``labels``."""
    lib = _load()
    indptr = np.ascontiguousarray(indptr, dtype=np.int64)
    indices = np.ascontiguousarray(indices, dtype=np.int32)
    weights = np.ascontiguousarray(weights, dtype=np.float32)
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    n = len(indptr) - 1
    out = np.empty(n, dtype=np.int32)
    if lib.oracle_leiden_refine(_p(indptr), _p(indices), _p(weights), n, gamma, _p(labels), _p(out)) != 0:
        raise ValueError("oracle_leiden_refine: invalid input")
    return out


def scale(nnz: int, wmax: float) -> int:
    """The fixed-point exponent S of the weights."""
    return int(_load().oracle_leiden_scale(nnz, wmax))
