"""Float64 reference of the UMAP layout step (test infrastructure only).

The arithmetic is ``oracle_umap_layout`` in oracle.c (the reading of the
method is spelled out there); this module marshals arrays and provides the
curve fit that gives the kernel parameters a, b from min_dist and spread:
1 / (1 + a x^(2b)) fitted by least squares to 1 for x < min_dist and
exp(-(x - min_dist) / spread) beyond, on 300 points of [0, 3 spread].
"""

from __future__ import annotations

import ctypes

import numpy as np

from . import _load, _p


def layout(indptr, indices, weights, Y0, n_epochs: int, a: float, b: float, gamma: float = 1.0,
           alpha0: float = 1.0, neg: int = 5, seed: int = 0) -> np.ndarray:
    """The embedding after ``n_epochs`` epochs from ``Y0`` (n x dim, float64)."""
    lib = _load()
    indptr = np.ascontiguousarray(indptr, dtype=np.int64)
    indices = np.ascontiguousarray(indices, dtype=np.int32)
    weights = np.ascontiguousarray(weights, dtype=np.float32)
    Y = np.array(Y0, dtype=np.float64, copy=True, order="C")
    n, dim = Y.shape
    st = lib.oracle_umap_layout(_p(indptr), _p(indices), _p(weights), n, dim, _p(Y), n_epochs, a, b, gamma, alpha0,
                                neg, ctypes.c_uint64(seed))
    if st != 0:
        raise ValueError("oracle_umap_layout: invalid arguments")
    return Y


def splitmix64_next(state: int) -> int:
    return int(_load().oracle_splitmix64_next(ctypes.c_uint64(state)))


def negative(seed: int, t: int, e: int, p: int, n: int) -> int:
    """The vertex that negative sample ``p`` of edge ``e`` draws in epoch ``t``."""
    return int(_load().oracle_umap_negative(ctypes.c_uint64(seed), t, e, p, n))


def fit_ab(min_dist: float = 0.5, spread: float = 1.0):
    """``(a, b)`` by least squares (scipy's curve_fit)."""
    from scipy.optimize import curve_fit

    x = np.linspace(0, spread * 3, 300)
    y = np.where(x < min_dist, 1.0, np.exp(-(x - min_dist) / spread))
    (a, b), _ = curve_fit(lambda x, a, b: 1.0 / (1.0 + a * x ** (2 * b)), x, y)
    return float(a), float(b)
