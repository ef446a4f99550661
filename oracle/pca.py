"""Float64 reference of the sparse PCA that produces the embedding the kNN
graph consumes (Methods, "Principal component analysis"); test
infrastructure only.

For a cells x genes matrix X (CSR):

  mu  = X^T 1 / n                       per-gene means
  S   = X^T X                           (the Gram matrix; only its upper
                                         triangle is accumulated, then copied)
  C   = (S - n mu mu^T) / (n - 1)       the centred covariance, without
                                         centring the sparse matrix
  C v = lambda v                        the top-k eigenpairs, eigenvalues in
                                         descending order
  Z   = X V - 1 (mu^T V)                the embedding, centred implicitly

Readings where the paper is silent: each loading is signed so that its entry
of largest magnitude is positive (the lower gene index on ties); the
eigendecomposition is a float64 symmetric solver (a library routine here).
"""

from __future__ import annotations

import numpy as np


def dense(indptr, indices, data, p: int) -> np.ndarray:
    """The CSR matrix as dense float64 (small cases only)."""
    n = len(indptr) - 1
    X = np.zeros((n, p), dtype=np.float64)
    for c in range(n):
        lo, hi = indptr[c], indptr[c + 1]
        X[c, indices[lo:hi]] += data[lo:hi].astype(np.float64)
    return X


def gram(indptr, indices, data, p: int):
    """``(mu, S)``: per-gene means and X^T X in float64 (each entry summed over
    the cells in order)."""
    n = len(indptr) - 1
    mu = np.zeros(p, dtype=np.float64)
    S = np.zeros((p, p), dtype=np.float64)
    for c in range(n):
        lo, hi = indptr[c], indptr[c + 1]
        g = np.asarray(indices[lo:hi])
        v = np.asarray(data[lo:hi], dtype=np.float64)
        mu[g] += v
        S[np.ix_(g, g)] += np.outer(v, v)
    return mu / n, S


def covariance(indptr, indices, data, p: int):
    """``(mu, C)`` with C = (S - n mu mu^T) / (n - 1)."""
    n = len(indptr) - 1
    mu, S = gram(indptr, indices, data, p)
    return mu, (S - n * np.outer(mu, mu)) / (n - 1)


def sign_rule(V: np.ndarray) -> np.ndarray:
    """Flip each column so that its largest-magnitude entry (lowest index on
    ties) is positive."""
    V = V.copy()
    for j in range(V.shape[1]):
        i = int(np.argmax(np.abs(V[:, j])))
        if V[i, j] < 0:
            V[:, j] = -V[:, j]
    return V


def pca(indptr, indices, data, p: int, k: int):
    """``(mu, C, evals (k, descending), V (p x k), Z (n x k))``."""
    mu, C = covariance(indptr, indices, data, p)
    w, U = np.linalg.eigh(C)
    order = np.argsort(-w, kind="stable")[:k]
    evals = w[order]
    V = sign_rule(U[:, order])
    n = len(indptr) - 1
    Z = np.zeros((n, k), dtype=np.float64)
    for c in range(n):
        lo, hi = indptr[c], indptr[c + 1]
        Z[c] = np.asarray(data[lo:hi], dtype=np.float64) @ V[indices[lo:hi]]
    Z -= mu @ V
    return mu, C, evals, V, Z
