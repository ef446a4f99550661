"""Float64 reference of the routed form's coarse partitions and candidate
sets (test infrastructure only).

The routed form splits the cells into P coarse partitions by Lloyd's
k-means and answers a query from the cells of the partitions it probes:

  kmeans         initial centroids = the given rows of X; each iteration
                 assigns every row to its nearest centroid (exact float64
                 distance from direct differences, lower centroid index on
                 ties), then moves each centroid to the mean of its rows,
                 the exact sum rounded to float64, divided by the count in
                 float64 and rounded to float32.  A centroid left without
                 rows takes the row that lies farthest from its own centroid
                 (largest distance, lower row index on ties; one row per empty
                 centroid, empty centroids in ascending order); that row
                 leaves its old centroid's mean.  A final assignment pass
                 gives the returned labels.
  inverted_lists offsets (P+1) and the rows of each partition in ascending
                 order.
  probed_candidates / routed_knn
                 the candidate set of query q is the union of the rows of
                 the partitions it probes (listed partitions, -1 entries
                 ignored); the answer is the exact kNN within that set with
                 q itself in slot 0; rows marked for exact search use every
                 row instead.

Only tests (and the smoke check) use this module.
"""

from __future__ import annotations

import math

import numpy as np

from . import knn, knn_subset


def assign(X: np.ndarray, C: np.ndarray):
    """Nearest centroid of every row: ``(labels int32, d2 float64)``."""
    idx, d2, _ = knn(np.ascontiguousarray(C, dtype=np.float32), 1, Q=X)
    return idx[:, 0].copy(), d2[:, 0].copy()


def centroid_means(X: np.ndarray, labels: np.ndarray, P: int, C_prev: np.ndarray):
    """Per-partition mean of the member rows: exact sum (math.fsum) rounded to
    float64, divided by the count in float64, rounded to float32.  Partitions
    without members keep ``C_prev`` (the caller relocates them first)."""
    C = np.array(C_prev, dtype=np.float32, copy=True)
    Xd = X.astype(np.float64)
    order = np.argsort(labels, kind="stable")
    bounds = np.searchsorted(labels[order], np.arange(P + 1))
    for p in range(P):
        rows = order[bounds[p]:bounds[p + 1]]
        if rows.size == 0:
            continue
        cnt = float(rows.size)
        for t in range(X.shape[1]):
            C[p, t] = np.float32(math.fsum(Xd[rows, t]) / cnt)
    return C


def relocate_empty(X: np.ndarray, labels: np.ndarray, d2: np.ndarray, P: int):
    """Give every empty partition (ascending) the row farthest from its own
    centroid (largest d2, lower index on ties), one row each.  Returns the
    new labels, the relocated centroids' rows and the number relocated."""
    labels = labels.copy()
    counts = np.bincount(labels, minlength=P)
    empty = np.flatnonzero(counts == 0)
    if empty.size == 0:
        return labels, {}, 0
    order = np.lexsort((np.arange(labels.size), -d2))
    moved = {}
    for e, r in zip(empty, order[: empty.size]):
        labels[r] = e
        moved[int(e)] = int(r)
    return labels, moved, int(empty.size)


def kmeans(X: np.ndarray, init_rows: np.ndarray, iters: int):
    """Lloyd's k-means as stated in the module docstring.

    Returns ``(centroids float32 P x d, labels int32 n, relocated)`` where
    ``labels`` come from the final assignment pass and ``relocated`` counts
    the empty-partition relocations over all iterations.
    """
    X = np.ascontiguousarray(X, dtype=np.float32)
    init_rows = np.asarray(init_rows, dtype=np.int64)
    P = init_rows.size
    C = X[init_rows].copy()
    relocated = 0
    for _ in range(iters):
        labels, d2 = assign(X, C)
        labels, moved, nrel = relocate_empty(X, labels, d2, P)
        relocated += nrel
        C = centroid_means(X, labels, P, C)
        for e, r in moved.items():
            C[e] = X[r]
    labels, _ = assign(X, C)
    return C, labels, relocated


def inverted_lists(labels: np.ndarray, P: int):
    """``(offsets int64 P+1, perm int32 n)``: rows of partition p ascending."""
    labels = np.asarray(labels)
    perm = np.argsort(labels, kind="stable").astype(np.int32)
    offsets = np.zeros(P + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(np.bincount(labels, minlength=P))
    return offsets, perm


def probed_candidates(offsets: np.ndarray, perm: np.ndarray, probes: np.ndarray, exact_rows=None):
    """CSR candidate sets: union of the probed partitions' rows per query
    (repeated or -1 probe entries ignored); rows flagged in ``exact_rows`` get
    every row."""
    n = perm.size
    probes = np.asarray(probes)
    off = [0]
    ids = []
    for q in range(probes.shape[0]):
        if exact_rows is not None and exact_rows[q]:
            ids.append(np.arange(n, dtype=np.int64))
        else:
            ps = np.unique(probes[q][probes[q] >= 0])
            parts = [perm[offsets[p]:offsets[p + 1]] for p in ps]
            ids.append(np.concatenate(parts).astype(np.int64) if parts else np.zeros(0, np.int64))
        off.append(off[-1] + ids[-1].size)
    return np.asarray(off, dtype=np.int64), np.concatenate(ids) if ids else np.zeros(0, np.int64)


def routed_knn(X: np.ndarray, k: int, offsets: np.ndarray, perm: np.ndarray, probes: np.ndarray,
               exact_rows=None, rows=None):
    """Exact kNN of every row (or of ``rows``, whose probe lists and flags are
    then given per selected row) within its probed partitions, or over all
    rows where ``exact_rows`` is set.  Returns ``(idx, d2, dist)``."""
    off, ids = probed_candidates(offsets, perm, probes, exact_rows)
    return knn_subset(X, k, off, ids, rows=rows)


def recall(found: np.ndarray, exact: np.ndarray) -> float:
    """Mean over rows of |found ∩ exact| / k (index sets, -1 ignored)."""
    hits = 0
    for a, b in zip(found, exact):
        hits += len(set(a[a >= 0].tolist()) & set(b.tolist()))
    return hits / exact.size
