"""Float64 reference of the energy distance between groups of cells
(Methods, "Perturbation distance computation"); test infrastructure only.

For groups X and Y of cells (rows of an embedding):

  E(X, Y) = 2 mean ||X_i - Y_j|| - mean ||X_i - X_i'|| - mean ||Y_j - Y_j'||

The cross mean runs over all n_X n_Y pairs; a within-group mean runs over
the n (n - 1) / 2 pairs of the upper triangle.  A group with fewer than two
cells has no within-group pairs and is skipped: its within mean counts as
0.  A cross pair with an empty group has no pairs: its mean is NaN.

The group-pair distance sums come from ``oracle_edistance_sums`` (oracle.c,
float64 direct differences, sequential sums); the means and the assembly
E[a, b] = 2 d[a, b] - d[a, a] - d[b, b] are plain float64 numpy here.

Groups are given as category offsets (G + 1, ascending, offsets[0] = 0) and
the cell-index array: group g holds rows cells[offsets[g]:offsets[g + 1]].
"""

from __future__ import annotations

import numpy as np

from . import _load, _p


def groups_from_labels(labels: np.ndarray, G: int | None = None):
    """``(offsets int64 G+1, cells int32)`` of integer labels: each group's
    rows in ascending order."""
    labels = np.asarray(labels)
    G = int(labels.max()) + 1 if G is None else G
    cells = np.argsort(labels, kind="stable").astype(np.int32)
    offsets = np.zeros(G + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(np.bincount(labels, minlength=G))
    return offsets, cells


def sums(X: np.ndarray, offsets: np.ndarray, cells: np.ndarray, pairs: np.ndarray) -> np.ndarray:
    """Sum of distances of every listed pair (a, b): all n_a n_b pairs for
    a != b, the upper triangle for a == b."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    cells = np.ascontiguousarray(cells, dtype=np.int32)
    pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    out = np.empty(pairs.shape[0], dtype=np.float64)
    st = _load().oracle_edistance_sums(_p(X), X.shape[0], X.shape[1], _p(offsets), offsets.size - 1, _p(cells),
                                       _p(pairs), pairs.shape[0], _p(out))
    if st != 0:
        raise ValueError("oracle_edistance_sums: invalid arguments")
    return out


def pair_counts(sizes: np.ndarray, pairs: np.ndarray) -> np.ndarray:
    """Number of distances behind each pair's sum (float64)."""
    sizes = np.asarray(sizes, dtype=np.float64)
    a, b = pairs[:, 0], pairs[:, 1]
    return np.where(a == b, sizes[a] * (sizes[a] - 1) / 2, sizes[a] * sizes[b])


def means(sizes: np.ndarray, pairs: np.ndarray, s: np.ndarray) -> np.ndarray:
    """Mean distance of each pair; within-group means of groups with fewer
    than two cells are 0 (skipped), cross means with an empty group NaN."""
    cnt = pair_counts(sizes, pairs)
    diag = pairs[:, 0] == pairs[:, 1]
    with np.errstate(invalid="ignore", divide="ignore"):
        m = s / cnt
    m = np.where(diag & (cnt == 0), 0.0, m)
    return np.where(~diag & (cnt == 0), np.nan, m)


def all_pairs(G: int) -> np.ndarray:
    """Every (a, b) with a <= b, row-major."""
    a, b = np.triu_indices(G)
    return np.stack([a, b], axis=1).astype(np.int32)


def pairwise(X: np.ndarray, offsets: np.ndarray, cells: np.ndarray):
    """``(E, D)``: G x G energy distances and mean distances (symmetric)."""
    G = offsets.size - 1
    pairs = all_pairs(G)
    sizes = np.diff(offsets)
    m = means(sizes, pairs, sums(X, offsets, cells, pairs))
    D = np.zeros((G, G), dtype=np.float64)
    D[pairs[:, 0], pairs[:, 1]] = m
    D[pairs[:, 1], pairs[:, 0]] = m
    dd = np.diag(D).copy()
    E = 2.0 * D - (dd[:, None] + dd[None, :])  # the within terms added first: E is exactly symmetric
    return E, D


def onesided_pairs(G: int, ref: int) -> np.ndarray:
    """The pairs a one-sided query needs: (ref, g) for every g, then (g, g)
    for every g != ref ((ref, ref) is the first list's entry g = ref)."""
    cross = np.stack([np.full(G, ref), np.arange(G)], axis=1)
    diag = np.array([[g, g] for g in range(G) if g != ref], dtype=np.int64).reshape(-1, 2)
    return np.concatenate([cross, diag]).astype(np.int32)


def onesided(X: np.ndarray, offsets: np.ndarray, cells: np.ndarray, ref: int) -> np.ndarray:
    """E(ref, g) for every group g (E(ref, ref) = 0)."""
    G = offsets.size - 1
    pairs = onesided_pairs(G, ref)
    sizes = np.diff(offsets)
    m = means(sizes, pairs, sums(X, offsets, cells, pairs))
    cross = m[:G]
    within = np.empty(G, dtype=np.float64)
    within[ref] = cross[ref]
    others = [g for g in range(G) if g != ref]
    within[others] = m[G:]
    return 2.0 * cross - (within[:, None] + within[ref])[:, 0]
