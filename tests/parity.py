"""Comparison rules between the HIP path and the CPU oracle.

kNN (tie-aware): a row passes when the GPU's neighbour set equals the
oracle's, or when every index in the symmetric difference sits at a
near-tie with the oracle's k-th distance: |D_ij - D_i(k)| / D_i(k) < 1e-5
(oracle float64 distances).  Where the sets agree the index order must
agree too (both sides order by (distance, index)), and distances must agree
to 1e-5 relative.

Connectivities: on rows untouched by near-tie swaps, CSR columns must be
identical and weights within 1e-5 relative; an entry present on one side
only must touch a near-tie row.
"""

from __future__ import annotations

import numpy as np

NEAR_TIE = 1e-5
REL_TOL = 1e-5


def cosine_pair_dist(X, ii, jj):
    """Cosine distances 1 - cos of row pairs (float64; the near-tie check only)."""
    a = np.asarray(X, dtype=np.float64)[np.asarray(ii)]
    b = np.asarray(X, dtype=np.float64)[np.asarray(jj)]
    na, nb = np.sqrt((a * a).sum(1)), np.sqrt((b * b).sum(1))
    c = np.where((na > 0) & (nb > 0), (a * b).sum(1) / np.maximum(na * nb, 1e-300), 0.0)
    return 1.0 - c


def compare_knn(X, rows, idx_g, dist_g, idx_o, dist_o, oracle, k, self_mode=True, pair_dist=None):
    """Compare GPU rows (already sliced to ``rows``) with oracle rows.

    ``pair_dist(X, ii, jj)`` gives the distances of row pairs for the near-tie
    check (default: Euclidean, from the oracle).  Returns a dict of counters;
    raises AssertionError on a real mismatch.
    """
    if pair_dist is None:
        def pair_dist(X_, ii, jj):
            return np.sqrt(oracle.pair_d2(X_, ii, jj))
    idx_g = np.asarray(idx_g)
    dist_g = np.asarray(dist_g, dtype=np.float64)
    idx_o = np.asarray(idx_o)
    dist_o = np.asarray(dist_o, dtype=np.float64)
    assert idx_g.shape == idx_o.shape == (len(rows), k)
    first = 1 if self_mode else 0
    if self_mode:
        assert (idx_g[:, 0] == rows).all(), "self must sit in column 0"
        assert (dist_g[:, 0] == 0).all()
    exact_rows = 0
    tie_rows = []
    for r in range(len(rows)):
        gi, oi = idx_g[r, first:], idx_o[r, first:]
        if np.array_equal(gi, oi):
            exact_rows += 1
            continue
        sg, so = set(gi.tolist()), set(oi.tolist())
        assert len(sg - {-1}) == int((gi >= 0).sum()), f"row {rows[r]}: repeated neighbour in GPU output"
        diff = sorted(sg ^ so)
        # an empty slot (-1) on one side only means the candidate counts differ
        assert -1 not in diff, f"row {rows[r]}: gpu={gi.tolist()} oracle={oi.tolist()}"
        if not diff:
            # same set, different order: only legal between exactly equal distances
            dg = dist_g[r, first:]
            assert (np.diff(dg) >= 0).all(), f"row {rows[r]}: GPU distances not ascending"
            tie_rows.append(rows[r])
            continue
        dk = pair_dist(X, np.array([rows[r]]), np.array([oi[-1]]))[0]
        dj = pair_dist(X, np.full(len(diff), rows[r]), np.array(diff))
        rel = np.abs(dj - dk) / max(dk, 1e-300)
        assert (rel < NEAR_TIE).all(), (
            f"row {rows[r]}: neighbour sets differ beyond a near-tie: gpu={gi.tolist()} oracle={oi.tolist()} "
            f"rel gaps={rel.tolist()}")
        tie_rows.append(rows[r])
    # distances: compare per index (robust to tie reorderings)
    rel_max = 0.0
    for r in range(len(rows)):
        dg = dict(zip(idx_g[r].tolist(), dist_g[r].tolist()))
        do = dict(zip(idx_o[r].tolist(), dist_o[r].tolist()))
        for j in (set(dg) & set(do)) - {-1}:
            a, b = dg[j], do[j]
            if b == 0:
                assert a == 0, f"row {rows[r]} col {j}: {a} vs 0"
                continue
            rel_max = max(rel_max, abs(a - b) / b)
    assert rel_max <= REL_TOL, f"distance relative error {rel_max}"
    return {"rows": len(rows), "exact_rows": exact_rows, "near_tie_rows": len(tie_rows), "dist_rel_max": rel_max,
            "tie_row_ids": tie_rows}


def csr_rows(indptr, indices, data):
    indptr = np.asarray(indptr)
    return [(indices[indptr[i]:indptr[i + 1]], data[indptr[i]:indptr[i + 1]]) for i in range(len(indptr) - 1)]


def compare_csr(g, o, tie_rows=()):
    """``g``, ``o``: (indptr, indices, data) numpy triples.  Returns max rel error."""
    gi, gx, gd = (np.asarray(a) for a in g)
    oi, ox, od = (np.asarray(a) for a in o)
    assert gi.shape == oi.shape
    n = len(gi) - 1
    ties = set(int(t) for t in tie_rows)
    rel_max = 0.0
    if not ties:
        np.testing.assert_array_equal(gi, oi)
        np.testing.assert_array_equal(gx, ox)
        nz = od != 0
        rel = np.abs(gd.astype(np.float64) - od) / np.abs(od.astype(np.float64))
        rel_max = float(rel[nz].max()) if nz.any() else 0.0
        assert rel_max <= REL_TOL, f"weight relative error {rel_max}"
        return rel_max
    for i in range(n):
        cg, vg = gx[gi[i]:gi[i + 1]], gd[gi[i]:gi[i + 1]]
        co, vo = ox[oi[i]:oi[i + 1]], od[oi[i]:oi[i + 1]]
        if i in ties:
            continue
        only = set(cg.tolist()) ^ set(co.tolist())
        for j in only:
            assert j in ties, f"row {i}: entry {j} on one side only and no near-tie row involved"
        common, ig, io = np.intersect1d(cg, co, return_indices=True)
        for a, b, j in zip(vg[ig], vo[io], common):
            if j in ties:
                continue
            rel_max = max(rel_max, abs(float(a) - float(b)) / abs(float(b)))
    assert rel_max <= REL_TOL, f"weight relative error {rel_max}"
    return rel_max


def check_graph_properties(indptr, indices, data, n, k, rho=None, sigma=None, dist=None):
    """Invariants that hold at any size."""
    indptr = np.asarray(indptr)
    indices = np.asarray(indices)
    data = np.asarray(data)
    nnz = int(indptr[-1])
    assert indptr[0] == 0 and (np.diff(indptr) >= 0).all()
    assert len(indices) == nnz == len(data)
    assert nnz <= 2 * n * (k - 1)
    assert ((data > 0) & (data <= 1)).all()
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(indptr))
    assert (rows != indices).all(), "diagonal entry"
    # ascending unique columns within rows
    same_row = rows[1:] == rows[:-1]
    assert (indices[1:][same_row] > indices[:-1][same_row]).all()
    # bitwise symmetry: sort the transpose's keys and compare
    key = rows * n + indices
    tkey = indices.astype(np.int64) * n + rows
    order = np.argsort(tkey, kind="stable")
    assert np.array_equal(tkey[order], key), "pattern not symmetric"
    assert np.array_equal(data[order].view(np.uint32), data.view(np.uint32)), "values not bitwise symmetric"
    if rho is not None and dist is not None and k > 1:
        dist = np.asarray(dist, dtype=np.float64)
        pos = np.where(dist[:, 1:] > 0, dist[:, 1:], np.inf).min(axis=1)
        pos[np.isinf(pos)] = 0
        np.testing.assert_array_equal(np.asarray(rho), pos)
    if rho is not None and sigma is not None and dist is not None and k > 1:
        rho = np.asarray(rho)
        sigma = np.asarray(sigma)
        ok = sigma > 0
        if ok.any():
            g = np.maximum(dist[ok, 1:] - rho[ok, None], 0)
            s = np.exp(-g / sigma[ok, None]).sum(axis=1)
            assert np.abs(s - np.log2(k)).max() <= 1e-6


def tie_aware_recall(dist_g, dist_o, k, self_mode=True):
    """Recall@k of an approximate result with exact distances.

    A returned neighbour counts as a hit when its distance is within the
    exact k-th distance (x (1 + 1e-5) for near-ties).  ``dist_g`` are the
    float64-exact distances the rerank returned for the approximate lists;
    ``dist_o`` the oracle's.  Returns the mean over rows.
    """
    first = 1 if self_mode else 0
    dg = np.asarray(dist_g, dtype=np.float64)[:, first:]
    dk = np.asarray(dist_o, dtype=np.float64)[:, -1:]
    hits = (dg <= dk * (1 + NEAR_TIE)).sum(axis=1)
    return float(np.minimum(hits, k - first).mean() / (k - first))
