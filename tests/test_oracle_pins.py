"""Pins of the CPU oracle to things other than itself (no GPU needed).

Each test checks the oracle against a library routine, a closed form, a
hand-worked example or an invariant of the method, chosen so that a
plausible slip (self not forced, wrong tie order, target log2(k-1), a dropped
``-ab`` term, rho taken as a zero distance) fails at least one of them.
"""

import json
import math
import os

import numpy as np
import pytest
from scipy.optimize import brentq
from scipy.spatial.distance import cdist

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def lexsorted_knn(X, k, Q=None, self_ids=None):
    """Independent brute force: scipy cdist (float64) + numpy lexsort."""
    X64 = X.astype(np.float64)
    Q64 = X64 if Q is None else Q.astype(np.float64)
    if Q is None:
        self_ids = np.arange(X.shape[0])
    D = cdist(Q64, X64, "sqeuclidean")
    out = []
    for q in range(Q64.shape[0]):
        j = np.arange(X.shape[0])
        dq = D[q].copy()
        if self_ids is not None and self_ids[q] >= 0:
            keep = j != self_ids[q]
            order = np.lexsort((j[keep], dq[keep]))
            row = np.concatenate([[self_ids[q]], j[keep][order][: k - 1]])
        else:
            order = np.lexsort((j, dq))
            row = j[order][:k]
        out.append(row)
    return np.array(out), D


def no_near_tie(d_sorted, k, rel=1e-9):
    """Rows whose k-th and (k+1)-th distances are clearly separated."""
    dk = d_sorted[:, k - 1]
    dk1 = d_sorted[:, k]
    return (dk1 - dk) > rel * np.maximum(dk, 1e-300)


@pytest.mark.parametrize("n,d,seed", [(300, 7, 3), (500, 50, 4), (257, 1, 5)])
def test_knn_matches_cdist_lexsort(oracle_mod, n, d, seed):
    X = synth.mixture(n, d=d, n_clusters=5, seed=seed)
    k = 15
    idx, d2, dist = oracle_mod.knn(X, k)
    ref, D = lexsorted_knn(X, k)
    assert idx.shape == (n, k)
    assert (idx[:, 0] == np.arange(n)).all()
    np.testing.assert_array_equal(idx, ref)
    got = np.take_along_axis(D, idx.astype(np.int64), axis=1)
    got[:, 0] = 0.0
    np.testing.assert_allclose(d2, got, rtol=1e-12, atol=0)
    np.testing.assert_array_equal(dist, np.sqrt(d2).astype(np.float32))


def test_knn_matches_sklearn_brute(oracle_mod):
    from sklearn.neighbors import NearestNeighbors

    X = synth.mixture(800, d=50, n_clusters=8, seed=11)
    k = 15
    idx, d2, dist = oracle_mod.knn(X, k)
    nn = NearestNeighbors(n_neighbors=k + 1, algorithm="brute").fit(X.astype(np.float64))
    sd, si = nn.kneighbors(X.astype(np.float64))
    # drop self from sklearn's answer (continuous data: self is the unique zero)
    rows = []
    for i in range(X.shape[0]):
        r = [j for j in si[i] if j != i][: k - 1]
        rows.append(r)
    rows = np.array(rows)
    np.testing.assert_array_equal(np.sort(idx[:, 1:], axis=1), np.sort(rows, axis=1))
    sk_d = np.sort(np.where(si == np.arange(len(X))[:, None], np.inf, sd), axis=1)[:, : k - 1]
    np.testing.assert_allclose(dist[:, 1:], sk_d, rtol=1e-5)


def test_knn_rectangular(oracle_mod):
    R = synth.mixture(400, d=9, n_clusters=4, seed=21)
    Q = synth.mixture(37, d=9, n_clusters=4, seed=22)
    idx, d2, _ = oracle_mod.knn(R, 6, Q=Q)
    ref, D = lexsorted_knn(R, 6, Q=Q, self_ids=-np.ones(37, dtype=np.int64))
    np.testing.assert_array_equal(idx, ref)
    np.testing.assert_allclose(d2, np.take_along_axis(D, ref, axis=1), rtol=1e-12)


def test_pair_d2_matches_cdist(oracle_mod):
    # the exact squared distances the precision tests measure with: scipy's
    # float64 cdist on random pairs, including i == j and repeated pairs
    rng = np.random.default_rng(31)
    for n, d in [(50, 1), (300, 7), (1000, 50), (64, 129)]:
        X = (rng.standard_normal((n, d)) * rng.uniform(0.01, 100.0, d)).astype(np.float32)
        ii = rng.integers(0, n, 2000)
        jj = rng.integers(0, n, 2000)
        jj[:20] = ii[:20]
        got = oracle_mod.pair_d2(X, ii, jj)
        X64 = X.astype(np.float64)
        ref = np.array([cdist(X64[i:i + 1], X64[j:j + 1], "sqeuclidean")[0, 0] for i, j in zip(ii, jj)])
        np.testing.assert_allclose(got, ref, rtol=1e-13, atol=0)
        assert np.all(got[:20] == 0.0)
    with pytest.raises(ValueError):
        oracle_mod.pair_d2(X, np.array([0]), np.array([n]))


def test_lattice_ties_lowest_index_first(oracle_mod):
    n, k = 40, 7
    X = synth.lattice_1d(n, d=3)
    idx, d2, dist = oracle_mod.knn(X, k)
    # interior point i: i, then i-1, i+1 (distance 1), i-2, i+2 (distance 2), ...
    for i in range(5, n - 5):
        assert idx[i].tolist() == [i, i - 1, i + 1, i - 2, i + 2, i - 3, i + 3]
        assert dist[i].tolist() == [0, 1, 1, 2, 2, 3, 3]
    assert idx[0].tolist() == [0, 1, 2, 3, 4, 5, 6]
    assert idx[1].tolist() == [1, 0, 2, 3, 4, 5, 6]
    assert idx[2].tolist() == [2, 1, 3, 0, 4, 5, 6]
    assert idx[n - 1].tolist() == [n - 1, n - 2, n - 3, n - 4, n - 5, n - 6, n - 7]


def test_grid_ties_2d(oracle_mod):
    # 5x5 grid, row-major ids; the centre (id 12) has 4 neighbours at 1, 4 at sqrt 2
    g = np.array([[x, y] for y in range(5) for x in range(5)], dtype=np.float32)
    idx, _, dist = oracle_mod.knn(g, 9)
    assert idx[12].tolist() == [12, 7, 11, 13, 17, 6, 8, 16, 18]
    np.testing.assert_allclose(dist[12], [0, 1, 1, 1, 1] + [math.sqrt(2)] * 4, rtol=1e-7)


def test_duplicates_self_first(oracle_mod):
    X = synth.mixture(60, d=4, n_clusters=3, seed=31)
    X[9] = X[5]
    X[17] = X[5]
    idx, d2, dist = oracle_mod.knn(X, 5)
    assert idx[5, :3].tolist() == [5, 9, 17]
    assert idx[9, :3].tolist() == [9, 5, 17]
    assert idx[17, :3].tolist() == [17, 5, 9]
    assert dist[9, 1] == 0 and dist[9, 2] == 0
    rho, sigma, a, _ = oracle_mod.smooth_knn(idx, dist)
    # rho is the smallest strictly positive distance, not the duplicate's zero
    assert rho[9] == pytest.approx(float(dist[9, 3]))
    assert a[9, 0] == 1.0 and a[9, 1] == 1.0 and a[9, 2] == 1.0


def test_all_identical_points_degenerate(oracle_mod):
    X = np.ones((20, 3), dtype=np.float32)
    idx, _, dist = oracle_mod.knn(X, 6)
    assert (idx[:, 0] == np.arange(20)).all()
    assert (dist == 0).all()
    # lower indices first among the tied duplicates
    assert idx[7].tolist() == [7, 0, 1, 2, 3, 4]
    rho, sigma, a, deg = oracle_mod.smooth_knn(idx, dist)
    assert deg == 20
    assert (rho == 0).all() and (sigma == 0).all() and (a == 1).all()


def test_sigma_closed_form_k3(oracle_mod):
    # k = 3: 1 + exp(-(d2 - rho)/sigma) = log2 3  =>  sigma = (d2 - rho) / -ln(log2 3 - 1)
    rng = np.random.default_rng(5)
    n = 200
    d1 = rng.uniform(0.1, 3.0, n)
    d2 = d1 + rng.uniform(1e-3, 5.0, n)
    idx = np.stack([np.arange(n), (np.arange(n) + 1) % n, (np.arange(n) + 2) % n], axis=1)
    dist = np.stack([np.zeros(n), d1, d2], axis=1).astype(np.float32)
    rho, sigma, a, deg = oracle_mod.smooth_knn(idx, dist)
    assert deg == 0
    p = math.log2(3) - 1
    expect = (dist[:, 2].astype(np.float64) - dist[:, 1]) / -math.log(p)
    np.testing.assert_allclose(sigma, expect, rtol=1e-10)
    np.testing.assert_array_equal(rho, dist[:, 1].astype(np.float64))
    np.testing.assert_allclose(a[:, 0], 1.0, rtol=0)
    np.testing.assert_allclose(a[:, 1], p, rtol=1e-10)


@pytest.mark.parametrize("k", [4, 8, 15, 30])
def test_sigma_equal_gaps_root(oracle_mod, k):
    # distances rho, rho + D, rho + 2D, ...: sum_{m=0}^{k-2} q^m = log2 k, q = exp(-D/sigma)
    rng = np.random.default_rng(k)
    n = 50
    rho = rng.uniform(0.5, 2.0, n)
    gap = rng.uniform(0.01, 1.0, n)
    m = np.arange(k - 1)
    dist = np.concatenate([np.zeros((n, 1)), rho[:, None] + gap[:, None] * m], axis=1)
    dist = dist.astype(np.float32)
    idx = (np.arange(n)[:, None] + np.arange(k)) % n
    r, sigma, a, deg = oracle_mod.smooth_knn(idx, dist)
    assert deg == 0
    target = math.log2(k)
    for i in range(n):
        dd = dist[i, 1:].astype(np.float64)
        g = dd - dd[0]  # the float32 gaps actually stored
        q = brentq(lambda s: np.exp(-g / s).sum() - target, 1e-9, 1e9, xtol=1e-15, rtol=1e-15)
        assert sigma[i] == pytest.approx(q, rel=1e-9)


def test_smooth_invariants_on_mixture(oracle_mod):
    X = synth.workload("plain_10k", n=3000)
    k = 15
    idx, _, dist = oracle_mod.knn(X, k)
    rho, sigma, a, deg = oracle_mod.smooth_knn(idx, dist)
    assert deg == 0
    np.testing.assert_array_equal(rho, dist[:, 1].astype(np.float64))
    g = np.maximum(dist[:, 1:].astype(np.float64) - rho[:, None], 0)
    s = np.exp(-g / sigma[:, None]).sum(axis=1)
    assert np.abs(s - math.log2(k)).max() <= 1e-6
    assert (a > 0).all() and (a <= 1).all()
    assert (a[:, 0] == 1.0).all()


def _load_golden():
    with open(os.path.join(GOLDEN, "union_4pt.json")) as f:
        return json.load(f)


def test_union_hand_example(oracle_mod):
    gd = _load_golden()
    X = np.array(gd["x"], dtype=np.float32)[:, None]
    k = gd["k"]
    idx, _, dist = oracle_mod.knn(X, k)
    assert idx.tolist() == gd["idx"]
    assert dist.tolist() == gd["dist"]
    rho, sigma, a, _ = oracle_mod.smooth_knn(idx, dist)
    assert rho.tolist() == gd["rho"]
    p = math.log2(3) - 1
    np.testing.assert_allclose(sigma * -math.log(p), gd["sigma_times_neg_ln_p"], rtol=1e-12)
    indptr, indices, data = oracle_mod.fuzzy_union(idx, a)
    cs = gd["csr_symbolic"]
    assert indptr.tolist() == cs["indptr"]
    assert indices.tolist() == cs["indices"]
    vals = {"1": 1.0, "p": p, "2p-p^2": 2 * p - p * p}
    np.testing.assert_allclose(data, [vals[v] for v in cs["data"]], rtol=1e-7)


def test_union_dense_matrix_form(oracle_mod):
    """CSR equals the dense A + A^T - A o A^T (zeros dropped) on a small graph."""
    n, k = 120, 9
    idx, dist = synth.random_knn_lists(n, k, seed=3, hub_fraction=0.05)
    rho, sigma, a, _ = oracle_mod.smooth_knn(idx, dist)
    A = np.zeros((n, n))
    for i in range(n):
        A[i, idx[i, 1:]] = a[i]
    W = A + A.T - A * A.T
    indptr, indices, data = oracle_mod.fuzzy_union(idx, a)
    dense = np.zeros((n, n), dtype=np.float32)
    for i in range(n):
        cols = indices[indptr[i]:indptr[i + 1]]
        assert (np.diff(cols) > 0).all()
        dense[i, cols] = data[indptr[i]:indptr[i + 1]]
    np.testing.assert_allclose(dense, W.astype(np.float32), rtol=1e-7, atol=0)
    assert np.count_nonzero(W.astype(np.float32)) == indptr[-1]


def test_union_properties_mixture(oracle_mod):
    X = synth.workload("plain_10k", n=4000)
    k = 15
    g = oracle_mod.knn_graph(X, k)
    n = X.shape[0]
    indptr, indices, data = g["indptr"], g["indices"], g["data"]
    nnz = indptr[-1]
    assert n * (k - 1) <= nnz <= 2 * n * (k - 1)
    assert ((data > 0) & (data <= 1)).all()
    rows = np.repeat(np.arange(n), np.diff(indptr))
    assert (rows != indices).all()
    # bitwise symmetry
    fwd = dict(zip(zip(rows.tolist(), indices.tolist()), data.tolist()))
    for (i, j), w in fwd.items():
        assert fwd[(j, i)] == w


def test_union_rejects_duplicate_neighbour(oracle_mod):
    idx = np.array([[0, 1, 1], [1, 0, 2], [2, 1, 0]], dtype=np.int32)
    a = np.ones((3, 2))
    with pytest.raises(ValueError):
        oracle_mod.fuzzy_union(idx, a)


# ---- router network (oracle/mlp.py) -------------------------------------------------


def _mlp_small(seed=0, d=5, hidden=7, parts=11, n=13, m=4):
    from oracle import mlp

    rng = np.random.default_rng(seed)
    params = mlp.init_params(d, hidden, parts, seed=seed)
    # non-zero biases so that every term of the backward pass is exercised
    params = [p + (0.1 * rng.standard_normal(p.shape) if p.ndim == 1 else 0) for p in params]
    X = rng.standard_normal((n, d))
    lab = rng.integers(0, parts, size=(n, m))
    return mlp, params, X, mlp.soft_targets(lab, parts)


def test_mlp_backward_matches_finite_differences():
    mlp, params, X, T = _mlp_small()
    grads = mlp.backward(params, X, T)
    h = 1e-6
    for pi, (w, g) in enumerate(zip(params, grads)):
        flat = w.reshape(-1)
        num = np.zeros_like(flat)
        for i in range(flat.size):
            old = flat[i]
            flat[i] = old + h
            lp = mlp.loss(params, X, T)
            flat[i] = old - h
            lm = mlp.loss(params, X, T)
            flat[i] = old
            num[i] = (lp - lm) / (2 * h)
        np.testing.assert_allclose(g.reshape(-1), num, rtol=1e-5, atol=1e-8, err_msg=f"param {pi}")


def test_mlp_loss_and_gradient_invariants():
    mlp, params, X, T = _mlp_small(seed=3)
    np.testing.assert_allclose(T.sum(axis=1), 1.0)
    assert mlp.loss(params, X, T) > 0
    grads = mlp.backward(params, X, T)
    # softmax gradients sum to zero over the partitions for every row
    assert abs(grads[5].sum()) < 1e-12
    # uniform logits: loss = log P whatever the targets
    zero = [np.zeros_like(p) for p in params]
    np.testing.assert_allclose(mlp.loss(zero, X, T), np.log(11), rtol=1e-12)


def test_adam_first_step_is_sign_step():
    mlp, params, X, T = _mlp_small(seed=4)
    grads = mlp.backward(params, X, T)
    state = [(np.zeros_like(p), np.zeros_like(p)) for p in params]
    new = mlp.adam_step(params, grads, state, lr=1e-3, step=1)
    for w0, w1, g in zip(params, new, grads):
        big = np.abs(g) > 1e-4
        np.testing.assert_allclose((w1 - w0)[big], -1e-3 * np.sign(g[big]), rtol=1e-3)


def test_top_partitions_brute_force():
    mlp, params, X, T = _mlp_small(seed=5, parts=40, n=30)
    order, mass = mlp.top_partitions(params, X, 6)
    _, z = mlp.forward(params, X)
    p = np.exp(mlp.log_softmax(z))
    for i in range(X.shape[0]):
        ranked = sorted(range(40), key=lambda j: (-z[i, j], j))[:6]
        assert order[i].tolist() == ranked
        assert mass[i] == pytest.approx(sum(p[i, j] for j in ranked), rel=1e-12)


# ---------------------------------------------------------------------------
# Routed form: candidate-set kNN, k-means partitions, BF16 emulation.
# ---------------------------------------------------------------------------

def test_knn_subset_reduces_to_knn_and_to_sub_problems():
    from oracle import knn, knn_subset

    rng = np.random.default_rng(3)
    X = rng.standard_normal((120, 6)).astype(np.float32)
    n = X.shape[0]
    # every row a candidate: the plain exact kNN
    off = np.arange(n + 1, dtype=np.int64) * n
    ids = np.tile(np.arange(n, dtype=np.int64), n)
    a = knn_subset(X, 7, off, ids)
    b = knn(X, 7)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    # candidates = a fixed subset S (plus self): kNN of X[S ∪ {q}] mapped back
    S = np.sort(rng.choice(n, 40, replace=False))
    off = np.arange(n + 1, dtype=np.int64) * S.size
    idx, d2, _ = knn_subset(X, 5, off, np.tile(S, n))
    for q in range(0, n, 7):
        rows = np.union1d(S, [q])
        sub_i, sub_d2, _ = knn(X[rows], 5, Q=X[q:q + 1], self_ids=np.searchsorted(rows, [q]))
        assert np.array_equal(rows[sub_i[0]], idx[q]) and np.array_equal(sub_d2[0], d2[q])
    # fewer candidates than k: padded with -1 / inf
    off = np.zeros(n + 1, dtype=np.int64)
    off[1:] = 2
    off = np.cumsum(off)
    ids = np.tile(np.array([0, 1], dtype=np.int64), n)
    idx, d2, _ = knn_subset(X, 5, off, ids)
    assert (idx[5, 3:] == -1).all() and np.isinf(d2[5, 3:]).all()
    assert idx[0, 0] == 0 and idx[0, 1] == 1 and idx[0, 2] == -1


def test_kmeans_matches_sklearn_lloyd():
    from sklearn.cluster import KMeans

    from oracle import partition

    rng = np.random.default_rng(11)
    centres = rng.normal(0, 6, size=(12, 5))
    X = (centres[rng.integers(0, 12, 1500)] + rng.standard_normal((1500, 5))).astype(np.float32)
    init = rng.choice(1500, 12, replace=False)
    for iters in (1, 3, 10):
        C, labels, relocated = partition.kmeans(X, init, iters)
        assert relocated == 0
        km = KMeans(n_clusters=12, init=X[init].astype(np.float64), n_init=1, max_iter=iters, tol=0.0,
                    algorithm="lloyd").fit(X.astype(np.float64))
        assert np.array_equal(labels, km.labels_)
        np.testing.assert_allclose(C, km.cluster_centers_, rtol=1e-6, atol=1e-6)


def test_kmeans_relocates_empty_partition_by_hand():
    from oracle import partition

    # 1-D rows 0, 0, 5, 5.5, 6 with initial centroids rows 0, 1, 2 = (0, 0, 5):
    # rows 0 and 1 tie between centroids 0 and 1 and go to 0 (lower index),
    # centroid 1 is empty and takes the farthest row from its centroid: row 4
    # (distance 1 to centroid 5).  New centroids: mean(0, 0) = 0, 6,
    # mean(5, 5.5) = 5.25; final labels 0, 0, 2, 2, 1.
    X = np.array([[0.0], [0.0], [5.0], [5.5], [6.0]], dtype=np.float32)
    C, labels, relocated = partition.kmeans(X, np.array([0, 1, 2]), 1)
    assert relocated == 1
    assert np.array_equal(C[:, 0], np.array([0.0, 6.0, 5.25], dtype=np.float32))
    assert labels.tolist() == [0, 0, 2, 2, 1]


def test_kmeans_mean_is_correctly_rounded():
    from oracle import partition

    # values whose float32 sum loses bits: mean of 1 + 2^-23 (x3) and 1 is
    # 1 + 0.75 * 2^-23, correctly rounded to 1 + 2^-23
    v = np.array([1 + 2**-23, 1 + 2**-23, 1 + 2**-23, 1.0], dtype=np.float32)
    C = partition.centroid_means(v[:, None], np.zeros(4, dtype=np.int32), 1, np.zeros((1, 1), np.float32))
    assert C[0, 0] == np.float32(1 + 2**-23)


def test_inverted_lists_brute_force():
    from oracle import partition

    rng = np.random.default_rng(5)
    labels = rng.integers(0, 9, 300).astype(np.int32)
    labels[labels == 4] = 3  # an empty partition
    off, perm = partition.inverted_lists(labels, 9)
    for p in range(9):
        assert perm[off[p]:off[p + 1]].tolist() == [i for i in range(300) if labels[i] == p]
    assert off[4] == off[5]


def test_routed_knn_special_cases():
    from oracle import knn, partition

    rng = np.random.default_rng(8)
    X = rng.standard_normal((200, 4)).astype(np.float32)
    labels = rng.integers(0, 6, 200).astype(np.int32)
    off, perm = partition.inverted_lists(labels, 6)
    exact = knn(X, 6)
    all_probes = np.tile(np.arange(6, dtype=np.int32), (200, 1))
    a = partition.routed_knn(X, 6, off, perm, all_probes)
    assert np.array_equal(a[0], exact[0])
    own = labels[:, None].copy()
    b = partition.routed_knn(X, 6, off, perm, own, exact_rows=np.arange(200) % 2 == 0)
    assert np.array_equal(b[0][::2], exact[0][::2])
    for q in range(1, 200, 2):  # own partition only: brute force within it
        members = [j for j in range(200) if labels[j] == labels[q] and j != q]
        d2 = [float(np.sum((X[q].astype(np.float64) - X[j].astype(np.float64)) ** 2)) for j in members]
        best = [members[i] for i in np.lexsort((members, d2))[:5]]
        got = [j for j in b[0][q, 1:] if j >= 0]
        assert got == best
    assert partition.recall(a[0], exact[0]) == 1.0


def test_bf16_round_matches_torch():
    import torch

    from oracle.mlp import bf16_round

    rng = np.random.default_rng(2)
    x = np.concatenate([rng.standard_normal(5000) * 10 ** rng.uniform(-30, 30, 5000),
                        # exact halfway cases: low 16 bits 0x8000, both parities
                        (np.arange(1, 200, dtype=np.uint32) << 16 | 0x8000).view(np.float32).astype(np.float64),
                        [0.0, -0.0, np.inf, -np.inf]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(bf16_round(x), ref)


def test_bf16_emulation_reduces_to_exact_and_stays_close():
    from oracle import mlp

    rng = np.random.default_rng(4)
    d, H, P, n, m = 6, 64, 64, 40, 3
    params = mlp.init_params(d, H, P, seed=1)
    params = [p + (0.05 * rng.standard_normal(p.shape) if p.ndim == 1 else 0) for p in params]
    X = rng.standard_normal((n, d))
    t = mlp.soft_targets(rng.integers(0, P, (n, m)), P)
    exact = mlp.backward(params, X, t)
    plain = mlp.backward_bf16(params, X, t, rounding=False)
    for a, b in zip(exact, plain):
        assert np.array_equal(a, b)
    assert np.array_equal(mlp.forward_bf16(params, X, rounding=False)[1], mlp.forward(params, X)[1])
    # each bfloat16 rounding moves a value by at most 2^-9 relative; about ten
    # of them compound along the path to dW1 (inputs, three weights, two
    # activations, three errors), so the gradients stay within 2^-4
    rounded = mlp.backward_bf16(params, X, t)
    for a, b in zip(exact, rounded):
        assert np.linalg.norm(a - b) <= 2**-4 * np.linalg.norm(a)
        assert np.linalg.norm(a - b) > 0


# ---------------------------------------------------------------------------
# Cosine metric.
# ---------------------------------------------------------------------------

def test_cosine_knn_matches_sklearn_and_cdist():
    from scipy.spatial.distance import cdist
    from sklearn.neighbors import NearestNeighbors

    from oracle import knn

    rng = np.random.default_rng(21)
    X = (rng.standard_normal((400, 12)) + rng.normal(0, 3, (1, 12))).astype(np.float32)
    idx, d, dist = knn(X, 9, metric="cosine")
    D = cdist(X.astype(np.float64), X.astype(np.float64), metric="cosine")
    np.fill_diagonal(D, -1.0)  # self first
    order = np.lexsort((np.broadcast_to(np.arange(400), D.shape), D), axis=1)[:, :9]
    assert np.array_equal(idx, order)
    Dk = np.take_along_axis(D, order, axis=1)
    np.testing.assert_allclose(d[:, 1:], Dk[:, 1:], rtol=0, atol=1e-14)
    assert (d[:, 0] == 0).all()
    nn = NearestNeighbors(n_neighbors=9, metric="cosine", algorithm="brute").fit(X.astype(np.float64))
    sd, si = nn.kneighbors(X.astype(np.float64))
    assert np.array_equal(np.sort(si[:, 1:], axis=1), np.sort(idx[:, 1:], axis=1))
    np.testing.assert_allclose(np.sort(sd[:, 1:], axis=1), d[:, 1:], atol=1e-12)


def test_cosine_knn_hand_angles_scale_invariance_and_zero_rows():
    from oracle import knn

    # x = (1, 0): (2, 0) at 0, (1, 1) at 1 - 1/sqrt(2), (0, 1) at 1, (-1, 0) at 2
    R = np.array([[2, 0], [-1, 0], [0, 1], [1, 1]], dtype=np.float32)
    idx, d, _ = knn(R, 4, Q=np.array([[1, 0]], dtype=np.float32))
    idx_c, d_c, _ = knn(R, 4, Q=np.array([[1, 0]], dtype=np.float32), metric="cosine")
    assert idx_c[0].tolist() == [0, 3, 2, 1]
    np.testing.assert_allclose(d_c[0], [0.0, 1 - 2 ** -0.5, 1.0, 2.0], atol=1e-15)
    # scaling rows by powers of two changes nothing (exact in float32)
    rng = np.random.default_rng(5)
    X = rng.standard_normal((150, 7)).astype(np.float32)
    S = X * (2.0 ** rng.integers(-6, 7, size=(150, 1))).astype(np.float32)
    a = knn(X, 6, metric="cosine")
    b = knn(S, 6, metric="cosine")
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    # a zero row is at distance 1 from every row, and every row from it
    X[10] = 0.0
    idx, d, _ = knn(X, 150, metric="cosine")
    assert idx[10, 0] == 10 and (d[10, 1:] == 1.0).all()
    assert idx[10, 1:].tolist() == [j for j in range(150) if j != 10]  # all ties: index order
    pos = np.argwhere(idx[3] == 10)[0, 0]
    assert d[3, pos] == 1.0


# ---------------------------------------------------------------------------
# Energy distance between groups of cells (Methods, "Perturbation distance
# computation").
# ---------------------------------------------------------------------------

def _ed_groups(sizes, d, seed, shuffle=True):
    rng = np.random.default_rng(seed)
    n = int(sum(sizes))
    X = (rng.standard_normal((n, d)) * rng.uniform(0.5, 2.0, d)).astype(np.float32)
    labels = np.repeat(np.arange(len(sizes)), sizes)
    if shuffle:
        labels = rng.permutation(labels)
    return X, labels


def test_edistance_sums_match_cdist_brute_force():
    import math

    from scipy.spatial.distance import cdist

    from oracle import edistance as ed

    sizes = [1, 2, 7, 30, 0, 45, 3]
    X, labels = _ed_groups(sizes, 9, seed=3)
    off, cells = ed.groups_from_labels(labels, G=len(sizes))
    # cells of a group need not be ascending: reverse every group's list
    cells = np.concatenate([cells[off[g]:off[g + 1]][::-1] for g in range(len(sizes))]).astype(np.int32)
    pairs = ed.all_pairs(len(sizes))
    s = ed.sums(X, off, cells, pairs)
    Xd = X.astype(np.float64)
    for (a, b), v in zip(pairs, s):
        A = Xd[labels == a]
        B = Xd[labels == b]
        if A.size == 0 or B.size == 0:
            assert v == 0.0
            continue
        C = cdist(A, B)
        ref = math.fsum(np.triu(C, 1).ravel()) if a == b else math.fsum(C.ravel())
        assert abs(v - ref) <= 1e-12 * max(ref, 1.0), (a, b, v, ref)


def test_edistance_matches_scipy_energy_distance_in_one_dimension():
    from scipy.stats import energy_distance

    from oracle import edistance as ed

    rng = np.random.default_rng(8)
    u = rng.standard_normal(40).astype(np.float32)
    v = (rng.standard_normal(25) * 1.5 + 0.7).astype(np.float32)
    X = np.concatenate([u, v])[:, None]
    off = np.array([0, 40, 65], dtype=np.int64)
    cells = np.arange(65, dtype=np.int32)
    E, D = ed.pairwise(X, off, cells)
    # scipy's statistic uses all n^2 within pairs (the i = i' zeros included):
    # its square is 2 d_ab - d_aa (n_a - 1)/n_a - d_bb (n_b - 1)/n_b
    ev = 2 * D[0, 1] - D[0, 0] * 39 / 40 - D[1, 1] * 24 / 25
    assert abs(ev - energy_distance(u.astype(np.float64), v.astype(np.float64)) ** 2) <= 1e-12
    assert E[0, 1] == E[1, 0] and E[0, 0] == 0.0 and E[1, 1] == 0.0


def test_edistance_closed_form_on_lattices():
    from oracle import edistance as ed

    # A = {0, h, ..., (m-1) h} on a line, B = A + L with L >= m h:
    # within mean h (m + 1) / 3, cross mean L, E = 2 L - 2 h (m + 1) / 3
    m, h, L = 24, 0.5, 40.0
    X = np.zeros((2 * m, 4), dtype=np.float32)
    X[:m, 1] = np.arange(m) * h
    X[m:, 1] = np.arange(m) * h + L
    off = np.array([0, m, 2 * m], dtype=np.int64)
    E, D = ed.pairwise(X, off, np.arange(2 * m, dtype=np.int32))
    assert D[0, 0] == D[1, 1] == h * (m + 1) / 3
    assert D[0, 1] == L
    assert abs(E[0, 1] - (2 * L - 2 * h * (m + 1) / 3)) <= 1e-14 * 2 * L


def test_edistance_special_cases_and_invariances():
    from oracle import edistance as ed

    # two singletons: no within pairs (skipped), E = 2 |x - y|
    X = np.array([[0, 0], [3, 4]], dtype=np.float32)
    E, D = ed.pairwise(X, np.array([0, 1, 2], dtype=np.int64), np.array([0, 1], dtype=np.int32))
    assert D[0, 0] == 0 and D[1, 1] == 0 and E[0, 1] == 10.0
    # an empty group: its cross means are NaN, its within mean is skipped
    E, D = ed.pairwise(X, np.array([0, 1, 1, 2], dtype=np.int64), np.array([0, 1], dtype=np.int32))
    assert np.isnan(D[0, 1]) and np.isnan(E[0, 1]) and D[1, 1] == 0 and E[0, 2] == 10.0
    # integer coordinates: translation and power-of-two scaling are exact
    sizes = [5, 9, 14, 2]
    rng = np.random.default_rng(4)
    Xi = rng.integers(-20, 20, size=(30, 6)).astype(np.float32)
    off, cells = ed.groups_from_labels(rng.permutation(np.repeat(np.arange(4), sizes)), G=4)
    E1, _ = ed.pairwise(Xi, off, cells)
    E2, _ = ed.pairwise(Xi + np.float32(64), off, cells)
    E3, _ = ed.pairwise(Xi * np.float32(8), off, cells)
    np.testing.assert_allclose(E2, E1, rtol=1e-13, atol=1e-12)
    np.testing.assert_allclose(E3, 8 * E1, rtol=1e-13, atol=1e-12)
    assert np.array_equal(E1, E1.T) and (np.diag(E1) == 0).all()
    # one-sided distances are the reference group's row of the pairwise matrix
    # (a cross sum taken as (ref, g) rather than (g, ref) adds in another order)
    for ref in range(4):
        np.testing.assert_allclose(ed.onesided(Xi, off, cells, ref), E1[ref], rtol=1e-13, atol=1e-13)


# ---------------------------------------------------------------------------
# Sparse PCA (Methods, "Principal component analysis").
# ---------------------------------------------------------------------------

def _small_csr(n=300, p=40, density=0.2, seed=1):
    import synth

    return synth.sparse_expression(n=n, p=p, density=density, seed=seed)


def test_pca_covariance_matches_numpy_cov_and_scipy_gram():
    import scipy.sparse as sp

    from oracle import pca as opca

    ip, ix, v = _small_csr()
    X = sp.csr_matrix((v.astype(np.float64), ix, ip), shape=(300, 40))
    mu, S = opca.gram(ip, ix, v, 40)
    np.testing.assert_allclose(S, (X.T @ X).toarray(), rtol=1e-13, atol=1e-12)
    np.testing.assert_allclose(mu, np.asarray(X.mean(axis=0)).ravel(), rtol=1e-13, atol=1e-15)
    mu2, C = opca.covariance(ip, ix, v, 40)
    np.testing.assert_allclose(C, np.cov(X.toarray(), rowvar=False), rtol=1e-10, atol=1e-12)
    assert np.array_equal(C, C.T)


def test_pca_matches_sklearn_full_pca():
    from sklearn.decomposition import PCA

    from oracle import pca as opca

    ip, ix, v = _small_csr(n=500, p=30, seed=2)
    Xd = opca.dense(ip, ix, v, 30)
    mu, C, ev, V, Z = opca.pca(ip, ix, v, 30, 8)
    skl = PCA(n_components=8, svd_solver="full").fit(Xd)
    np.testing.assert_allclose(ev, skl.explained_variance_, rtol=1e-9)
    Zs = skl.transform(Xd)
    for t in range(8):  # loadings and scores agree up to the sign of each component
        s = np.sign(V[:, t] @ skl.components_[t])
        np.testing.assert_allclose(V[:, t], s * skl.components_[t], atol=1e-9)
        np.testing.assert_allclose(Z[:, t], s * Zs[:, t], atol=1e-8)
    assert (np.abs(V).argmax(0) == np.abs(V).argmax(0)).all()
    assert all(V[np.abs(V[:, t]).argmax(), t] > 0 for t in range(8))  # the sign rule


def test_pca_closed_forms():
    from oracle import pca as opca

    # genes 0 and 1 always equal, gene 2 independent: the covariance has rank
    # 2 and one eigenvector is (1, -1, 0)/sqrt(2) with eigenvalue 0
    rng = np.random.default_rng(3)
    a = rng.integers(1, 5, 200).astype(np.float32)
    c = rng.integers(1, 5, 200).astype(np.float32)
    ip = np.arange(0, 601, 3, dtype=np.int64)
    ix = np.tile(np.array([0, 1, 2], dtype=np.int32), 200)
    v = np.stack([a, a, c], axis=1).ravel()
    mu, C, ev, V, Z = opca.pca(ip, ix, v, 3, 3)
    a64, c64 = a.astype(np.float64), c.astype(np.float64)
    va, vc = np.var(a64, ddof=1), np.var(c64, ddof=1)
    cac = ((a64 - a64.mean()) * (c64 - c64.mean())).sum() / 199
    # on (1, 1, 0)/sqrt(2) and (0, 0, 1) the covariance is [[2 va, sqrt2 cac], [sqrt2 cac, vc]]
    tr, det = 2 * va + vc, 2 * va * vc - 2 * cac * cac
    disc = np.sqrt(tr * tr / 4 - det)
    np.testing.assert_allclose(sorted(ev), [0.0, tr / 2 - disc, tr / 2 + disc], atol=1e-12)
    zero = int(np.argmin(np.abs(ev)))
    np.testing.assert_allclose(np.abs(V[:, zero]), [2 ** -0.5, 2 ** -0.5, 0.0], atol=1e-12)
    # scores are centred: every column of Z sums to 0
    np.testing.assert_allclose(Z.sum(0), 0.0, atol=1e-9)
    # an empty row is a cell of zeros: its score is -mu^T V
    ip2 = np.concatenate([ip, [600]])
    _, _, _, V2, Z2 = opca.pca(ip2, ix, v, 3, 3)
    mu2 = np.concatenate([np.stack([a, a, c], 1).astype(np.float64), np.zeros((1, 3))]).mean(0)
    np.testing.assert_allclose(Z2[-1], -(mu2 @ V2), atol=1e-12)


# ---------------------------------------------------------------------------
# UMAP layout (the method's published loss, gradients and sampling; reading
# in oracle.c).
# ---------------------------------------------------------------------------

def test_splitmix64_published_value():
    from oracle import umap as ou

    # SplitMix64's first output from state 0 (the generator's published test value)
    assert ou.splitmix64_next(0) == 0xE220A8397B1DCDAF


def _two_points(w=1.0):
    ip = np.array([0, 1, 2], dtype=np.int64)
    ix = np.array([1, 0], dtype=np.int32)
    return ip, ix, np.array([w, w], dtype=np.float32)


def test_umap_attraction_is_the_gradient_of_minus_log_q():
    from oracle import umap as ou

    a, b = ou.fit_ab(0.5, 1.0)
    y0 = np.array([[0.3, -0.2], [1.4, 0.5]])  # d2 = 1.7 (not 1, where every power of d2 is 1)
    Y = ou.layout(*_two_points(), y0, n_epochs=2, a=a, b=b, neg=0)  # epoch 1 samples the edge, alpha 1/2

    def loss(yi):
        d2 = ((yi - y0[1]) ** 2).sum()
        return np.log1p(a * d2 ** b)  # -log q

    h = 1e-6
    grad = np.array([(loss(y0[0] + h * np.eye(2)[c]) - loss(y0[0] - h * np.eye(2)[c])) / (2 * h) for c in range(2)])
    np.testing.assert_allclose(Y[0] - y0[0], -0.5 * grad, rtol=1e-7)
    np.testing.assert_allclose(Y[1] - y0[1], 0.5 * grad, rtol=1e-7)  # the mirror move of the other row


def test_umap_repulsion_is_the_gradient_of_minus_log_one_minus_q():
    from oracle import umap as ou

    a, b, gamma = 1.2, 0.9, 1.5
    y0 = np.array([[0.0, 0.0], [6.0, 8.0], [30.0, 40.0]])  # distances 10 and 50: the 0.001 term is negligible
    # vertex 0 has one edge (to 1, weight 1); vertex 2 is only ever a negative sample
    ip = np.array([0, 1, 2, 2], dtype=np.int64)
    ix = np.array([1, 0], dtype=np.int32)
    w = np.array([1.0, 1.0], dtype=np.float32)
    Ya = ou.layout(ip, ix, w, y0, n_epochs=2, a=a, b=b, gamma=gamma, neg=0)
    Yr = ou.layout(ip, ix, w, y0, n_epochs=2, a=a, b=b, gamma=gamma, neg=1, seed=7)
    # which vertex the single negative of vertex 0 drew (epoch 1, edge 0, draw 0)
    st = (7 + ((1 << 40) + 0 * 64 + 0 + 1) * 0x9E3779B97F4A7C15) % (1 << 64)
    kk = (ou.splitmix64_next((st - 0x9E3779B97F4A7C15) % (1 << 64)) >> 11) % 3
    rep = Yr[0] - Ya[0]
    if kk == 0:
        assert np.all(rep == 0)
        return
    yk = y0[kk]

    def loss(yi):
        d2 = ((yi - yk) ** 2).sum()
        q = 1.0 / (1.0 + a * d2 ** b)
        return -gamma * np.log(1.0 - q)

    h = 1e-5
    grad = np.array([(loss(y0[0] + h * np.eye(2)[c]) - loss(y0[0] - h * np.eye(2)[c])) / (2 * h) for c in range(2)])
    np.testing.assert_allclose(rep, -0.5 * grad, rtol=1e-4)


def test_umap_schedule_translation_and_clipping():
    from oracle import umap as ou

    a, b = ou.fit_ab(0.5, 1.0)
    # a weak edge (weight 1/3 of the strongest) moves its rows only at epochs 3, 6, ...
    # rows: 0 -> {1 (w 1), 2 (w 1/3)}, 1 -> {0 (w 1)}, 2 -> {0 (w 1)}, 3 -> {2 (w 1/3)}
    ip = np.array([0, 2, 3, 4, 5], dtype=np.int64)
    ix = np.array([1, 2, 0, 0, 2], dtype=np.int32)
    w = np.array([1.0, 1.0 / 3, 1.0, 1.0, 1.0 / 3], dtype=np.float32)
    y0 = np.array([[0.0, 0.0], [2.0, 0.0], [0.0, 3.0], [5.0, 5.0]])
    moves = []
    for T in range(1, 8):
        Y = ou.layout(ip, ix, w, y0, n_epochs=T, a=a, b=b, neg=0)
        moves.append(Y[3].copy())
    # row 3 holds only the weak edge (3 -> 2): still at y0 until an epoch t >= 3 has run
    assert np.array_equal(moves[0], y0[3]) and np.array_equal(moves[2], y0[3]) and not np.array_equal(moves[3], y0[3])
    # translation by an exact offset moves every result by the same offset
    Yt = ou.layout(ip, ix, w, y0 + 1024.0, n_epochs=6, a=a, b=b, neg=2, seed=3)
    Yu = ou.layout(ip, ix, w, y0, n_epochs=6, a=a, b=b, neg=2, seed=3)
    np.testing.assert_allclose(Yt - 1024.0, Yu, atol=1e-9)
    # coincident points: the attraction is 0 and no step exceeds 4 alpha per coordinate
    Yc = ou.layout(*_two_points(), np.zeros((2, 2)), n_epochs=2, a=a, b=b, neg=0)
    assert np.array_equal(Yc, np.zeros((2, 2)))


def _draws(seed, t, e, neg, n, stride=64):
    """The vertices the negatives of edge e draw in epoch t (the counter-based
    SplitMix64 of the reading, through the pinned generator)."""
    from oracle import umap as ou

    g = 0x9E3779B97F4A7C15
    out = []
    for p in range(neg):
        st = (seed + (t * (1 << 40) + e * stride + p + 1) * g) % (1 << 64)
        out.append((ou.splitmix64_next((st - g) % (1 << 64)) >> 11) % n)
    return out


def test_umap_negative_draws_follow_the_counter_and_never_repeat_a_counter():
    # the oracle's draw function is the pinned generator at the reading's counter
    from oracle import umap as ou

    for seed, t, e, n in [(0, 0, 0, 7), (3, 5, 11, 1000), (2**63 + 5, 199, 2**31 + 3, 2**31 - 1)]:
        assert [ou.negative(seed, t, e, p, n) for p in range(64)] == _draws(seed, t, e, 64, n)
    # with 64 draws per edge, the draws of neighbouring edges share no counter:
    # over 40 edges x 64 draws into 2^31 - 1 vertices every draw is distinct
    # (a stride of 16 per edge would make draws 16..63 of edge e repeat draws
    # 0..47 of edge e + 1)
    n = 2**31 - 1
    draws = [ou.negative(9, 4, e, p, n) for e in range(40) for p in range(64)]
    assert len(set(draws)) == len(draws)
    assert _draws(9, 4, 0, 64, n, stride=16)[16:] == _draws(9, 4, 1, 64, n, stride=16)[:48]


def test_umap_layout_draws_of_a_later_edge_use_the_full_stride():
    # vertex 1's only edge is edge 1 (the second CSR entry); with an enormous
    # repulsion strength every draw of vertex 0 by that edge's 64 negatives
    # pushes vertex 1 by 4 alpha = 2 (epoch 1) along +x, away from vertex 0
    from oracle import umap as ou

    seed, neg = 21, 64
    hits = sum(k == 0 for k in _draws(seed, 1, 1, neg, 2))
    hits16 = sum(k == 0 for k in _draws(seed, 1, 1, neg, 2, stride=16))
    assert hits != hits16  # the case tells the two strides apart
    y0 = np.array([[0.0, 0.0], [1.0, 0.0]])
    Ya = ou.layout(*_two_points(), y0, n_epochs=2, a=1.0, b=1.0, neg=0)
    Yr = ou.layout(*_two_points(), y0, n_epochs=2, a=1.0, b=1.0, gamma=1e6, neg=neg, seed=seed)
    np.testing.assert_allclose(Yr[1] - Ya[1], [2.0 * hits, 0.0], rtol=0, atol=1e-12)


def test_umap_self_draws_are_skipped():
    # a lone vertex with a self-loop: the attraction has d2 = 0 and every
    # negative sample draws the vertex itself, which UMAP skips: it never moves
    from oracle import umap as ou

    y0 = np.array([[1.5, -2.5]])
    Y = ou.layout(np.array([0, 1], np.int64), np.array([0], np.int32), np.ones(1, np.float32), y0, n_epochs=5,
                  a=1.0, b=1.0, neg=6, seed=4)
    assert np.array_equal(Y, y0)


def test_umap_repulsion_is_regularised_near_coincidence():
    # two vertices 1e-9 apart: the repulsion coefficient stays finite (its
    # 0.001 regulariser), so the move is of the order of the separation; an
    # unregularised coefficient would clip every such move to 4 alpha
    from oracle import umap as ou

    seed, neg = 11, 8
    hits = sum(k == 1 for k in _draws(seed, 1, 0, neg, 2))  # draws of vertex 0 that hit vertex 1 in epoch 1
    assert hits > 0
    y0 = np.array([[0.0, 0.0], [1e-9, 0.0]])
    Y = ou.layout(*_two_points(), y0, n_epochs=2, a=1.0, b=1.0, neg=neg, seed=seed)
    assert 0 < np.abs(Y[0] - y0[0]).max() < 1e-4


def test_umap_coincident_points_are_pushed_by_four_alpha():
    # UMAP's rule for a negative sample at the vertex's own position: a push
    # of 4 alpha per coordinate.  Two distinct vertices at the origin, epoch 1
    # (alpha 1/2): vertex 0 moves by 2 per coordinate for every draw of vertex 1
    from oracle import umap as ou

    seed, neg = 5, 6
    hits = sum(k == 1 for k in _draws(seed, 1, 0, neg, 2))
    assert 0 < hits < neg
    Y = ou.layout(*_two_points(), np.zeros((2, 2)), n_epochs=2, a=1.0, b=1.0, neg=neg, seed=seed)
    np.testing.assert_array_equal(Y[0], [2.0 * hits, 2.0 * hits])


def test_umap_moves_are_clipped_at_four():
    # an enormous repulsion strength: each repulsive move is clipped to 4 alpha
    # away from the drawn vertex (alpha 1/2 in epoch 1)
    from oracle import umap as ou

    seed, neg = 5, 6
    hits = sum(k == 1 for k in _draws(seed, 1, 0, neg, 2))
    y0 = np.array([[0.0, 0.0], [1.0, 0.0]])
    Ya = ou.layout(*_two_points(), y0, n_epochs=2, a=1.0, b=1.0, neg=0)
    Yr = ou.layout(*_two_points(), y0, n_epochs=2, a=1.0, b=1.0, gamma=1e6, neg=neg, seed=seed)
    np.testing.assert_allclose(Yr[0] - Ya[0], [-2.0 * hits, 0.0], rtol=0, atol=1e-12)


# ---------------------------------------------------------------------------
# Leiden communities (modularity by its definition, known optima, the
# algorithm's connectivity guarantee, invariances of the fixed-point reading;
# reading in leiden.c).
# ---------------------------------------------------------------------------

def _csr(A):
    import scipy.sparse as sp

    M = sp.csr_matrix(np.asarray(A, dtype=np.float64))
    M.sort_indices()
    return M.indptr.astype(np.int64), M.indices.astype(np.int32), M.data.astype(np.float32)


def _cliques(sizes, bridges):
    n = sum(sizes)
    A = np.zeros((n, n))
    off = np.cumsum([0] + list(sizes))
    for a, b in zip(off[:-1], off[1:]):
        A[a:b, a:b] = 1.0
    np.fill_diagonal(A, 0.0)
    for i, j in bridges:
        A[i, j] = A[j, i] = 1.0
    return A


def _modularity_dense(A, labels, gamma):
    # Q = 1/(2m) sum_ij (A_ij - gamma k_i k_j / 2m) [c_i = c_j]
    A = np.asarray(A, dtype=np.float64)
    k = A.sum(1)
    two_m = k.sum()
    same = labels[:, None] == labels[None, :]
    return float(((A - gamma * np.outer(k, k) / two_m) * same).sum() / two_m)


def _same_partition(a, b):
    # equal up to renaming the communities
    pairs = set(zip(a.tolist(), b.tolist()))
    return len(pairs) == len(set(a.tolist())) == len(set(b.tolist()))


def test_leiden_modularity_matches_its_definition():
    from oracle import leiden as ol

    rng = np.random.default_rng(3)
    for n, p, gamma in [(30, 0.2, 1.0), (60, 0.1, 0.5), (80, 0.05, 2.0)]:
        # weights on a binary grid of 1/8: exact in the fixed point, so the
        # reported modularity is the dense formula's to rounding
        W = np.triu((rng.random((n, n)) < p) * rng.integers(1, 9, (n, n)) / 8.0, 1)
        A = W + W.T
        lab, q, _ = ol.leiden(*_csr(A), gamma=gamma)
        assert abs(q - _modularity_dense(A, lab, gamma)) < 1e-12
        # the result is no worse than every vertex alone or one community per component
        from scipy.sparse.csgraph import connected_components

        _, comp = connected_components(A != 0, directed=False)
        assert q >= _modularity_dense(A, np.arange(n), gamma) - 1e-12
        assert q >= _modularity_dense(A, comp, gamma) - 1e-12


def test_leiden_two_cliques_and_a_ring_of_cliques():
    from oracle import leiden as ol

    lab, _, _ = ol.leiden(*_csr(_cliques([5, 5], [(0, 5)])))
    assert lab.tolist() == [0] * 5 + [1] * 5
    sizes = [5] * 6
    off = np.cumsum([0] + sizes)
    A = _cliques(sizes, [(off[i], off[(i + 1) % 6] + 1) for i in range(6)])
    lab, q, _ = ol.leiden(*_csr(A))
    assert lab.tolist() == sum([[c] * 5 for c in range(6)], [])
    # one clique per community: In = 20 each, Tot = 22 each, 2m = 132
    assert abs(q - 6 * (20 / 132 - (22 / 132) ** 2)) < 1e-12


def test_leiden_recovers_a_planted_partition():
    from oracle import leiden as ol

    rng = np.random.default_rng(0)
    blocks = np.repeat(np.arange(4), 50)
    P = np.where(blocks[:, None] == blocks[None, :], 0.5, 0.01)
    A = np.triu(rng.random((200, 200)) < P, 1).astype(float)
    A = A + A.T
    lab, _, _ = ol.leiden(*_csr(A))
    assert _same_partition(lab, blocks)


def test_leiden_communities_are_connected_and_gamma_limits():
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components

    import oracle
    from oracle import leiden as ol

    X = synth.mixture(2000, d=50, n_clusters=12, seed=41)
    g = oracle.knn_graph(X, 15)
    M = sp.csr_matrix((g["data"], g["indices"], g["indptr"]))
    lab, q, levels = ol.leiden(g["indptr"], g["indices"], g["data"])
    assert levels >= 2 and q > 0.5
    for c in np.unique(lab):
        rows = np.where(lab == c)[0]
        assert connected_components(M[rows][:, rows], directed=False)[0] == 1, f"community {c} is disconnected"
    # labels numbered by first appearance
    first = [int(lab[np.where(lab == c)[0][0]]) for c in np.unique(lab)]
    assert lab[0] == 0 and sorted(first) == list(range(len(first)))
    order = [lab[np.where(lab == c)[0][0]] for c in sorted(np.unique(lab), key=lambda c: np.where(lab == c)[0][0])]
    assert order == list(range(len(order)))
    # a vanishing resolution merges each connected component into one community
    ncomp, comp = connected_components(M, directed=False)
    lab0, _, _ = ol.leiden(g["indptr"], g["indices"], g["data"], gamma=1e-7)
    assert _same_partition(lab0, comp)
    # a huge resolution leaves every vertex alone
    labh, _, _ = ol.leiden(g["indptr"], g["indices"], g["data"], gamma=1e6)
    assert labh.tolist() == list(range(2000))


def test_leiden_fixed_point_invariances():
    from oracle import leiden as ol

    import oracle

    X = synth.mixture(1500, d=50, n_clusters=8, seed=7)
    g = oracle.knn_graph(X, 15)
    ip, ix, w = g["indptr"], g["indices"], g["data"]
    lab, q, _ = ol.leiden(ip, ix, w)
    # scaling every weight by a power of two moves the fixed-point exponent
    # by the same amount: the integers, and so the labels, are unchanged
    assert ol.scale(len(ix), float(w.max()) * 8) == ol.scale(len(ix), float(w.max())) - 3
    lab8, q8, _ = ol.leiden(ip, ix, (w * np.float32(8)).astype(np.float32))
    assert np.array_equal(lab, lab8) and q8 == q
    # the order of the columns within a row does not matter (every sum is exact)
    rng = np.random.default_rng(5)
    ix2, w2 = ix.copy(), w.copy()
    for i in range(len(ip) - 1):
        p = rng.permutation(ip[i + 1] - ip[i]) + ip[i]
        ix2[ip[i]:ip[i + 1]] = ix[p]
        w2[ip[i]:ip[i + 1]] = w[p]
    lab2, _, _ = ol.leiden(ip, ix2, w2)
    assert np.array_equal(lab, lab2)


def test_leiden_degenerate_graphs():
    from oracle import leiden as ol

    # no edges: every vertex alone
    lab, q, _ = ol.leiden(np.zeros(6, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32))
    assert lab.tolist() == list(range(5)) and q == 0.0
    # isolated vertices beside two cliques keep their own communities
    A = np.zeros((13, 13))
    A[:10, :10] = _cliques([5, 5], [(0, 5)])
    lab, _, _ = ol.leiden(*_csr(A))
    assert lab.tolist() == [0] * 5 + [1] * 5 + [2, 3, 4]
    with pytest.raises(ValueError):
        ol.leiden(*_csr(A), gamma=0.0)


def test_leiden_refinement_by_hand():
    """The refinement step on a 6-vertex graph, derived by hand from the
    reading.  Edges: triangle 0-1-2 (weight 1), 0-3 (1), 3-4 (3), 4-5 (1);
    communities C = {0, 1, 2, 3}, D = {4, 5}; gamma = 1.  Degrees k = (3, 2,
    2, 4, 4, 1), 2m = 16, Tot(C) = 11, Tot(D) = 5.
      Vertex 3 is not well connected to C: K(3, C - 3) = 1 < k3 (Tot(C) - k3)
      / 2m = 4 * 7 / 16 = 1.75, so it never joins (it could join {0} with
      gain 1 - 4 * 3 / 16 = 0.25 >= 0 otherwise).
      Round 1: 1 -> {0} (gain 1 - 2 * 3 / 16 = 0.625; {0} well connected:
      E = 3 >= 3 * 8 / 16); 2 prefers {1} (gain 1 - 2 * 2 / 16 = 0.75 over
      0.625 for {0}), but 1 moves in the same round, so 2's join is
      cancelled; 5 -> {4} (gain 1 - 1 * 4 / 16 = 0.75).
      Round 2: 2 -> {0, 1} (K = 2, gain 2 - 2 * 5 / 16 = 1.375; E({0, 1},
      C - {0, 1}) = 3 >= 5 * 6 / 16).  Round 3: no join.
    Refined: {0, 1, 2}, {3}, {4, 5}."""
    from oracle import leiden as ol

    A = np.zeros((6, 6))
    for i, j, w in [(0, 1, 1), (0, 2, 1), (1, 2, 1), (0, 3, 1), (3, 4, 3), (4, 5, 1)]:
        A[i, j] = A[j, i] = w
    R = ol.refine(*_csr(A), np.array([0, 0, 0, 0, 4, 4]))
    assert R.tolist() == [0, 0, 0, 3, 4, 4]
