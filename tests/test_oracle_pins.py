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
