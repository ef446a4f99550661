"""Parity of the HIP Leiden path (rsc_leiden, through the C ABI) with the
oracle: the same labels bit for bit and the same modularity on the same
graphs (the reading is deterministic, so any difference is an error)."""

import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rsc():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_02402_amd as rsc

    rsc.load()
    return rsc


def gpu_leiden(rsc, indptr, indices, data, gamma=1.0):
    import torch

    g = tuple(torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (indptr, indices, data))
    labels, st = rsc.leiden(g, gamma=gamma)
    torch.cuda.synchronize()
    assert st["sweeps"] >= st["levels"] and st["move_bytes"] >= 0
    return labels.cpu().numpy(), st["quality"], st["levels"], st["n_communities"]


def check(rsc, indptr, indices, data, label, gamma=1.0):
    from oracle import leiden as ol

    n = len(indptr) - 1
    log(f"[leiden parity] {label}: n={n} nnz={len(indices)} gamma={gamma}")
    lab_g, q_g, lv_g, nc_g = gpu_leiden(rsc, indptr, indices, data, gamma)
    lab_o, q_o, lv_o = ol.leiden(indptr, indices, data, gamma)
    diff = int((lab_g != lab_o).sum())
    log(f"  communities {nc_g} (oracle {lab_o.max() + 1}), levels {lv_g} (oracle {lv_o}), "
        f"modularity {q_g:.15f} (oracle {q_o:.15f}), labels differing {diff}")
    np.testing.assert_array_equal(lab_g, lab_o)
    assert q_g == q_o
    assert lv_g == lv_o
    assert nc_g == lab_o.max() + 1
    return lab_g, q_g


def csr_from_dense(W):
    n = W.shape[0]
    indptr = np.zeros(n + 1, dtype=np.int64)
    cols, vals = [], []
    for i in range(n):
        nz = np.nonzero(W[i])[0]
        cols.append(nz)
        vals.append(W[i, nz])
        indptr[i + 1] = indptr[i] + len(nz)
    return (indptr, np.concatenate(cols).astype(np.int32) if cols else np.zeros(0, np.int32),
            np.concatenate(vals).astype(np.float32) if vals else np.zeros(0, np.float32))


def test_mixture_10k_graph(rsc, oracle_mod):
    X = synth.workload("plain_10k")
    o = oracle_mod.knn_graph(X, 15)
    lab, q = check(rsc, o["indptr"], o["indices"], o["data"], "10k mixture kNN graph")
    assert q > 0.9


@pytest.mark.parametrize("gamma", [0.25, 0.5, 2.0, 4.0])
def test_resolutions(rsc, oracle_mod, gamma):
    X = synth.mixture(4000, d=50, n_clusters=12, seed=61)
    o = oracle_mod.knn_graph(X, 15)
    check(rsc, o["indptr"], o["indices"], o["data"], "4000-cell mixture", gamma=gamma)


def test_random_lists_with_hubs(rsc, oracle_mod):
    """kNN-shaped lists without cluster structure and ~1% hub rows (in-degree
    up to ~500): rows longer than a wave take the table path, and the levels
    run long."""
    idx, dist = synth.random_knn_lists(3000, 15, seed=62, hub_fraction=0.02)
    p, x, d, _, _ = oracle_mod.connectivities(idx, dist)
    assert (np.diff(p) > 64).any()
    check(rsc, p, x, d, "random kNN lists with hubs")


def test_hub_rows_beyond_the_lds_table(rsc, oracle_mod):
    """Hub rows of up to 830 entries: at the first level every neighbour is
    its own community, more distinct communities than a wave's LDS table
    holds (256 slots), so those rows take the global table."""
    idx, dist = synth.random_knn_lists(4000, 15, seed=64, hub_fraction=0.004)
    p, x, d, _, _ = oracle_mod.connectivities(idx, dist)
    assert (np.diff(p) > 256).sum() >= 10
    check(rsc, p, x, d, "hub rows beyond the LDS table")


def test_cliques_and_edge_cases(rsc, oracle_mod):
    # two 8-cliques joined by one edge
    n = 16
    W = np.zeros((n, n), np.float32)
    W[:8, :8] = 1.0
    W[8:, 8:] = 1.0
    np.fill_diagonal(W, 0.0)
    W[7, 8] = W[8, 7] = 1.0
    lab, _ = check(rsc, *csr_from_dense(W), "two cliques")
    assert (lab[:8] == 0).all() and (lab[8:] == 1).all()
    # a ring of 12 5-cliques
    m, c = 12, 5
    W = np.zeros((m * c, m * c), np.float32)
    for b in range(m):
        W[b * c:(b + 1) * c, b * c:(b + 1) * c] = 1.0
        W[b * c + c - 1, ((b + 1) % m) * c] = W[((b + 1) % m) * c, b * c + c - 1] = 1.0
    np.fill_diagonal(W, 0.0)
    check(rsc, *csr_from_dense(W), "ring of cliques")
    # isolated vertices, self-loops, a zero-weight edge and a weight spread over many binades
    rng = np.random.default_rng(63)
    W = np.zeros((200, 200), np.float32)
    for _ in range(600):
        i, j = rng.integers(0, 180, 2)
        w = np.float32(rng.uniform(0.5, 1.0) * 2.0 ** -rng.integers(0, 30))
        W[i, j] = W[j, i] = w
    for i in range(0, 180, 7):
        W[i, i] = 0.75
    W[3, 5] = W[5, 3] = 0.0
    p, x, d = csr_from_dense(W)
    # keep the explicit zero: it is a stored entry of weight 0
    rows = np.repeat(np.arange(200), np.diff(p))
    entries = list(zip(rows.tolist(), x.tolist(), d.tolist())) + [(3, 5, 0.0), (5, 3, 0.0)]
    entries.sort()
    p = np.zeros(201, np.int64)
    for r, _, _ in entries:
        p[r + 1] += 1
    p = np.cumsum(p)
    x = np.array([e[1] for e in entries], np.int32)
    d = np.array([e[2] for e in entries], np.float32)
    check(rsc, p, x, d, "isolated vertices, self-loops, zero weight")
    # no edges at all: every vertex its own community
    p0 = np.zeros(11, np.int64)
    lab, q = check(rsc, p0, np.zeros(0, np.int32), np.zeros(0, np.float32), "no edges")
    assert (lab == np.arange(10)).all() and q == 0.0
    # one vertex
    check(rsc, np.array([0, 1], np.int64), np.array([0], np.int32), np.array([1.0], np.float32), "single self-loop")


def test_gpu_graph_end_to_end(rsc, oracle_mod):
    """The GPU's own kNN graph of a 30,000-cell mixture (rsc_knn +
    rsc_connectivities), clustered by the GPU and by the oracle."""
    import torch

    X = synth.mixture(30000, d=50, n_clusters=25, law="zipf", seed=64)
    _, _, g = rsc.knn_graph(torch.from_numpy(X).cuda(), 15)
    torch.cuda.synchronize()
    p, x, d = (t.cpu().numpy() for t in (g.indptr, g.indices, g.data))
    check(rsc, p, x, d, "GPU kNN graph, 30k cells")


def test_rejects_malformed_graphs(rsc):
    import torch

    from paper_2603_02402_amd import RscError

    def call(p, x, d, gamma=1.0):
        g = tuple(torch.from_numpy(np.asarray(a)).cuda() for a in (p, x, d))
        return rsc.leiden(g, gamma=gamma)

    p = np.array([0, 1, 2], np.int64)
    with pytest.raises(RscError, match="column"):
        call(p, np.array([1, 5], np.int32), np.array([1.0, 1.0], np.float32))
    with pytest.raises(RscError, match="weight"):
        call(p, np.array([1, 0], np.int32), np.array([1.0, -1.0], np.float32))
    with pytest.raises(RscError, match="weight"):
        call(p, np.array([1, 0], np.int32), np.array([1.0, np.nan], np.float32))
    with pytest.raises(RscError, match="row pointers"):
        call(np.array([0, 2, 1], np.int64), np.array([1, 0], np.int32), np.array([1.0, 1.0], np.float32))
    with pytest.raises(RscError, match="gamma"):
        call(p, np.array([1, 0], np.int32), np.array([1.0, 1.0], np.float32), gamma=0.0)
