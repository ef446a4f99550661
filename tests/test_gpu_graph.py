"""Parity of the HIP connectivities path (rsc_connectivities) with the oracle."""

import sys

import numpy as np
import pytest

import synth
from tests.parity import check_graph_properties, compare_csr, compare_knn

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


def gpu_conn(rsc, idx, dist):
    import torch

    g = rsc.connectivities(torch.from_numpy(np.ascontiguousarray(idx)).cuda(),
                           torch.from_numpy(np.ascontiguousarray(dist)).cuda())
    torch.cuda.synchronize()
    return (g.indptr.cpu().numpy(), g.indices.cpu().numpy(), g.data.cpu().numpy(), g.rho.cpu().numpy(),
            g.sigma.cpu().numpy())


def check_conn_on_lists(rsc, oracle_mod, idx, dist, label):
    n, k = idx.shape
    log(f"[graph parity] {label}: n={n} k={k}")
    gp, gx, gd, grho, gsig = gpu_conn(rsc, idx, dist)
    op, ox, od, orho, osig = oracle_mod.connectivities(idx, dist)
    rel = compare_csr((gp, gx, gd), (op, ox, od))
    np.testing.assert_array_equal(grho, orho)
    pos = osig > 0
    assert (gsig[~pos] == 0).all()
    srel = np.abs(gsig[pos] - osig[pos]) / osig[pos]
    log(f"  nnz={gp[-1]} weight rel max {rel:.2e}, sigma rel max {srel.max() if srel.size else 0:.2e}")
    assert (srel <= 1e-5).all()
    check_graph_properties(gp, gx, gd, n, k, grho, gsig, dist)
    return gp, gx, gd


def test_hand_example(rsc, oracle_mod):
    import json
    import os

    p = os.path.join(os.path.dirname(__file__), "golden", "union_4pt.json")
    gd = json.load(open(p))
    idx = np.array(gd["idx"], dtype=np.int32)
    dist = np.array(gd["dist"], dtype=np.float32)
    gp, gx, gv, grho, gsig = gpu_conn(rsc, idx, dist)
    cs = gd["csr_symbolic"]
    p_ = np.log2(3) - 1
    vals = {"1": 1.0, "p": p_, "2p-p^2": 2 * p_ - p_ * p_}
    assert gp.tolist() == cs["indptr"]
    assert gx.tolist() == cs["indices"]
    np.testing.assert_allclose(gv, [vals[v] for v in cs["data"]], rtol=1e-7)
    np.testing.assert_array_equal(grho, gd["rho"])


def test_on_oracle_knn_10k(rsc, oracle_mod):
    X = synth.workload("plain_10k")
    idx, _, dist = oracle_mod.knn(X, 15)
    check_conn_on_lists(rsc, oracle_mod, idx, dist, "oracle kNN of the 10k mixture")


@pytest.mark.parametrize("n,k,hub", [(50, 2, 0.1), (333, 3, 0.05), (1000, 15, 0.01), (3000, 32, 0.02),
                                      (700, 63, 0.05), (20, 1, 0.1),
                                      (3000, 63, 0.003)])  # 9 rows of more than 512 entries, up to 1414
def test_synthetic_lists(rsc, oracle_mod, n, k, hub):
    idx, dist = synth.random_knn_lists(n, k, seed=n + k, hub_fraction=hub)
    check_conn_on_lists(rsc, oracle_mod, idx, dist, f"synthetic lists hub={hub}")


def test_degenerate_rows(rsc, oracle_mod):
    # rows whose nearest distances tie (>= log2 k slots at rho) and duplicate points (zeros)
    n, k = 400, 15
    idx, dist = synth.random_knn_lists(n, k, seed=5)
    dist = dist.copy()
    dist[:50, 1:6] = 2.0            # 5 slots at rho: log2 15 < 5 -> sigma = 0
    dist[50:80, 1:] = 0.0           # all duplicates: rho = 0
    dist[80:120, 1:3] = 0.0         # duplicates then positive distances
    dist[80:120, 3:] = np.sort(dist[80:120, 3:], axis=1)
    check_conn_on_lists(rsc, oracle_mod, idx, dist, "degenerate rows")


def test_bad_graph_is_rejected(rsc):
    import torch

    idx, dist = synth.random_knn_lists(100, 5, seed=1)
    bad = idx.copy()
    bad[3, 2] = 100  # out of range
    with pytest.raises(rsc.RscError) as e:
        rsc.connectivities(torch.from_numpy(bad).cuda(), torch.from_numpy(dist).cuda())
    assert e.value.status == -8
    bad = idx.copy()
    bad[7, 2] = bad[7, 1]  # repeated neighbour
    with pytest.raises(rsc.RscError):
        rsc.connectivities(torch.from_numpy(bad).cuda(), torch.from_numpy(dist).cuda())


def test_end_to_end_10k(rsc, oracle_mod):
    """kNN + connectivities on the GPU vs the oracle's whole step (tie-aware)."""
    import torch

    X = synth.workload("plain_10k")
    idx, dist, g = rsc.knn_graph(torch.from_numpy(X).cuda(), 15)
    torch.cuda.synchronize()
    o = oracle_mod.knn_graph(X, 15)
    res = compare_knn(X, np.arange(X.shape[0]), idx.cpu().numpy(), dist.cpu().numpy(), o["idx"], o["dist"],
                      oracle_mod, 15)
    rel = compare_csr((g.indptr.cpu().numpy(), g.indices.cpu().numpy(), g.data.cpu().numpy()),
                      (o["indptr"], o["indices"], o["data"]), tie_rows=res["tie_row_ids"])
    log(f"[graph parity] end-to-end 10k: knn {res['exact_rows']} exact rows, weight rel max {rel:.2e}")


@pytest.mark.parametrize("n", [1, 7, 300])
def test_k1_lists_have_no_edges(rsc, oracle_mod, n):
    """k = 1: every list holds only the row itself, so the graph is empty and rho = sigma = 0."""
    idx = np.arange(n, dtype=np.int32).reshape(n, 1)
    dist = np.zeros((n, 1), dtype=np.float32)
    gp, _, _ = check_conn_on_lists(rsc, oracle_mod, idx, dist, "k=1 lists")
    assert gp[-1] == 0


@pytest.mark.parametrize("n,k", [(1, 1), (2, 2), (3, 2), (3, 3), (16, 15), (40, 33)])
def test_end_to_end_few_cells(rsc, oracle_mod, n, k):
    """kNN + connectivities of a handful of cells (k up to n) against the oracle's whole step."""
    import torch

    X = synth.mixture(n, d=50, n_clusters=2, seed=1000 + 10 * n + k)
    log(f"[graph parity] end-to-end n={n} k={k}")
    idx, dist, g = rsc.knn_graph(torch.from_numpy(X).cuda(), k)
    torch.cuda.synchronize()
    o = oracle_mod.knn_graph(X, k)
    res = compare_knn(X, np.arange(n), idx.cpu().numpy(), dist.cpu().numpy(), o["idx"], o["dist"], oracle_mod, k)
    rel = compare_csr((g.indptr.cpu().numpy(), g.indices.cpu().numpy(), g.data.cpu().numpy()),
                      (o["indptr"], o["indices"], o["data"]), tie_rows=res["tie_row_ids"])
    log(f"  knn {res['exact_rows']} exact rows, nnz {int(o['indptr'][-1])}, weight rel max {rel:.2e}")
    if k == 1:
        assert int(g.indptr.cpu().numpy()[-1]) == 0


def test_synthetic_lists_1m(rsc, oracle_mod):
    """Graph stage at the 1M-cell scale on seeded kNN-shaped lists, full parity."""
    n, k = 1_000_000, 15
    idx, dist = synth.random_knn_lists(n, k, seed=2024)
    check_conn_on_lists(rsc, oracle_mod, idx, dist, "synthetic 1M lists")


def test_graph_deterministic(rsc):
    idx, dist = synth.random_knn_lists(20000, 15, seed=9, hub_fraction=0.02)
    a = gpu_conn(rsc, idx, dist)
    b = gpu_conn(rsc, idx, dist)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x.view(np.uint8), y.view(np.uint8))


@pytest.mark.parametrize("n,k", [(3000, 66), (2000, 100), (1500, 256)])
def test_large_k_lists(rsc, oracle_mod, n, k):
    """Rows with more than 64 neighbour slots (smooth kNN from memory)."""
    idx, dist = synth.random_knn_lists(n, k, seed=n + k)
    check_conn_on_lists(rsc, oracle_mod, idx, dist, f"synthetic lists k={k}")
