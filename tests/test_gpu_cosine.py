"""Cosine metric (1 - cos): parity of the HIP path (through the C ABI) with
the float64 oracle; the same near-tie rule as the Euclidean path."""

import sys

import numpy as np
import pytest

import synth
from tests.parity import compare_csr, compare_knn, cosine_pair_dist

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


def gpu(rsc, X, k, Q=None, **kw):
    import torch

    Xt = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    Qt = None if Q is None else torch.from_numpy(np.ascontiguousarray(Q)).cuda()
    ws = rsc.Workspace()
    idx, dist = rsc.knn(Xt, k, Q=Qt, workspace=ws, metric=rsc.RSC_COSINE, **kw)
    torch.cuda.synchronize()
    return idx.cpu().numpy(), dist.cpu().numpy(), rsc.read_knn_stats(ws)


def check(rsc, oracle_mod, X, k, label):
    n = X.shape[0]
    log(f"[cosine] {label}: n={n} d={X.shape[1]} k={k}")
    idx_g, dist_g, st = gpu(rsc, X, k)
    idx_o, _, dist_o = oracle_mod.knn(X, k, metric="cosine")
    res = compare_knn(X, np.arange(n), idx_g, dist_g, idx_o, dist_o, oracle_mod, k, pair_dist=cosine_pair_dist)
    log(f"  {res['exact_rows']}/{n} rows identical, near-tie rows {res['near_tie_rows']}, dist rel max "
        f"{res['dist_rel_max']:.2e}, stats {st}")
    assert st["max_err_ratio"] < 1.0
    return res, st


def test_cosine_10k_full_parity(rsc, oracle_mod):
    X = synth.workload("plain_10k")
    res, st = check(rsc, oracle_mod, X, 15, "10k mixture")
    assert res["exact_rows"] + res["near_tie_rows"] == X.shape[0]


@pytest.mark.parametrize("n,d,k", [(1000, 50, 15), (2049, 17, 30), (777, 128, 7), (300, 3, 1)])
def test_cosine_shapes(rsc, oracle_mod, n, d, k):
    rng = np.random.default_rng(n + d)
    X = (rng.standard_normal((n, d)) + rng.normal(0, 2, (1, d))).astype(np.float32)
    check(rsc, oracle_mod, X, k, f"random n={n} d={d} k={k}")


def test_cosine_zero_rows_and_collinear_rows(rsc, oracle_mod):
    rng = np.random.default_rng(7)
    X = rng.standard_normal((600, 20)).astype(np.float32)
    X[5] = 0.0
    X[17] = 0.0
    X[40] = 3.0 * X[41]  # same direction: distance ~0
    X[42] = 0.5 * X[41]
    idx_g, dist_g, st = gpu(rsc, X, 12)
    idx_o, _, dist_o = oracle_mod.knn(X, 12, metric="cosine")
    compare_knn(X, np.arange(600), idx_g, dist_g, idx_o, dist_o, oracle_mod, 12, pair_dist=cosine_pair_dist)
    assert (dist_g[5, 1:] == 1.0).all() and idx_g[5, 1:].tolist() == [j for j in range(13) if j != 5][:11]
    assert set(idx_g[41, 1:3].tolist()) == {40, 42}


def test_cosine_rectangular(rsc, oracle_mod):
    rng = np.random.default_rng(11)
    R = rng.standard_normal((3000, 30)).astype(np.float32)
    Q = rng.standard_normal((500, 30)).astype(np.float32)
    idx_g, dist_g, _ = gpu(rsc, R, 10, Q=Q)
    idx_o, _, dist_o = oracle_mod.knn(R, 10, Q=Q, metric="cosine")

    def qr_dist(_, ii, jj):
        a = Q[np.asarray(ii)].astype(np.float64)
        b = R[np.asarray(jj)].astype(np.float64)
        return 1.0 - (a * b).sum(1) / np.sqrt((a * a).sum(1) * (b * b).sum(1))

    res = compare_knn(R, np.arange(len(Q)), idx_g, dist_g, idx_o, dist_o, oracle_mod, 10, self_mode=False,
                      pair_dist=qr_dist)
    log(f"[cosine] rectangular: {res['exact_rows']}/{len(Q)} identical, near-tie rows {res['near_tie_rows']}")


def test_cosine_end_to_end_graph(rsc, oracle_mod):
    """kNN + connectivities under the cosine distance vs the oracle's whole step."""
    import torch

    X = synth.mixture(4000, n_clusters=8, seed=12)
    idx, dist, g = rsc.knn_graph(torch.from_numpy(X).cuda(), 15, metric=rsc.RSC_COSINE)
    torch.cuda.synchronize()
    o = oracle_mod.knn_graph(X, 15, metric="cosine")
    res = compare_knn(X, np.arange(X.shape[0]), idx.cpu().numpy(), dist.cpu().numpy(), o["idx"], o["dist"],
                      oracle_mod, 15, pair_dist=cosine_pair_dist)
    rel = compare_csr((g.indptr.cpu().numpy(), g.indices.cpu().numpy(), g.data.cpu().numpy()),
                      (o["indptr"], o["indices"], o["data"]), tie_rows=res["tie_row_ids"])
    log(f"[cosine] end-to-end graph: {res['exact_rows']} identical kNN rows, weight rel max {rel:.2e}")


def test_cosine_bf16_recall(rsc, oracle_mod):
    X = synth.workload("plain_10k")
    idx_g, _, _ = gpu(rsc, X, 15, precision=rsc.RSC_BF16)
    idx_o, _, _ = oracle_mod.knn(X, 15, metric="cosine")
    hits = sum(len(set(a[1:].tolist()) & set(b[1:].tolist())) for a, b in zip(idx_g, idx_o))
    rec = hits / (X.shape[0] * 14)
    log(f"[cosine] bf16 10k recall@15 = {rec:.5f}")
    assert rec >= 0.99
