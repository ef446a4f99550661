"""Parity of the HIP kNN path (through the C ABI) with the FP64 CPU oracle."""

import sys

import numpy as np
import pytest

import synth
from tests.parity import compare_knn

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


def gpu_knn(rsc, X, k, Q=None, **kw):
    import torch

    Xt = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    Qt = None if Q is None else torch.from_numpy(np.ascontiguousarray(Q)).cuda()
    ws = rsc.Workspace()
    idx, dist = rsc.knn(Xt, k, Q=Qt, workspace=ws, **kw)
    torch.cuda.synchronize()
    return idx.cpu().numpy(), dist.cpu().numpy(), rsc.read_knn_stats(ws)


def check_full(rsc, oracle_mod, X, k, label):
    n = X.shape[0]
    log(f"[knn parity] {label}: n={n} d={X.shape[1]} k={k}")
    idx_g, dist_g, stats = gpu_knn(rsc, X, k)
    idx_o, _, dist_o = oracle_mod.knn(X, k)
    res = compare_knn(X, np.arange(n), idx_g, dist_g, idx_o, dist_o, oracle_mod, k)
    log(f"  {res['exact_rows']}/{n} rows identical, near-tie rows {res['near_tie_rows']}, "
        f"dist rel max {res['dist_rel_max']:.2e}, stats {stats}")
    assert stats["max_err_ratio"] < 1.0, "screen error exceeded its certified bound"
    return res, stats


def test_plain_10k_full_parity(rsc, oracle_mod):
    X = synth.workload("plain_10k")
    res, stats = check_full(rsc, oracle_mod, X, 15, "10k mixture, 20 clusters")
    assert res["exact_rows"] + res["near_tie_rows"] == X.shape[0]


@pytest.mark.parametrize("n,d,k", [
    (1, 50, 1), (2, 50, 2), (15, 50, 15), (16, 50, 15), (33, 50, 15), (100, 50, 15), (1000 + 17, 50, 15),
    (513, 1, 5), (300, 3, 15), (700, 64, 15), (257, 65, 15), (400, 128, 7), (500, 16, 32), (600, 50, 2),
    (600, 50, 3), (450, 50, 63), (2050, 50, 15),
])
def test_shapes_and_ragged_tails(rsc, oracle_mod, n, d, k):
    X = synth.mixture(n, d=d, n_clusters=5, seed=n * 131 + d * 7 + k)
    check_full(rsc, oracle_mod, X, k, f"shape n={n} d={d} k={k}")


def test_duplicates(rsc, oracle_mod):
    X = synth.mixture(3000, d=50, n_clusters=10, seed=77)
    rng = np.random.default_rng(0)
    src = rng.choice(3000, 200, replace=False)
    dst = rng.choice(3000, 200, replace=False)
    X[dst] = X[src]
    X[100:140] = X[99]  # 41 identical rows: more duplicates than the screen width
    check_full(rsc, oracle_mod, X, 15, "injected duplicates")


def test_all_identical(rsc, oracle_mod):
    X = np.full((500, 50), 3.25, dtype=np.float32)
    idx_g, dist_g, _ = gpu_knn(rsc, X, 15)
    idx_o, _, dist_o = oracle_mod.knn(X, 15)
    np.testing.assert_array_equal(idx_g, idx_o)
    np.testing.assert_array_equal(dist_g, dist_o)


def test_lattice_exact_ties(rsc, oracle_mod):
    X = synth.lattice_1d(2000, d=50, spacing=0.5)
    idx_g, dist_g, _ = gpu_knn(rsc, X, 15)
    idx_o, _, dist_o = oracle_mod.knn(X, 15)
    np.testing.assert_array_equal(idx_g, idx_o)
    np.testing.assert_array_equal(dist_g, dist_o)


def test_far_from_origin(rsc, oracle_mod):
    # norm cancellation: a large common offset makes ||x||^2 - 2 x.y lose digits
    X = synth.mixture(4000, d=50, n_clusters=8, seed=5) + np.float32(300.0)
    res, stats = check_full(rsc, oracle_mod, X, 15, "offset +300")
    log(f"  rescanned rows: {stats['rescanned_rows']}")
    # the offset inflates every certificate bound: all rows escalate (measured 4000 of 4000)
    assert stats["escalated_rows"] > 0


def test_rectangular(rsc, oracle_mod):
    R = synth.mixture(5000, d=50, n_clusters=12, seed=8)
    Q = synth.mixture(777, d=50, n_clusters=12, seed=9)
    for k in (1, 15):
        idx_g, dist_g, stats = gpu_knn(rsc, R, k, Q=Q)
        idx_o, _, dist_o = oracle_mod.knn(R, k, Q=Q)
        res = compare_knn(R, np.arange(len(Q)), idx_g, dist_g, idx_o, dist_o, oracle_mod, k, self_mode=False)
        log(f"[knn parity] rectangular k={k}: {res}")


def test_deterministic(rsc):
    X = synth.workload("plain_10k", n=6000)
    a = gpu_knn(rsc, X, 15)
    b = gpu_knn(rsc, X, 15)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1].view(np.uint32), b[1].view(np.uint32))


def test_plain_1m_sampled_parity(rsc, oracle_mod):
    """Full 1M-cell workload on the GPU, launch shape as benchmarked; oracle on sampled rows."""
    import torch

    X = synth.workload("plain_1m")
    log("[knn parity] 1M cells, 100 Zipf clusters: GPU full run")
    Xt = torch.from_numpy(X).cuda()
    ws = rsc.Workspace()
    idx, dist = rsc.knn(Xt, 15, workspace=ws)
    torch.cuda.synchronize()
    stats = rsc.read_knn_stats(ws)
    log(f"  stats {stats}")
    # every row the first certificate failed (escalated to the wider screen)
    # plus a seeded sample of the others
    esc = rsc.read_knn_escalated(ws, X.shape[0], X.shape[0], X.shape[1], 15)
    log(f"  escalated rows read back: {len(esc)}")
    assert len(esc) == stats["escalated_rows"] > 0
    rows = synth.sample_rows(X.shape[0], 96, seed=123)
    rows = np.unique(np.concatenate([rows, [0, X.shape[0] - 1], esc]))
    idx_g = idx[torch.from_numpy(rows).cuda()].cpu().numpy()
    dist_g = dist[torch.from_numpy(rows).cuda()].cpu().numpy()
    log(f"  oracle on {len(rows)} sampled rows")
    idx_o, _, dist_o = oracle_mod.knn_rows(X, rows, 15)
    res = compare_knn(X, rows, idx_g, dist_g, idx_o, dist_o, oracle_mod, 15)
    log(f"  {res}")
    assert stats["max_err_ratio"] < 1.0
    # whole-output properties: self first, ascending distances, distinct neighbours
    idx_all = idx.cpu().numpy()
    dist_all = dist.cpu().numpy()
    assert (idx_all[:, 0] == np.arange(X.shape[0])).all()
    assert (np.diff(dist_all, axis=1) >= 0).all()
    s = np.sort(idx_all, axis=1)
    assert not (s[:, 1:] == s[:, :-1]).any()
    assert ((idx_all >= 0) & (idx_all < X.shape[0])).all()


# ---------------------------------------------------------------------------
# Larger k and d (exact path): the running top-m spans 1, 2 or 4 registers per
# lane (m <= 64, 128, 256), the main screen splits the references into about
# k / 32 ranges, and the exhaustive rescan uses the same top-m lists.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,d,k", [
    (3000, 50, 65), (3000, 50, 66), (2500, 50, 100), (2000, 30, 128), (2000, 30, 129), (1500, 20, 255),
    (1500, 129, 15), (1200, 200, 40), (1100, 256, 64), (900, 256, 200),
])
def test_large_k_and_d(rsc, oracle_mod, n, d, k):
    X = synth.mixture(n, d=d, n_clusters=6, seed=n + d + k)
    check_full(rsc, oracle_mod, X, k, f"large k/d n={n} d={d} k={k}")


def test_large_k_rescan_on_ties(rsc, oracle_mod):
    """A lattice (every distance a multiple of the spacing) and injected
    duplicates with k = 100: rows the screens cannot certify go to the
    exhaustive float64 scan."""
    X = synth.lattice_1d(1500, d=20, spacing=0.5)
    idx_g, dist_g, st = gpu_knn(rsc, X, 100)
    idx_o, _, dist_o = oracle_mod.knn(X, 100)
    log(f"[knn parity] lattice k=100: stats {st}")
    assert st["rescanned_rows"] > 0  # measured 1176: the exhaustive scan ran
    np.testing.assert_array_equal(idx_g, idx_o)
    np.testing.assert_array_equal(dist_g, dist_o)
    Y = synth.mixture(2000, d=50, n_clusters=4, seed=31)
    Y[100:400] = Y[99]  # 301 identical rows: more than k
    idx_g, dist_g, st = gpu_knn(rsc, Y, 150)
    idx_o, _, dist_o = oracle_mod.knn(Y, 150)
    log(f"[knn parity] duplicates k=150: stats {st}")
    assert st["rescanned_rows"] > 0  # measured 382
    res = compare_knn(Y, np.arange(2000), idx_g, dist_g, idx_o, dist_o, oracle_mod, 150)
    assert res["exact_rows"] + res["near_tie_rows"] == 2000


def test_large_k_rectangular_and_cosine(rsc, oracle_mod):
    R = synth.mixture(4000, d=64, n_clusters=10, seed=41)
    Q = synth.mixture(300, d=64, n_clusters=10, seed=42)
    for k in (64, 128, 200):
        idx_g, dist_g, _ = gpu_knn(rsc, R, k, Q=Q)
        idx_o, _, dist_o = oracle_mod.knn(R, k, Q=Q)
        compare_knn(R, np.arange(len(Q)), idx_g, dist_g, idx_o, dist_o, oracle_mod, k, self_mode=False)
    from tests.parity import cosine_pair_dist

    X = synth.mixture(2500, d=50, n_clusters=8, seed=43)
    idx_g, dist_g, _ = gpu_knn(rsc, X, 100, metric=rsc.RSC_COSINE)
    idx_o, _, dist_o = oracle_mod.knn(X, 100, metric="cosine")
    res = compare_knn(X, np.arange(2500), idx_g, dist_g, idx_o, dist_o, oracle_mod, 100, pair_dist=cosine_pair_dist)
    assert res["exact_rows"] + res["near_tie_rows"] == 2500
