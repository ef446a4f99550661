"""UMAP layout: parity of the HIP path (through the C ABI) with the float64
oracle, plus the determinism and the degenerate cases of the schedule.

Both sides run the same float64 operations in the same order (explicitly
rounded on the GPU, no contraction in the oracle) and take the powers d2^b
and d2^(b-1) correctly rounded (double-double on the GPU, quadruple precision
rounded in the oracle), so the layouts are the same function of the inputs:
the float32 outputs must agree bit for bit at every depth.  (With the math libraries'
own pow, which each miss the nearest double in about 1 case in 1000, the
layouts agree bitwise for a few epochs and then part: the dynamics amplify a
one-ulp difference.)
"""

import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

A, B = 0.5830300203414425, 1.3341669924314914


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


@pytest.fixture(scope="module")
def graph():
    import oracle

    X = synth.mixture(2000, d=50, n_clusters=12, seed=41)
    g = oracle.knn_graph(X, 15)
    return g["indptr"], g["indices"], g["data"]


def gpu_layout(rsc, csr, Y0, **kw):
    import torch

    indptr, indices, data = csr
    dev = torch.device("cuda:0")
    t = (torch.from_numpy(np.asarray(indptr, dtype=np.int64)).to(dev),
         torch.from_numpy(np.asarray(indices, dtype=np.int32)).to(dev),
         torch.from_numpy(np.asarray(data, dtype=np.float32)).to(dev))
    Y = rsc.umap_layout(t, torch.from_numpy(np.ascontiguousarray(Y0, dtype=np.float32)).to(dev), **kw)
    torch.cuda.synchronize()
    return Y.cpu().numpy()


def cpu_layout(csr, Y0, n_epochs, **kw):
    from oracle import umap as ou

    indptr, indices, data = csr
    kw = dict(kw)
    a, b = kw.pop("a", A), kw.pop("b", B)
    return ou.layout(indptr, indices, data, Y0.astype(np.float64), n_epochs, a, b, **kw)


def report(tag, got, want):
    err = np.abs(got.astype(np.float64) - want.astype(np.float32).astype(np.float64))
    same = float(np.mean(got == want.astype(np.float32)))
    log(f"[umap] {tag}: max |diff| {err.max():.3e}, bitwise-equal fraction {same:.6f}")
    return err


@pytest.mark.parametrize("n_epochs", [2, 5])
def test_first_epochs_match_oracle(rsc, graph, n_epochs):
    Y0 = synth.umap_init(2000, 2, seed=1)
    log(f"[umap] first epochs n=2000 dim=2 n_epochs={n_epochs}")
    got = gpu_layout(rsc, graph, Y0, n_epochs=n_epochs, seed=3)
    want = cpu_layout(graph, Y0, n_epochs, seed=3)
    report(f"{n_epochs} epochs", got, want)
    assert np.array_equal(got, want.astype(np.float32))


@pytest.mark.parametrize("n_epochs", [20, 200])
def test_long_runs_match_oracle(rsc, graph, n_epochs):
    Y0 = synth.umap_init(2000, 2, seed=2)
    log(f"[umap] {n_epochs} epochs n=2000 dim=2")
    got = gpu_layout(rsc, graph, Y0, n_epochs=n_epochs, seed=7)
    want = cpu_layout(graph, Y0, n_epochs, seed=7)
    report(f"{n_epochs} epochs", got, want)
    assert np.array_equal(got, want.astype(np.float32))


@pytest.mark.parametrize("dim", [1, 3, 8])
def test_other_dims_match_oracle(rsc, graph, dim):
    Y0 = synth.umap_init(2000, dim, seed=4 + dim)
    log(f"[umap] dim={dim} 6 epochs")
    got = gpu_layout(rsc, graph, Y0, n_epochs=6, seed=11, neg=3, gamma=0.5, alpha0=0.7)
    want = cpu_layout(graph, Y0, 6, seed=11, neg=3, gamma=0.5, alpha0=0.7)
    report(f"dim {dim}", got, want)
    assert np.array_equal(got, want.astype(np.float32))


def test_deterministic(rsc, graph):
    Y0 = synth.umap_init(2000, 2, seed=5)
    a = gpu_layout(rsc, graph, Y0, n_epochs=30, seed=9)
    b = gpu_layout(rsc, graph, Y0, n_epochs=30, seed=9)
    assert np.array_equal(a, b)
    c = gpu_layout(rsc, graph, Y0, n_epochs=30, seed=10)
    assert not np.array_equal(a, c)


def test_isolated_and_weak_edges(rsc):
    # vertex 3 has no edges; the edge 4-5 is below w_max / n_epochs and is
    # never sampled; with no negatives nothing else touches 3, 4 or 5
    indptr = np.array([0, 2, 4, 6, 6, 7, 8], dtype=np.int64)
    indices = np.array([1, 2, 0, 2, 0, 1, 5, 4], dtype=np.int32)
    data = np.array([1.0, 0.5, 1.0, 0.25, 0.5, 0.25, 0.01, 0.01], dtype=np.float32)
    Y0 = synth.umap_init(6, 2, seed=6)
    got = gpu_layout(rsc, (indptr, indices, data), Y0, n_epochs=10, neg=0)
    want = cpu_layout((indptr, indices, data), Y0, 10, neg=0)
    report("small graph", got, want)
    assert np.array_equal(got[3:], Y0[3:])
    assert not np.array_equal(got[:3], Y0[:3])
    assert np.array_equal(got, want.astype(np.float32))


def test_coincident_points_and_empty_graph(rsc):
    # all points at one place: attraction is 0 and every repulsion takes the
    # coincident-point move; a graph with no edges leaves the layout as is
    n = 50
    indptr = np.arange(0, 2 * n + 1, 2, dtype=np.int64)
    indices = np.stack([(np.arange(n) + 1) % n, (np.arange(n) - 1) % n], 1).ravel().astype(np.int32)
    data = np.ones(2 * n, dtype=np.float32)
    Y0 = np.full((n, 2), 3.0, dtype=np.float32)
    got = gpu_layout(rsc, (indptr, indices, data), Y0, n_epochs=2, seed=1)
    want = cpu_layout((indptr, indices, data), Y0, 2, seed=1)
    assert np.array_equal(got, want.astype(np.float32))
    empty = (np.zeros(n + 1, dtype=np.int64), np.zeros(0, dtype=np.int32), np.zeros(0, dtype=np.float32))
    Y1 = synth.umap_init(n, 2, seed=8)
    assert np.array_equal(gpu_layout(rsc, empty, Y1, n_epochs=5), Y1)


def test_bad_graph_rejected(rsc):
    import torch

    from paper_2603_02402_amd import RscError

    indptr = np.array([0, 1, 2], dtype=np.int64)
    Y0 = synth.umap_init(2, 2, seed=1)
    for indices, data in (([1, 2], [1.0, 1.0]), ([1, 0], [1.0, -1.0])):
        with pytest.raises(RscError):
            gpu_layout(rsc, (indptr, np.array(indices, np.int32), np.array(data, np.float32)), Y0, n_epochs=3)
    with pytest.raises(RscError):
        gpu_layout(rsc, (np.array([0, 2, 1], np.int64), np.array([1, 0], np.int32), np.ones(2, np.float32)), Y0,
                   n_epochs=3)
    bad_y = Y0.copy()
    bad_y[1, 0] = np.nan
    with pytest.raises(RscError, match="non-finite initial"):
        gpu_layout(rsc, (indptr, np.array([1, 0], np.int32), np.ones(2, np.float32)), bad_y, n_epochs=3)
    torch.cuda.synchronize()


def test_pipeline_end_to_end(rsc):
    # kNN -> connectivities -> layout on the GPU against the oracle's whole
    # pipeline on the same cells
    import torch

    import oracle

    X = synth.mixture(3000, d=50, n_clusters=9, seed=43)
    idx, dist, g = rsc.knn_graph(torch.from_numpy(X).to("cuda:0"), 15)
    o = oracle.knn_graph(X, 15)
    assert np.array_equal(g.indptr.cpu().numpy(), o["indptr"])
    assert np.array_equal(g.indices.cpu().numpy(), o["indices"])
    assert np.array_equal(g.data.cpu().numpy(), o["data"])
    Y0 = synth.umap_init(3000, 2, seed=44)
    got = rsc.umap_layout(g, torch.from_numpy(Y0).to("cuda:0"), n_epochs=50, seed=5).cpu().numpy()
    want = cpu_layout((o["indptr"], o["indices"], o["data"]), Y0, 50, seed=5)
    report("end to end", got, want)
    assert np.array_equal(got, want.astype(np.float32))


@pytest.mark.parametrize("kw", [dict(neg=0), dict(gamma=0.0), dict(neg=64, seed=123), dict(alpha0=0.25, a=1.2, b=0.8)])
def test_parameters_match_oracle(rsc, graph, kw):
    Y0 = synth.umap_init(2000, 2, seed=9)
    log(f"[umap] parameters {kw}")
    got = gpu_layout(rsc, graph, Y0, n_epochs=12, **kw)
    want = cpu_layout(graph, Y0, 12, **kw)
    report(f"params {kw}", got, want)
    assert np.array_equal(got, want.astype(np.float32))


def test_single_vertex_and_self_draws(rsc):
    # n = 1: every negative sample draws the vertex itself; n = 2 with one
    # edge: about half of them do
    one = (np.array([0, 0], np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32))
    Y1 = synth.umap_init(1, 2, seed=3)
    assert np.array_equal(gpu_layout(rsc, one, Y1, n_epochs=4), Y1)
    two = (np.array([0, 1, 2], np.int64), np.array([1, 0], np.int32), np.ones(2, np.float32))
    Y2 = synth.umap_init(2, 3, seed=4)
    got = gpu_layout(rsc, two, Y2, n_epochs=9, neg=7, seed=8)
    want = cpu_layout(two, Y2, 9, neg=7, seed=8)
    assert np.array_equal(got, want.astype(np.float32))


def test_overflowing_power_turns_nan_on_both_sides(rsc):
    # b = 60 and points 1e6 apart: d2^b and d2^(b-1) exceed the largest
    # double, the attraction is inf / inf, and the layout turns NaN exactly
    # where the oracle's does (no move is silently dropped)
    two = (np.array([0, 1, 2, 2], np.int64), np.array([1, 0], np.int32), np.ones(2, np.float32))
    Y0 = np.array([[0.0, 0.0], [1e6, 0.0], [5.0, 5.0]], np.float32)
    got = gpu_layout(rsc, two, Y0, n_epochs=3, a=1.0, b=60.0, neg=3, seed=2)
    want = cpu_layout(two, Y0, 3, a=1.0, b=60.0, neg=3, seed=2).astype(np.float32)
    assert np.isnan(want[:2]).all() and np.isfinite(want[2]).all()
    assert np.array_equal(got, want, equal_nan=True)


@pytest.fixture(scope="module")
def full_graph():
    import oracle

    n, k = 1_000_000, 15
    idx, dist = synth.random_knn_lists(n, k, seed=12)
    indptr, indices, data, _, _ = oracle.connectivities(idx, dist)
    return indptr, indices, data


@pytest.mark.parametrize("n_epochs", [3, 6])
def test_full_size_epochs_match_oracle(rsc, full_graph, n_epochs):
    # the bench's graph size: 1M vertices, kNN-shaped lists of 15 with hubs,
    # connectivities from the oracle; with 3 epochs the edges of weight >=
    # w_max / 2 are sampled, with 6 those of weight >= w_max / 6, over 5
    # active epochs
    indptr, indices, data = full_graph
    n = len(indptr) - 1
    log(f"[umap] full size n={n} nnz={len(indices)} {n_epochs} epochs")
    Y0 = synth.umap_init(n, 2, seed=13)
    got = gpu_layout(rsc, (indptr, indices, data), Y0, n_epochs=n_epochs, seed=17)
    want = cpu_layout((indptr, indices, data), Y0, n_epochs, seed=17)
    report(f"full size {n_epochs} epochs", got, want)
    assert np.array_equal(got, want.astype(np.float32))
