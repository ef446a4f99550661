"""The allocation-free connectivities entry point (rsc_connectivities_noalloc)
against the workspace one (rsc_connectivities), through the C ABI: two calls
in a row on the library's fixed scratch, the second with a smaller input, each
bitwise equal to the workspace call's CSR, rho and sigma."""

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


def _noalloc(rsc, idx, dist):
    import torch

    n, k = idx.shape
    cap = 2 * n * (k - 1)
    dev = idx.device
    # outputs pre-filled with garbage: the call must write every entry it reports
    indptr = torch.full((n + 1,), -7, dtype=torch.int64, device=dev)
    indices = torch.full((cap,), -7, dtype=torch.int32, device=dev)
    data = torch.full((cap,), float("nan"), dtype=torch.float32, device=dev)
    rho = torch.full((n,), float("nan"), dtype=torch.float64, device=dev)
    sigma = torch.full((n,), float("nan"), dtype=torch.float64, device=dev)
    nnz = rsc.connectivities_noalloc(idx, dist, (indptr, indices, data), rho, sigma)
    torch.cuda.synchronize()
    return (indptr.cpu().numpy(), indices[:nnz].cpu().numpy(), data[:nnz].cpu().numpy(), rho.cpu().numpy(),
            sigma.cpu().numpy())


def _with_workspace(rsc, idx, dist):
    import torch

    g = rsc.connectivities(idx, dist)
    torch.cuda.synchronize()
    return (g.indptr.cpu().numpy(), g.indices.cpu().numpy(), g.data.cpu().numpy(), g.rho.cpu().numpy(),
            g.sigma.cpu().numpy())


def _same(a, b, label):
    names = ["indptr", "indices", "data", "rho", "sigma"]
    for name, x, y in zip(names, a, b):
        assert x.shape == y.shape, f"{label}: {name} shape {x.shape} vs {y.shape}"
        assert np.array_equal(x.view(np.uint8), y.view(np.uint8)), f"{label}: {name} differs"


def test_noalloc_matches_workspace_call_twice(rsc):
    import torch

    cases = [(60000, 15, 71), (7001, 15, 72)]  # the second call is smaller: stale scratch must not leak in
    for n, k, seed in cases:
        need = rsc.load().rsc_connectivities_workspace_bytes(n, k)
        log(f"[noalloc] n={n} k={k} seed={seed} workspace {need} bytes "
            f"(scratch {rsc.load().rsc_connectivities_noalloc_max_bytes()})")
        idx_h, dist_h = synth.random_knn_lists(n, k, seed=seed)
        idx = torch.from_numpy(idx_h).cuda()
        dist = torch.from_numpy(dist_h).cuda()
        got = _noalloc(rsc, idx, dist)
        ref = _with_workspace(rsc, idx, dist)
        _same(got, ref, f"n={n}")
        log(f"  nnz={got[0][-1]} bitwise equal to rsc_connectivities")


def test_noalloc_on_a_knn_result_and_small_k(rsc):
    import torch

    X = torch.from_numpy(synth.mixture(5000, d=50, n_clusters=10, seed=73)).cuda()
    for k in (15, 2):
        idx, dist = rsc.knn(X, k)
        log(f"[noalloc] kNN result n=5000 k={k}")
        _same(_noalloc(rsc, idx, dist), _with_workspace(rsc, idx, dist), f"k={k}")


def test_noalloc_rejects_problems_beyond_its_scratch(rsc):
    import torch

    lib = rsc.load()
    cap_bytes = lib.rsc_connectivities_noalloc_max_bytes()
    n, k = 300000, 15
    assert lib.rsc_connectivities_workspace_bytes(n, k) > cap_bytes
    idx = torch.zeros((n, k), dtype=torch.int32, device="cuda")
    dist = torch.zeros((n, k), dtype=torch.float32, device="cuda")
    out = (torch.empty(n + 1, dtype=torch.int64, device="cuda"),
           torch.empty(2 * n * (k - 1), dtype=torch.int32, device="cuda"),
           torch.empty(2 * n * (k - 1), dtype=torch.float32, device="cuda"))
    with pytest.raises(rsc.RscError, match="scratch"):
        rsc.connectivities_noalloc(idx, dist, out)
