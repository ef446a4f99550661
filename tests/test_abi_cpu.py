"""The C ABI library loads, exports what include/rsc.h declares, and validates
arguments on the host (no GPU needed: every case here fails validation
before anything is enqueued)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rsc.h")
LIB = os.path.join(ROOT, "paper_2603_02402_amd", "librsc.so")

FAKE = ctypes.c_void_p(0x10000)  # never dereferenced: validation fails first


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(rsc_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import paper_2603_02402_amd.build as b

        b.build()
    from paper_2603_02402_amd import _lib

    return _lib.load(LIB)


def test_header_declares_the_calls():
    names = declared_functions()
    for n in ["rsc_knn", "rsc_knn_ex", "rsc_connectivities", "rsc_knn_workspace_bytes",
              "rsc_connectivities_workspace_bytes", "rsc_last_error", "rsc_abi_version"]:
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    from paper_2603_02402_amd import _lib

    for name in declared_functions():
        assert hasattr(lib, name), name
        assert name in _lib.SIGNATURES, f"binding lacks {name}"


def test_abi_version(lib):
    assert lib.rsc_abi_version() == 1


def test_workspace_sizes(lib):
    from paper_2603_02402_amd import _lib

    o = _lib.KnnOpts(0, 0, 0, 0)
    n, d, k = 10000, 50, 15
    ws = lib.rsc_knn_workspace_bytes(n, n, d, k, ctypes.byref(o))
    # counters + norms + candidates (idx + key, width 32) + flag list
    assert ws >= n * 4 + 2 * n * 32 * 4 + n * 4
    assert ws % 256 == 0
    assert lib.rsc_knn_workspace_bytes(n, n, d, 0, None) == 0
    assert lib.rsc_knn_workspace_bytes(n, n, 0, k, None) == 0
    assert lib.rsc_knn_workspace_bytes(5, 5, d, 6, None) == 0
    g = lib.rsc_connectivities_workspace_bytes(n, k)
    # per edge: float64 weight, float32 union weight, int32 slot, 8-byte reverse record
    assert g >= n * (k - 1) * (8 + 4 + 4 + 8)
    assert lib.rsc_connectivities_workspace_bytes(0, k) == 0


def _knn(lib, n=100, d=50, k=15, X=FAKE, idx=FAKE, dist=FAKE, ws=FAKE, ws_bytes=1 << 30):
    return lib.rsc_knn(X, n, d, k, idx, dist, ws, ws_bytes, None)


def _err(lib):
    return lib.rsc_last_error().decode()


def _lib_mod():
    from paper_2603_02402_amd import _lib

    return _lib


def test_knn_validation(lib):
    assert _knn(lib, k=0) == -1
    assert _knn(lib, k=101) == -1
    assert _knn(lib, d=0) == -1
    assert _knn(lib, n=0) == -1
    assert _knn(lib, n=2**31) == -5 and "int32" in _err(lib)
    assert _knn(lib, d=257) == -6 and "256" in _err(lib)
    assert _knn(lib, k=256, n=1000) == -6 and "255" in _err(lib)
    # the reduced-precision screens stay at d <= 128, k <= 63
    bf = _lib_mod().KnnOpts(1, 0, 0, 0)
    assert lib.rsc_knn_opt(FAKE, 1000, 129, 15, ctypes.byref(bf), FAKE, FAKE, FAKE, 1 << 30, None) == -6
    assert lib.rsc_knn_opt(FAKE, 1000, 50, 64, ctypes.byref(bf), FAKE, FAKE, FAKE, 1 << 30, None) == -6
    # large k and d are sized on the exact path
    assert lib.rsc_knn_workspace_bytes(1000, 1000, 256, 255, None) > 0
    assert _knn(lib, X=None) == -1
    assert _knn(lib, idx=None) == -1
    assert _knn(lib, X=ctypes.c_void_p(0x10002)) == -1 and "aligned" in _err(lib)
    assert _knn(lib, ws=None) == -7
    assert _knn(lib, ws=ctypes.c_void_p(0x10080)) == -7
    assert _knn(lib, ws_bytes=1000) == -7 and "too small" in _err(lib)


def test_knn_ex_validation(lib):
    from paper_2603_02402_amd import _lib

    def call(nq=10, nr=100, d=50, k=15, opts=None):
        return lib.rsc_knn_ex(FAKE, nq, FAKE, nr, d, k, opts, FAKE, FAKE, FAKE, 1 << 30, None)

    assert call(k=101) == -1
    bad = _lib.KnnOpts(7, 0, 0, 0)
    assert call(opts=ctypes.byref(bad)) == -1
    narrow = _lib.KnnOpts(0, 15, 0, 0)
    assert call(opts=ctypes.byref(narrow)) == -1 and "screen" in _err(lib)
    wide = _lib.KnnOpts(0, 65, 0, 0)
    assert call(opts=ctypes.byref(wide)) == -1
    assert call(opts=ctypes.byref(_lib.KnnOpts(2, 100, 0, 0))) == -1 and "512" in _err(lib)
    assert lib.rsc_knn_workspace_bytes(1000, 1000, 50, 15, ctypes.byref(_lib.KnnOpts(2, 512, 0, 0))) > \
        lib.rsc_knn_workspace_bytes(1000, 1000, 50, 15, ctypes.byref(_lib.KnnOpts(2, 64, 0, 0)))


def test_connectivities_validation(lib):
    nnz = ctypes.c_int64(0)

    def call(n=100, k=15, cap=None, ws_bytes=1 << 30, idx=FAKE, nnz_p=ctypes.byref(nnz)):
        cap = 2 * n * (k - 1) if cap is None else cap
        return lib.rsc_connectivities(idx, FAKE, n, k, FAKE, FAKE, FAKE, cap, nnz_p, None, None, FAKE, ws_bytes,
                                      None)

    assert call(k=0) == -1
    assert call(k=101) == -1
    assert call(n=2**31) == -5
    assert call(cap=2 * 100 * 14 - 1) == -4 and "capacity" in _err(lib)
    assert call(ws_bytes=100) == -7
    assert call(idx=None) == -1
    assert call(nnz_p=None) == -1


def test_connectivities_noalloc_validation(lib):
    """The allocation-free call checks its arguments like rsc_connectivities
    and rejects a problem whose workspace exceeds its fixed scratch before
    touching the GPU."""
    cap_bytes = lib.rsc_connectivities_noalloc_max_bytes()
    assert cap_bytes == 64 << 20
    k = 15
    fits = 1000
    assert lib.rsc_connectivities_workspace_bytes(fits, k) <= cap_bytes
    big = 300000
    assert lib.rsc_connectivities_workspace_bytes(big, k) > cap_bytes
    nnz = ctypes.c_int64(0)

    def call(n, cap, idx=FAKE):
        return lib.rsc_connectivities_noalloc(idx, FAKE, n, k, FAKE, FAKE, FAKE, cap, ctypes.byref(nnz), None, None,
                                              None)

    assert call(big, 2 * big * (k - 1)) == -4  # RSC_ERR_CAPACITY: beyond the scratch
    assert "scratch" in _err(lib)
    assert call(fits, 2 * fits * (k - 1) - 1) == -4  # CSR capacity too small
    assert "capacity" in _err(lib)
    assert call(fits, 2 * fits * (k - 1), idx=None) == -1
    assert call(0, 1) == -1


def test_leiden_validation(lib):
    def call(n=100, nnz=1000, gamma=1.0, ptr=FAKE, idx=FAKE, w=FAKE, lab=FAKE, ws=FAKE, ws_bytes=1 << 30):
        return lib.rsc_leiden(ptr, idx, w, n, nnz, gamma, lab, None, ws, ws_bytes, None)

    assert call(n=0) == -1
    assert call(nnz=-1) == -1
    assert call(n=1 << 31) == -5  # RSC_ERR_OVERFLOW
    assert call(gamma=0.0) == -1 and "gamma" in _err(lib)
    assert call(gamma=float("inf")) == -1
    assert call(gamma=float("nan")) == -1
    assert call(ptr=None) == -1
    assert call(idx=None) == -1
    assert call(lab=None) == -1
    assert call(w=ctypes.c_void_p(0x10002)) == -1 and "misaligned" in _err(lib)
    assert lib.rsc_leiden_workspace_bytes(0, 10) == 0
    assert lib.rsc_leiden_workspace_bytes(10, -1) == 0


def test_connectivities_batched_validation(lib):
    import numpy as np

    nnz = ctypes.c_int64(0)

    def call(off, k=15, cap=None, ws_bytes=1 << 40, nnz_p=ctypes.byref(nnz)):
        off = np.ascontiguousarray(np.asarray(off, dtype=np.int64))
        n = int(off[-1])
        cap = 2 * n * (k - 1) if cap is None else cap
        return lib.rsc_connectivities_batched(FAKE, FAKE, off.ctypes.data_as(ctypes.c_void_p), len(off) - 1, k, FAKE,
                                              FAKE, FAKE, cap, nnz_p, ctypes.c_void_p(0x100000), ws_bytes, None)

    assert call([1, 100]) == -1 and "offsets" in _err(lib)
    assert call([0, 100, 110]) == -1 and "at least k" in _err(lib)
    assert call([0, 100], k=0) == -1
    assert call([0, 400], k=300) == -6
    assert call([0, 100, 300], cap=2 * 300 * 14 - 1) == -4
    assert call([0, 100, 300], ws_bytes=100) == -7
    assert call([0, 100, 300], nnz_p=None) == -1
    assert lib.rsc_connectivities_batched(FAKE, FAKE, None, 1, 15, FAKE, FAKE, FAKE, 1 << 20, ctypes.byref(nnz),
                                          FAKE, 1 << 40, None) == -1
    off = np.array([0, 100, 300], dtype=np.int64)
    p = off.ctypes.data_as(ctypes.c_void_p)
    # the batched workspace holds the single-graph one plus the offsets
    assert lib.rsc_connectivities_batched_workspace_bytes(p, 2, 15) >= lib.rsc_connectivities_workspace_bytes(300, 15)
    bad = np.array([0, 100, 105], dtype=np.int64)
    assert lib.rsc_connectivities_batched_workspace_bytes(bad.ctypes.data_as(ctypes.c_void_p), 2, 15) == 0


def test_error_is_thread_local_and_cleared(lib):
    assert _knn(lib, k=0) == -1
    assert _err(lib) != ""
    assert lib.rsc_knn_workspace_bytes(10, 10, 5, 3, None) > 0


def test_profile_calls_without_gpu(lib):
    assert lib.rsc_profile_enable(0) == 0
    assert lib.rsc_profile_reset() == 0
    ms = ctypes.c_double(-1)
    cnt = ctypes.c_int64(-1)
    assert lib.rsc_profile_get(b"screen_fp32", ctypes.byref(ms), ctypes.byref(cnt)) == 0
    assert ms.value == 0.0 and cnt.value == 0


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_2603_02402_amd import _lib

    with pytest.raises(ImportError):
        _lib.load.__wrapped__ if hasattr(_lib.load, "__wrapped__") else None
        saved = _lib._lib
        try:
            _lib._lib = None
            _lib.load(str(tmp_path / "missing.so"))
        finally:
            _lib._lib = saved


def test_batched_validation(lib):
    import numpy as np

    def call(off, d=50, k=15, ws_bytes=1 << 40):
        off = np.ascontiguousarray(np.asarray(off, dtype=np.int64))
        return lib.rsc_knn_batched(FAKE, off.ctypes.data_as(ctypes.c_void_p), len(off) - 1, d, k, FAKE, FAKE,
                                   ctypes.c_void_p(0x100000), ws_bytes, None)

    assert call([1, 100]) == -1 and "offsets[0]" in _err(lib)
    assert call([0, 100, 110]) == -1 and "at least k" in _err(lib)
    assert call([0, 100], k=64) == -6
    assert call([0, 100], d=0) == -1
    assert call([0, 100, 300], ws_bytes=100) == -7
    off = np.array([0, 100, 300], dtype=np.int64)
    p = off.ctypes.data_as(ctypes.c_void_p)
    assert lib.rsc_knn_batched_workspace_bytes(p, 2, 50, 15) > 0
    bad = np.array([0, 100, 105], dtype=np.int64)
    assert lib.rsc_knn_batched_workspace_bytes(bad.ctypes.data_as(ctypes.c_void_p), 2, 50, 15) == 0
    assert lib.rsc_batch_policy_name(0) != b""
    assert lib.rsc_batch_policy_name(99) == b""
    assert lib.rsc_batch_trial_name(0) == b""  # no autotune call yet
    assert lib.rsc_batch_trial_name(-1) == b""


def test_routed_validation(lib):
    from paper_2603_02402_amd import _lib

    st = _lib.RoutedStats()

    def probed(n=1000, d=50, k=15, parts=64, probes=8, ws_bytes=1 << 40, X=FAKE):
        return lib.rsc_knn_probed(X, n, d, k, FAKE, FAKE, parts, FAKE, probes, None, FAKE, FAKE, None,
                                  ctypes.byref(st), ctypes.c_void_p(0x100000), ws_bytes, None)

    assert probed(k=0) == -1
    assert probed(k=1001) == -1
    assert probed(parts=8193) == -6 and "8192" in _err(lib)
    assert probed(probes=65) == -6
    assert probed(d=129) == -6
    assert probed(n=2**31) == -5
    assert probed(X=None) == -1
    assert probed(ws_bytes=1000) == -7 and "workspace" in _err(lib)
    assert lib.rsc_knn_probed_workspace_bytes(1000, 50, 15, 64, 8) > 1000 * 8 * 4
    assert lib.rsc_knn_probed_workspace_bytes(1000, 50, 15, 9000, 8) == 0

    h = ctypes.c_void_p(0)
    assert lib.rsc_router_create(ctypes.byref(h), 50, 100, 64, 0) == -1 and "multiple of 64" in _err(lib)
    assert lib.rsc_router_create(ctypes.byref(h), 50, 64, 8192, 0) == -1
    assert lib.rsc_router_create(ctypes.byref(h), 0, 64, 64, 0) == -1
    assert lib.rsc_router_info(None, None, None, None, None, None) == -1
    assert lib.rsc_router_train_workspace_bytes(None, 64, 10) == 0
    assert lib.rsc_knn_routed_workspace_bytes(None, 10, 50, 5, 64, 8) == 0
    lib.rsc_router_destroy(None)

    def kmeans(n=1000, d=50, parts=64, iters=5, ws_bytes=1 << 40):
        return lib.rsc_partition_kmeans(FAKE, n, d, parts, FAKE, iters, FAKE, FAKE, None, None, None,
                                        ctypes.c_void_p(0x100000), ws_bytes, None)

    assert kmeans(parts=1001) == -1
    assert kmeans(iters=-1) == -1
    assert kmeans(d=129) == -1
    assert kmeans(ws_bytes=100) == -7
    assert lib.rsc_partition_kmeans_workspace_bytes(1000, 50, 64) > 1000 * 4
    assert lib.rsc_partition_kmeans_workspace_bytes(10, 50, 64) == 0
    assert lib.rsc_partition_lists(FAKE, 10, 0, FAKE, FAKE, ctypes.c_void_p(0x100000), 1 << 20, None) == -1
    assert lib.rsc_partition_labels(None, 10, 3, FAKE, 10, FAKE, None) == -1


def test_metric_validation(lib):
    from paper_2603_02402_amd import _lib

    bad = _lib.KnnOpts(0, 0, 2, 0)
    assert lib.rsc_knn_ex(FAKE, 10, FAKE, 100, 50, 15, ctypes.byref(bad), FAKE, FAKE, FAKE, 1 << 30, None) == -1
    assert "metric" in _err(lib)
    cos = _lib.KnnOpts(0, 0, 1, 0)
    eu = _lib.KnnOpts(0, 0, 0, 0)
    # the cosine form keeps the normalised rows in its workspace
    assert lib.rsc_knn_workspace_bytes(1000, 1000, 50, 15, ctypes.byref(cos)) > \
        lib.rsc_knn_workspace_bytes(1000, 1000, 50, 15, ctypes.byref(eu)) + 1000 * 50 * 4 - 1


def test_fp8_residual_validation(lib):
    from paper_2603_02402_amd import _lib

    def opts(prec, parts, metric=0):
        return _lib.KnnOpts(prec, 0, metric, parts)

    def call(o, n=1000):
        return lib.rsc_knn_opt(FAKE, n, 50, 15, ctypes.byref(o), FAKE, FAKE, FAKE, 1 << 40, None)

    assert call(opts(1, 16)) == -1 and "fp8_residual" in _err(lib)      # BF16 screen
    assert call(opts(0, 16)) == -1                                        # FP32 screen
    assert call(opts(2, 16, metric=1)) == -1                              # cosine metric
    assert call(opts(2, 1)) == -1 and "partition" in _err(lib)
    assert call(opts(2, 4097)) == -1
    assert call(opts(2, 1001)) == -1                                      # more partitions than rows
    assert lib.rsc_knn_workspace_bytes(1000, 1000, 50, 15, ctypes.byref(opts(2, 1001))) == 0
    # the residual variant holds its partitions, lists and map beyond the plain FP8 workspace
    plain = lib.rsc_knn_workspace_bytes(1000, 1000, 50, 15, ctypes.byref(opts(2, 0)))
    resid = lib.rsc_knn_workspace_bytes(1000, 1000, 50, 15, ctypes.byref(opts(2, 16)))
    assert resid > plain + 16 * 50 * 4 + 2 * 1000 * 4


def test_edistance_validation(lib):
    import numpy as np

    def call(offsets, G, pairs, n_pairs, ws_bytes=1 << 30, d=50):
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        pr = np.ascontiguousarray(pairs, dtype=np.int32)
        return lib.rsc_edistance_sums(FAKE, 1000, d, off.ctypes.data_as(ctypes.c_void_p), G, FAKE,
                                      pr.ctypes.data_as(ctypes.c_void_p), n_pairs, FAKE, FAKE, ws_bytes, None)

    good_pairs = [[0, 1], [1, 1]]
    assert call([1, 5, 9], 2, good_pairs, 2) == -1 and "offsets[0]" in _err(lib)
    assert call([0, 5, 3], 2, good_pairs, 2) == -1 and "non-decreasing" in _err(lib)
    assert call([0, 5, 9], 2, [[0, 2], [1, 1]], 2) == -1 and "out of range" in _err(lib)
    assert call([0, 5, 9], 2, [[-1, 0], [1, 1]], 2) == -1
    assert call([0, 5, 9], 0, good_pairs, 2) == -1
    assert call([0, 5, 9], 2, good_pairs, 2, d=0) == -1
    assert call([0, 5, 9], 2, good_pairs, 2, ws_bytes=16) == -7 and "workspace" in _err(lib)
    assert lib.rsc_edistance_sums_workspace_bytes(0, 5, 100, 50) == 0
    assert lib.rsc_edistance_sums_workspace_bytes(3, 5, 100, 0) == 0
    assert lib.rsc_edistance_pairwise_workspace_bytes(1000, 10**5, 50) > \
        lib.rsc_edistance_onesided_workspace_bytes(1000, 10**5, 50) > 10**5 * 50 * 4
    off = np.array([0, 5, 9], dtype=np.int64)
    assert lib.rsc_edistance_onesided(FAKE, 1000, 50, off.ctypes.data_as(ctypes.c_void_p), 2, FAKE, 2, FAKE, FAKE,
                                      1 << 30, None) == -1 and "reference" in _err(lib)


def test_edistance_groups_validation(lib):
    assert lib.rsc_edistance_groups(None, 10, 3, FAKE, FAKE, FAKE, 1 << 20, None) == -1
    assert lib.rsc_edistance_groups(FAKE, 0, 3, FAKE, FAKE, FAKE, 1 << 20, None) == -1
    assert lib.rsc_edistance_groups(FAKE, 10, 0, FAKE, FAKE, FAKE, 1 << 20, None) == -1
    assert "edistance_groups" in _err(lib)


def test_umap_validation(lib):
    def call(n=100, nnz=1000, dim=2, n_epochs=200, a=0.58, b=1.33, gamma=1.0, alpha0=1.0, neg=5, ws=1 << 30):
        return lib.rsc_umap_layout(FAKE, FAKE, FAKE, n, nnz, dim, FAKE, n_epochs, a, b, gamma, alpha0, neg,
                                   ctypes.c_uint64(0), FAKE, ws, None)

    assert lib.rsc_umap_layout(None, FAKE, FAKE, 100, 1000, 2, FAKE, 200, 0.58, 1.33, 1.0, 1.0, 5,
                               ctypes.c_uint64(0), FAKE, 1 << 30, None) == -1 and "null" in _err(lib)
    for bad in (dict(n=0), dict(dim=0), dict(dim=9), dict(n_epochs=0), dict(neg=-1), dict(neg=65), dict(a=0.0),
                dict(b=-1.0), dict(gamma=-0.5), dict(alpha0=0.0), dict(nnz=-1)):
        assert call(**bad) == -1, bad
    assert call(n_epochs=1 << 23) != 0 and "epochs" in _err(lib)
    assert call(nnz=1 << 32) != 0 and "2^32" in _err(lib)
    assert call(ws=64) == -7 and "workspace" in _err(lib)
    assert lib.rsc_umap_workspace_bytes(100, 1000, 9, 5) == 0
    assert lib.rsc_umap_workspace_bytes(100, 1000, 2, 65) == 0
    # float64 eps / next, uint32 positions / list / rows and two float64
    # embeddings; the moves live in LDS, so neg does not size it
    assert lib.rsc_umap_workspace_bytes(100, 1000, 2, 5) >= 1000 * (16 + 12) + 2 * 100 * 2 * 8
    assert lib.rsc_umap_workspace_bytes(100, 1000, 2, 5) == lib.rsc_umap_workspace_bytes(100, 1000, 2, 64)


def test_umap_default_curve_is_the_fit():
    # the binding's default (a, b) is the least-squares fit for min_dist 0.5,
    # spread 1 that the oracle computes
    from oracle import umap as ou

    import paper_2603_02402_amd as rsc

    a, b = ou.fit_ab(0.5, 1.0)
    assert abs(rsc.UMAP_A - a) < 1e-6 * a and abs(rsc.UMAP_B - b) < 1e-6 * b
