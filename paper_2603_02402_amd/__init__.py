"""MI355X-native kNN graph: exact kNN, smooth-kNN rho/sigma, fuzzy-union CSR.

Python face of ``librsc.so`` (C ABI in ``include/rsc.h``).  Inputs and
outputs are torch tensors on the current HIP device; work is enqueued on
torch's current stream.  Functions mirror the C calls:

* :func:`knn`             -> ``rsc_knn`` / ``rsc_knn_ex``
* :func:`connectivities`  -> ``rsc_connectivities``
* :func:`knn_graph`       -> both, the whole neighbourhood-graph step
* :func:`knn_batched`     -> ``rsc_knn_batched`` (many samples, one launch)
* :func:`connectivities_batched` -> ``rsc_connectivities_batched``
* :func:`connectivities_noalloc` -> ``rsc_connectivities_noalloc``
* :mod:`.routed`          -> partitions, the router network, probed and
  routed kNN (``rsc_partition_*``, ``rsc_router_*``, ``rsc_knn_probed``,
  ``rsc_knn_routed``)
* :mod:`.edistance`       -> energy distances between groups of cells
  (``rsc_edistance_*``)
* :mod:`.pca`             -> the sparse PCA that produces the embedding
  (``rsc_pca``, ``rsc_pca_covariance``)
* :mod:`.umap`            -> the UMAP layout of the graph (``rsc_umap_layout``)
* :mod:`.leiden`          -> Leiden communities of the graph (``rsc_leiden``)
"""

from __future__ import annotations

import ctypes
from dataclasses import dataclass

from . import _lib
from ._lib import (RSC_BF16, RSC_COSINE, RSC_EUCLIDEAN, RSC_FP8_E4M3, RSC_FP32, KnnOpts, KnnStats, RscError,
                   check, load)

__all__ = [
    "knn", "knn_graph", "connectivities", "knn_workspace_bytes", "connectivities_workspace_bytes",
    "read_knn_stats", "profile_enable", "profile_reset", "profile_get", "RscError", "Workspace",
    "RSC_FP32", "RSC_BF16", "RSC_FP8_E4M3", "RSC_EUCLIDEAN", "RSC_COSINE", "abi_version", "knn_batched", "knn_batched_autotune",
    "knn_batched_workspace_bytes", "connectivities_batched", "Router", "partition_kmeans", "partition_lists", "partition_labels",
    "knn_probed", "knn_routed", "edistance_groups", "edistance_sums", "edistance_pairwise", "edistance_onesided",
    "pca", "pca_covariance", "umap_layout", "UMAP_A", "UMAP_B", "leiden",
]


def _torch():
    import torch

    return torch


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check_dev(*ts):
    for t in ts:
        if t is not None and not t.is_cuda:
            raise ValueError("tensors must live on the GPU")
        if t is not None and not t.is_contiguous():
            raise ValueError("tensors must be contiguous")


def abi_version() -> int:
    return int(load().rsc_abi_version())


def _opts(precision: int = RSC_FP32, screen: int = 0, metric: int = RSC_EUCLIDEAN, fp8_residual: int = 0):
    return KnnOpts(precision, screen, metric, fp8_residual)


def knn_workspace_bytes(n_query: int, n_ref: int, d: int, k: int, precision: int = RSC_FP32,
                        screen: int = 0, metric: int = RSC_EUCLIDEAN, fp8_residual: int = 0) -> int:
    o = _opts(precision, screen, metric, fp8_residual)
    return int(load().rsc_knn_workspace_bytes(n_query, n_ref, d, k, ctypes.byref(o)))


def connectivities_workspace_bytes(n: int, k: int) -> int:
    return int(load().rsc_connectivities_workspace_bytes(n, k))


class Workspace:
    """A reusable device byte buffer that grows on demand."""

    def __init__(self, device=None):
        self.device = device
        self.buf = None

    def get(self, nbytes: int):
        torch = _torch()
        nbytes = max(int(nbytes), 256)
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = torch.empty(nbytes, dtype=torch.uint8, device=self.device or "cuda")
        return self.buf


def knn(X, k: int, Q=None, precision: int = RSC_FP32, screen: int = 0, out=None, workspace: Workspace | None = None,
        metric: int = RSC_EUCLIDEAN, fp8_residual: int = 0):
    """k nearest neighbours.

    ``knn(X, k)``: every row of ``X`` (n x d float32) among the rows of ``X``;
    column 0 is the row itself.  ``knn(X, k, Q=Q)``: rows of ``Q`` among
    the rows of ``X`` (all k columns from ``X``).  ``precision`` selects the
    screen (``RSC_FP32`` exact; ``RSC_BF16`` / ``RSC_FP8_E4M3`` approximate,
    re-ranked in float64; ``fp8_residual`` = P selects the FP8 screen's
    residual variant over P partitions).  Returns ``(idx int32, dist float32)``, each
    ``n_query x k``.
    """
    torch = _torch()
    _check_dev(X, Q)
    if X.dtype != torch.float32 or X.dim() != 2:
        raise ValueError("X must be a 2-D float32 tensor")
    n, d = X.shape
    nq = n if Q is None else Q.shape[0]
    if Q is not None and (Q.dtype != torch.float32 or Q.dim() != 2 or Q.shape[1] != d):
        raise ValueError("Q must be a float32 tensor with X's column count")
    lib = load()
    o = _opts(precision, screen, metric, fp8_residual)
    need = lib.rsc_knn_workspace_bytes(nq, n, d, k, ctypes.byref(o))
    if need == 0:
        # invalid sizes: let the call itself report the reason
        need = 256
    ws = (workspace or Workspace(X.device)).get(need)
    if out is None:
        idx = torch.empty((nq, k), dtype=torch.int32, device=X.device)
        dist = torch.empty((nq, k), dtype=torch.float32, device=X.device)
    else:
        idx, dist = out
    if Q is None and precision == RSC_FP32 and screen == 0 and metric == RSC_EUCLIDEAN and fp8_residual == 0:
        st = lib.rsc_knn(_ptr(X), n, d, k, _ptr(idx), _ptr(dist), _ptr(ws), ws.numel(), _stream())
    elif Q is None:
        st = lib.rsc_knn_opt(_ptr(X), n, d, k, ctypes.byref(o), _ptr(idx), _ptr(dist), _ptr(ws), ws.numel(),
                             _stream())
    else:
        st = lib.rsc_knn_ex(_ptr(Q), nq, _ptr(X), n, d, k, ctypes.byref(o), _ptr(idx), _ptr(dist), _ptr(ws),
                            ws.numel(), _stream())
    check(st)
    return idx, dist


def read_knn_stats(workspace: Workspace) -> dict:
    s = KnnStats()
    ws = workspace.buf
    check(load().rsc_knn_read_stats(_ptr(ws), ws.numel(), ctypes.byref(s), _stream()))
    return {"escalated_rows": int(s.escalated_rows), "rescanned_rows": int(s.rescanned_rows),
            "max_err_ratio": float(s.max_err_ratio),
            "max_ref_norm": float(s.max_ref_norm)}


def read_knn_escalated(workspace: Workspace, n_query: int, n_ref: int, d: int, k: int, opts=None,
                       square: bool = True):
    """Sorted rows whose first certificate failed in the last kNN call on
    ``workspace`` (``rsc_knn_read_escalated``); sizes and options as in that call."""
    import numpy as np

    ws = workspace.buf
    count = ctypes.c_int64(0)
    o = ctypes.byref(opts) if opts is not None else None
    lib = load()
    check(lib.rsc_knn_read_escalated(_ptr(ws), ws.numel(), n_query, n_ref, d, k, o, int(square), None, 0,
                                     ctypes.byref(count), _stream()))
    rows = np.zeros(max(int(count.value), 1), dtype=np.int32)
    check(lib.rsc_knn_read_escalated(_ptr(ws), ws.numel(), n_query, n_ref, d, k, o, int(square),
                                     rows.ctypes.data_as(ctypes.c_void_p), rows.size, ctypes.byref(count),
                                     _stream()))
    return np.sort(rows[: int(count.value)])


@dataclass
class Graph:
    indptr: object
    indices: object
    data: object
    rho: object
    sigma: object

    @property
    def nnz(self) -> int:
        return int(self.indices.numel())


def connectivities(idx, dist, want_rho_sigma: bool = True, workspace: Workspace | None = None, out=None):
    """Fuzzy simplicial set of a kNN result as CSR (see ``rsc_connectivities``)."""
    torch = _torch()
    _check_dev(idx, dist)
    if idx.dtype != torch.int32 or dist.dtype != torch.float32 or idx.shape != dist.shape or idx.dim() != 2:
        raise ValueError("idx (int32) and dist (float32) must be n x k")
    n, k = idx.shape
    lib = load()
    need = lib.rsc_connectivities_workspace_bytes(n, k)
    ws = (workspace or Workspace(idx.device)).get(need if need else 256)
    cap = max(1, 2 * n * (k - 1))
    if out is None:
        indptr = torch.empty(n + 1, dtype=torch.int64, device=idx.device)
        indices = torch.empty(cap, dtype=torch.int32, device=idx.device)
        data = torch.empty(cap, dtype=torch.float32, device=idx.device)
    else:
        indptr, indices, data = out
        cap = indices.numel()
    rho = torch.empty(n, dtype=torch.float64, device=idx.device) if want_rho_sigma else None
    sigma = torch.empty(n, dtype=torch.float64, device=idx.device) if want_rho_sigma else None
    nnz = ctypes.c_int64(0)
    st = lib.rsc_connectivities(_ptr(idx), _ptr(dist), n, k, _ptr(indptr), _ptr(indices), _ptr(data), cap,
                                ctypes.byref(nnz), _ptr(rho), _ptr(sigma), _ptr(ws), ws.numel(), _stream())
    check(st)
    m = int(nnz.value)
    return Graph(indptr, indices[:m], data[:m], rho, sigma)


def connectivities_noalloc(idx, dist, out, rho=None, sigma=None):
    """``rsc_connectivities_noalloc``: the same CSR as :func:`connectivities`,
    written into the caller's ``out = (indptr, indices, data)`` with the
    library's fixed scratch instead of a workspace; ``rho`` / ``sigma`` are
    optional float64 outputs.  Returns the nnz."""
    torch = _torch()
    _check_dev(idx, dist)
    if idx.dtype != torch.int32 or dist.dtype != torch.float32 or idx.shape != dist.shape or idx.dim() != 2:
        raise ValueError("idx (int32) and dist (float32) must be n x k")
    n, k = idx.shape
    indptr, indices, data = out
    nnz = ctypes.c_int64(0)
    st = load().rsc_connectivities_noalloc(_ptr(idx), _ptr(dist), n, k, _ptr(indptr), _ptr(indices), _ptr(data),
                                           indices.numel(), ctypes.byref(nnz), _ptr(rho), _ptr(sigma), _stream())
    check(st)
    return int(nnz.value)


def knn_graph(X, k: int, workspace: Workspace | None = None, metric: int = RSC_EUCLIDEAN):
    """The whole step: ``(idx, dist, Graph)``."""
    ws = workspace or Workspace(X.device)
    idx, dist = knn(X, k, workspace=ws, metric=metric)
    g = connectivities(idx, dist, workspace=ws)
    return idx, dist, g


def _host_offsets(offsets):
    import numpy as np

    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    return off, off.ctypes.data_as(ctypes.c_void_p)


def knn_batched_workspace_bytes(offsets, d: int, k: int) -> int:
    off, p = _host_offsets(offsets)
    return int(load().rsc_knn_batched_workspace_bytes(p, len(off) - 1, d, k))


def knn_batched(X, offsets, k: int, out=None, workspace: Workspace | None = None):
    """Exact kNN of every sample of a batch (rows ``offsets[s]..offsets[s+1]-1``
    of ``X``; ``offsets`` on the host).  Returns global-row ``(idx, dist)``."""
    torch = _torch()
    _check_dev(X)
    n, d = X.shape
    off, p = _host_offsets(offsets)
    S = len(off) - 1
    lib = load()
    need = lib.rsc_knn_batched_workspace_bytes(p, S, d, k)
    ws = (workspace or Workspace(X.device)).get(need if need else 256)
    if out is None:
        idx = torch.empty((n, k), dtype=torch.int32, device=X.device)
        dist = torch.empty((n, k), dtype=torch.float32, device=X.device)
    else:
        idx, dist = out
    check(lib.rsc_knn_batched(_ptr(X), p, S, d, k, _ptr(idx), _ptr(dist), _ptr(ws), ws.numel(), _stream()))
    return idx, dist


def connectivities_batched(idx, dist, offsets, workspace: Workspace | None = None, out=None):
    """Per-sample fuzzy simplicial sets of a batched kNN result as one
    block-diagonal CSR (``offsets`` on the host; see
    ``rsc_connectivities_batched``).  Returns a :class:`Graph` without
    rho/sigma."""
    torch = _torch()
    _check_dev(idx, dist)
    if idx.dtype != torch.int32 or dist.dtype != torch.float32 or idx.shape != dist.shape or idx.dim() != 2:
        raise ValueError("idx (int32) and dist (float32) must be n x k")
    n, k = idx.shape
    off, p = _host_offsets(offsets)
    S = len(off) - 1
    lib = load()
    need = lib.rsc_connectivities_batched_workspace_bytes(p, S, k)
    ws = (workspace or Workspace(idx.device)).get(need if need else 256)
    cap = max(1, 2 * n * (k - 1))
    if out is None:
        indptr = torch.empty(n + 1, dtype=torch.int64, device=idx.device)
        indices = torch.empty(cap, dtype=torch.int32, device=idx.device)
        data = torch.empty(cap, dtype=torch.float32, device=idx.device)
    else:
        indptr, indices, data = out
        cap = indices.numel()
    nnz = ctypes.c_int64(0)
    check(lib.rsc_connectivities_batched(_ptr(idx), _ptr(dist), p, S, k, _ptr(indptr), _ptr(indices), _ptr(data),
                                         cap, ctypes.byref(nnz), _ptr(ws), ws.numel(), _stream()))
    m = int(nnz.value)
    return Graph(indptr, indices[:m], data[:m], None, None)


def knn_batched_autotune(X, offsets, k: int, workspace: Workspace | None = None):
    """Choose the batched tile shape and schedule by measurement; returns
    ``(chosen_trial, {trial_description: ms})`` (see ``rsc_knn_batched_autotune``)."""
    _check_dev(X)
    n, d = X.shape
    off, p = _host_offsets(offsets)
    S = len(off) - 1
    lib = load()
    need = lib.rsc_knn_batched_workspace_bytes(p, S, d, k)
    ws = (workspace or Workspace(X.device)).get(need if need else 256)
    chosen = ctypes.c_int32(-1)
    times = (ctypes.c_float * _lib.RSC_BATCH_TRIALS)()
    check(lib.rsc_knn_batched_autotune(_ptr(X), p, S, d, k, _ptr(ws), ws.numel(), _stream(), ctypes.byref(chosen),
                                       times))
    table = {}
    for i in range(_lib.RSC_BATCH_TRIALS):
        name = lib.rsc_batch_trial_name(i).decode()
        if not name:
            break
        table[name] = float(times[i])
    return int(chosen.value), table


def profile_enable(on: bool = True) -> None:
    check(load().rsc_profile_enable(1 if on else 0))


def profile_reset() -> None:
    check(load().rsc_profile_reset())


def profile_get(name: str):
    ms = ctypes.c_double(0)
    cnt = ctypes.c_int64(0)
    check(load().rsc_profile_get(name.encode(), ctypes.byref(ms), ctypes.byref(cnt)))
    return float(ms.value), int(cnt.value)


from .routed import (Router, knn_probed, knn_routed, partition_kmeans, partition_labels,  # noqa: E402
                     partition_lists)
from .edistance import (edistance_groups, edistance_onesided, edistance_pairwise,  # noqa: E402
                        edistance_sums)
from .pca import pca, pca_covariance  # noqa: E402
from .umap import UMAP_A, UMAP_B, umap_layout  # noqa: E402
from .leiden import leiden  # noqa: E402
