"""Python face of the sparse-PCA calls (argument marshalling only).

* :func:`pca_covariance` -> ``rsc_pca_covariance``
* :func:`pca`            -> ``rsc_pca``

The CSR arrays (``indptr`` int64, ``indices`` int32, ``data`` float32) live
on the current HIP device; work goes to torch's current stream.
"""

from __future__ import annotations

import ctypes

from ._lib import check, load


def _torch():
    import torch

    return torch


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _check_csr(indptr, indices, data):
    torch = _torch()
    for t, dt in ((indptr, torch.int64), (indices, torch.int32), (data, torch.float32)):
        if not t.is_cuda or not t.is_contiguous() or t.dtype != dt:
            raise ValueError("CSR arrays must be contiguous GPU tensors (int64 indptr, int32 indices, float32 data)")


def _ws(workspace, nbytes, device):
    from . import Workspace

    return (workspace or Workspace(device)).get(nbytes if nbytes else 256)


def pca_covariance(indptr, indices, data, p: int, workspace=None):
    """``(mean float64 [p], cov float64 [p, p])`` of a cells x genes CSR matrix."""
    torch = _torch()
    _check_csr(indptr, indices, data)
    n = indptr.numel() - 1
    lib = load()
    ws = _ws(workspace, lib.rsc_pca_workspace_bytes(n, p, 0), indptr.device)
    mean = torch.empty(p, dtype=torch.float64, device=indptr.device)
    cov = torch.empty((p, p), dtype=torch.float64, device=indptr.device)
    check(lib.rsc_pca_covariance(_ptr(indptr), _ptr(indices), _ptr(data), n, p, _ptr(mean), _ptr(cov), _ptr(ws),
                                 ws.numel(), _stream()))
    return mean, cov


def pca(indptr, indices, data, p: int, k: int, want_cov: bool = False, workspace=None):
    """``(mean, evals, loadings [p, k], scores float32 [n, k])`` (+ cov)."""
    torch = _torch()
    _check_csr(indptr, indices, data)
    n = indptr.numel() - 1
    lib = load()
    need = lib.rsc_pca_workspace_bytes(n, p, k)
    ws = _ws(workspace, need, indptr.device)
    dev = indptr.device
    mean = torch.empty(p, dtype=torch.float64, device=dev)
    cov = torch.empty((p, p), dtype=torch.float64, device=dev) if want_cov else None
    evals = torch.empty(k, dtype=torch.float64, device=dev)
    loadings = torch.empty((p, k), dtype=torch.float64, device=dev)
    scores = torch.empty((n, k), dtype=torch.float32, device=dev)
    check(lib.rsc_pca(_ptr(indptr), _ptr(indices), _ptr(data), n, p, k, _ptr(mean), _ptr(cov), _ptr(evals),
                      _ptr(loadings), _ptr(scores), _ptr(ws), ws.numel(), _stream()))
    return (mean, evals, loadings, scores, cov) if want_cov else (mean, evals, loadings, scores)
