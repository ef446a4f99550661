"""Python face of the energy-distance calls (argument marshalling only).

Mirrors ``include/rsc.h``:

* :func:`edistance_groups`    -> ``rsc_edistance_groups`` (category offsets and
  the cell-index array of integer labels, stable radix sort on the GPU)
* :func:`edistance_sums`      -> ``rsc_edistance_sums``
* :func:`edistance_pairwise`  -> ``rsc_edistance_pairwise``
* :func:`edistance_onesided`  -> ``rsc_edistance_onesided``

``offsets`` are host int64 (G + 1); ``cells`` and ``X`` live on the current
HIP device; work goes to torch's current stream.
"""

from __future__ import annotations

import ctypes

import numpy as np

from ._lib import check, load


def _torch():
    import torch

    return torch


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _host_i64(a) -> np.ndarray:
    if hasattr(a, "cpu"):
        a = a.cpu().numpy()
    return np.ascontiguousarray(a, dtype=np.int64)


def _check(X, cells):
    torch = _torch()
    for t in (X, cells):
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError("X and cells must be contiguous GPU tensors")
    if X.dtype != torch.float32 or X.dim() != 2:
        raise ValueError("X must be a 2-D float32 tensor")
    if cells.dtype != torch.int32:
        raise ValueError("cells must be int32")


def _ws(workspace, nbytes, device):
    from . import Workspace

    return (workspace or Workspace(device)).get(nbytes if nbytes else 256)


def edistance_groups(labels, n_groups: int, workspace=None):
    """``(offsets host int64 G+1, cells device int32)`` of device int32 labels
    in [0, G): each group's rows in ascending order (``rsc_edistance_groups``)."""
    torch = _torch()
    if not labels.is_cuda or not labels.is_contiguous() or labels.dtype != torch.int32:
        raise ValueError("labels must be a contiguous int32 GPU tensor")
    n = labels.numel()
    lib = load()
    ws = _ws(workspace, lib.rsc_edistance_groups_workspace_bytes(n, n_groups), labels.device)
    offsets = torch.empty(n_groups + 1, dtype=torch.int64, device=labels.device)
    cells = torch.empty(max(n, 1), dtype=torch.int32, device=labels.device)[:n]
    check(lib.rsc_edistance_groups(_ptr(labels), n, n_groups, _ptr(offsets), _ptr(cells), _ptr(ws), ws.numel(),
                                   _stream()))
    return offsets.cpu().numpy(), cells


def edistance_sums(X, offsets, cells, pairs, workspace=None):
    """Sums of distances of the listed group pairs (host int32 n x 2):
    ``device float64 [n_pairs]``."""
    torch = _torch()
    _check(X, cells)
    off = _host_i64(offsets)
    pr = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    G = off.size - 1
    lib = load()
    ws = _ws(workspace, lib.rsc_edistance_sums_workspace_bytes(G, pr.shape[0], int(off[-1]), X.shape[1]), X.device)
    sums = torch.empty(max(pr.shape[0], 1), dtype=torch.float64, device=X.device)[:pr.shape[0]]
    check(lib.rsc_edistance_sums(_ptr(X), X.shape[0], X.shape[1], off.ctypes.data_as(ctypes.c_void_p), G,
                                 _ptr(cells), pr.ctypes.data_as(ctypes.c_void_p), pr.shape[0], _ptr(sums), _ptr(ws),
                                 ws.numel(), _stream()))
    return sums


def edistance_pairwise(X, offsets, cells, want_means: bool = False, workspace=None):
    """``E`` (G x G float64; with ``want_means`` also the mean distances D)."""
    torch = _torch()
    _check(X, cells)
    off = _host_i64(offsets)
    G = off.size - 1
    lib = load()
    ws = _ws(workspace, lib.rsc_edistance_pairwise_workspace_bytes(G, int(off[-1]), X.shape[1]), X.device)
    E = torch.empty((G, G), dtype=torch.float64, device=X.device)
    D = torch.empty((G, G), dtype=torch.float64, device=X.device) if want_means else None
    check(lib.rsc_edistance_pairwise(_ptr(X), X.shape[0], X.shape[1], off.ctypes.data_as(ctypes.c_void_p), G,
                                     _ptr(cells), _ptr(E), _ptr(D), _ptr(ws), ws.numel(), _stream()))
    return (E, D) if want_means else E


def edistance_onesided(X, offsets, cells, ref: int, workspace=None):
    """E from group ``ref`` to every group (float64 [G], E[ref] = 0)."""
    torch = _torch()
    _check(X, cells)
    off = _host_i64(offsets)
    G = off.size - 1
    lib = load()
    ws = _ws(workspace, lib.rsc_edistance_onesided_workspace_bytes(G, int(off[-1]), X.shape[1]), X.device)
    E = torch.empty(G, dtype=torch.float64, device=X.device)
    check(lib.rsc_edistance_onesided(_ptr(X), X.shape[0], X.shape[1], off.ctypes.data_as(ctypes.c_void_p), G,
                                     _ptr(cells), int(ref), _ptr(E), _ptr(ws), ws.numel(), _stream()))
    return E
