"""Python face of the Leiden call (argument marshalling only):
:func:`leiden` -> ``rsc_leiden``."""

from __future__ import annotations

import ctypes

from ._lib import LeidenStats, check, load


def leiden(graph, gamma: float = 1.0, workspace=None):
    """Leiden communities of a symmetric CSR graph (a :class:`Graph` or
    ``(indptr, indices, data)`` on the GPU).  Returns ``(labels, stats)``:
    labels a new int32 tensor numbered by first appearance; stats a dict of
    ``rsc_leiden_stats`` (quality = the modularity of the labels)."""
    import torch

    from . import Workspace

    if hasattr(graph, "indptr"):
        indptr, indices, data = graph.indptr, graph.indices, graph.data
    else:
        indptr, indices, data = graph
    for t in (indptr, indices, data):
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError("graph arrays must be contiguous GPU tensors")
    if indptr.dtype != torch.int64 or indices.dtype != torch.int32 or data.dtype != torch.float32:
        raise ValueError("graph arrays must be int64 indptr, int32 indices, float32 data")
    n = indptr.numel() - 1
    nnz = indices.numel()
    lib = load()
    need = lib.rsc_leiden_workspace_bytes(n, nnz)
    if need == 0:
        raise ValueError("leiden: unsupported size (1 <= n <= 2^31 - 2, 0 <= nnz <= 2^40)")
    ws = (workspace or Workspace(indptr.device)).get(need)
    labels = torch.empty(n, dtype=torch.int32, device=indptr.device)
    st = LeidenStats()
    check(lib.rsc_leiden(ctypes.c_void_p(indptr.data_ptr()), ctypes.c_void_p(indices.data_ptr()),
                         ctypes.c_void_p(data.data_ptr()), n, nnz, gamma, ctypes.c_void_p(labels.data_ptr()),
                         ctypes.byref(st), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                         ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
    return labels, {f: getattr(st, f) for f, _ in st._fields_ if f != "reserved"}
