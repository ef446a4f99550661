"""Python face of the UMAP layout call (argument marshalling only):
:func:`umap_layout` -> ``rsc_umap_layout``."""

from __future__ import annotations

import ctypes

from ._lib import check, load

# the least-squares fit of UMAP's similarity curve for min_dist 0.5, spread 1
UMAP_A, UMAP_B = 0.5830300203414425, 1.3341669924314914


def umap_layout(graph, Y0, n_epochs: int = 200, a: float = UMAP_A, b: float = UMAP_B, gamma: float = 1.0,
                alpha0: float = 1.0, neg: int = 5, seed: int = 0, workspace=None):
    """Lay out the graph (a :class:`Graph` or ``(indptr, indices, data)``)
    starting from ``Y0`` (float32 [n, dim] on the GPU); returns the layout
    (a new float32 tensor)."""
    import torch

    from . import Workspace

    if hasattr(graph, "indptr"):
        indptr, indices, data = graph.indptr, graph.indices, graph.data
    else:
        indptr, indices, data = graph
    for t in (indptr, indices, data, Y0):
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError("graph arrays and Y0 must be contiguous GPU tensors")
    if Y0.dtype != torch.float32 or Y0.dim() != 2:
        raise ValueError("Y0 must be a float32 [n, dim] tensor")
    n, dim = Y0.shape
    nnz = indices.numel()
    Y = Y0.clone()
    lib = load()
    need = lib.rsc_umap_workspace_bytes(n, nnz, dim, neg)
    if need == 0:
        raise ValueError("umap_layout: unsupported shape (n < 2^31, nnz < 2^32 - 1, 1 <= dim <= 8, 0 <= neg <= 64)")
    ws = (workspace or Workspace(Y.device)).get(need if need else 256)
    check(lib.rsc_umap_layout(ctypes.c_void_p(indptr.data_ptr()), ctypes.c_void_p(indices.data_ptr()),
                              ctypes.c_void_p(data.data_ptr()), n, nnz, dim, ctypes.c_void_p(Y.data_ptr()), n_epochs,
                              a, b, gamma, alpha0, neg, ctypes.c_uint64(seed), ctypes.c_void_p(ws.data_ptr()),
                              ws.numel(), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
    return Y
