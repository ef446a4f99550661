"""Python face of the routed form (argument marshalling only).

Mirrors the C calls of ``include/rsc.h``:

* :func:`partition_kmeans`  -> ``rsc_partition_kmeans``
* :func:`partition_lists`   -> ``rsc_partition_lists``
* :func:`partition_labels`  -> ``rsc_partition_labels``
* :class:`Router`           -> ``rsc_router_*``
* :func:`knn_probed`        -> ``rsc_knn_probed``
* :func:`knn_routed`        -> ``rsc_knn_routed``

Tensors live on the current HIP device; work goes to torch's current stream.
"""

from __future__ import annotations

import ctypes

from ._lib import RoutedStats, check, load


def _torch():
    import torch

    return torch


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _check_dev(*ts):
    for t in ts:
        if t is not None and (not t.is_cuda or not t.is_contiguous()):
            raise ValueError("tensors must be contiguous and on the GPU")


def _ws(workspace, nbytes, device):
    from . import Workspace

    return (workspace or Workspace(device)).get(nbytes if nbytes else 256)


def partition_kmeans(X, parts: int, init_rows, iters: int, lists: bool = True, workspace=None):
    """Lloyd's k-means of the rows of ``X`` (see ``rsc_partition_kmeans``).

    ``init_rows``: device int32 row ids of the initial centroids.  Returns
    ``(centroids, assign, offsets, perm, relocated)`` (offsets/perm None
    unless ``lists``).
    """
    torch = _torch()
    _check_dev(X, init_rows)
    n, d = X.shape
    lib = load()
    ws = _ws(workspace, lib.rsc_partition_kmeans_workspace_bytes(n, d, parts), X.device)
    C = torch.empty((parts, d), dtype=torch.float32, device=X.device)
    assign = torch.empty(n, dtype=torch.int32, device=X.device)
    offsets = torch.empty(parts + 1, dtype=torch.int64, device=X.device) if lists else None
    perm = torch.empty(n, dtype=torch.int32, device=X.device) if lists else None
    rel = ctypes.c_int64(0)
    check(lib.rsc_partition_kmeans(_ptr(X), n, d, parts, _ptr(init_rows), iters, _ptr(C), _ptr(assign),
                                   _ptr(offsets), _ptr(perm), ctypes.byref(rel), _ptr(ws), ws.numel(), _stream()))
    return C, assign, offsets, perm, int(rel.value)


def partition_lists(labels, parts: int, workspace=None):
    """Inverted lists ``(offsets int64, perm int32)`` of device labels."""
    torch = _torch()
    _check_dev(labels)
    n = labels.numel()
    lib = load()
    ws = _ws(workspace, lib.rsc_partition_lists_workspace_bytes(parts), labels.device)
    offsets = torch.empty(parts + 1, dtype=torch.int64, device=labels.device)
    perm = torch.empty(n, dtype=torch.int32, device=labels.device)
    check(lib.rsc_partition_lists(_ptr(labels), n, parts, _ptr(offsets), _ptr(perm), _ptr(ws), ws.numel(),
                                  _stream()))
    return offsets, perm


def partition_labels(idx, assign):
    """``assign[idx]`` for an n x k kNN result (-1 where idx is out of range)."""
    torch = _torch()
    _check_dev(idx, assign)
    n, k = idx.shape
    labels = torch.empty((n, k), dtype=torch.int32, device=idx.device)
    check(load().rsc_partition_labels(_ptr(idx), n, k, _ptr(assign), assign.numel(), _ptr(labels), _stream()))
    return labels


class Router:
    """The partition router network; owns its device weights."""

    def __init__(self, d: int, hidden: int, parts: int, seed: int = 0):
        self._h = ctypes.c_void_p(0)
        check(load().rsc_router_create(ctypes.byref(self._h), d, hidden, parts, seed))
        self.d, self.hidden, self.parts = d, hidden, parts

    def close(self):
        if self._h:
            load().rsc_router_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        d, h, p = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        npar, steps = ctypes.c_int64(), ctypes.c_int64()
        check(load().rsc_router_info(self._h, ctypes.byref(d), ctypes.byref(h), ctypes.byref(p),
                                     ctypes.byref(npar), ctypes.byref(steps)))
        return {"d": d.value, "hidden": h.value, "parts": p.value, "n_params": npar.value, "steps": steps.value}

    def train(self, X, labels, epochs: int, batch: int, lr: float, workspace=None, log: bool = True):
        """Adam over ``epochs`` passes; returns the per-epoch mean losses (host)."""
        _check_dev(X, labels)
        n = X.shape[0]
        m = labels.shape[1]
        lib = load()
        ws = _ws(workspace, lib.rsc_router_train_workspace_bytes(self._h, batch, n), X.device)
        losses = (ctypes.c_float * epochs)() if log else None
        check(lib.rsc_router_train(self._h, _ptr(X), n, _ptr(labels), m, epochs, batch, lr, losses, _ptr(ws),
                                   ws.numel(), _stream()))
        return [float(v) for v in losses] if log else None

    def gradients(self, X, labels, workspace=None):
        """``(grad float32 n_params, loss float32 1)`` at the current weights."""
        torch = _torch()
        _check_dev(X, labels)
        n = X.shape[0]
        lib = load()
        ws = _ws(workspace, lib.rsc_router_gradients_workspace_bytes(self._h, n), X.device)
        grad = torch.empty(self.info()["n_params"], dtype=torch.float32, device=X.device)
        loss = torch.empty(1, dtype=torch.float32, device=X.device)
        check(lib.rsc_router_gradients(self._h, _ptr(X), n, _ptr(labels), labels.shape[1], _ptr(grad), _ptr(loss),
                                       _ptr(ws), ws.numel(), _stream()))
        return grad, loss

    def logits(self, X, workspace=None):
        torch = _torch()
        _check_dev(X)
        n = X.shape[0]
        lib = load()
        ws = _ws(workspace, lib.rsc_router_infer_workspace_bytes(self._h), X.device)
        z = torch.empty((n, self.parts), dtype=torch.float32, device=X.device)
        check(lib.rsc_router_logits(self._h, _ptr(X), n, _ptr(z), _ptr(ws), ws.numel(), _stream()))
        return z

    def probe(self, X, probes: int, workspace=None):
        """``(parts int32 n x probes, mass float32 n)``."""
        torch = _torch()
        _check_dev(X)
        n = X.shape[0]
        lib = load()
        ws = _ws(workspace, lib.rsc_router_infer_workspace_bytes(self._h), X.device)
        parts = torch.empty((n, probes), dtype=torch.int32, device=X.device)
        mass = torch.empty(n, dtype=torch.float32, device=X.device)
        check(lib.rsc_router_probe(self._h, _ptr(X), n, probes, _ptr(parts), _ptr(mass), _ptr(ws), ws.numel(),
                                   _stream()))
        return parts, mass

    def save(self, path: str):
        check(load().rsc_router_save(self._h, str(path).encode()))

    def load_file(self, path: str):
        check(load().rsc_router_load(self._h, str(path).encode()))


def _stats_dict(s: RoutedStats) -> dict:
    return {f: (float(getattr(s, f)) if f.startswith("mean_") else int(getattr(s, f))) for f, _ in s._fields_}


def _out(n, k, device, out):
    torch = _torch()
    if out is not None:
        return out
    return (torch.empty((n, k), dtype=torch.int32, device=device),
            torch.empty((n, k), dtype=torch.float32, device=device))


def knn_probed(X, k: int, offsets, perm, probe_parts, exact_rows=None, out=None, workspace=None):
    """kNN of every row within the partitions it probes (``rsc_knn_probed``).
    Returns ``(idx, dist, route uint8, stats)``."""
    torch = _torch()
    _check_dev(X, offsets, perm, probe_parts, exact_rows)
    n, d = X.shape
    parts = offsets.numel() - 1
    probes = probe_parts.shape[1]
    lib = load()
    ws = _ws(workspace, lib.rsc_knn_probed_workspace_bytes(n, d, k, parts, probes), X.device)
    idx, dist = _out(n, k, X.device, out)
    route = torch.empty(n, dtype=torch.uint8, device=X.device)
    st = RoutedStats()
    check(lib.rsc_knn_probed(_ptr(X), n, d, k, _ptr(offsets), _ptr(perm), parts, _ptr(probe_parts), probes,
                             _ptr(exact_rows), _ptr(idx), _ptr(dist), _ptr(route), ctypes.byref(st), _ptr(ws),
                             ws.numel(), _stream()))
    return idx, dist, route, _stats_dict(st)


def knn_routed(router: Router, X, k: int, offsets, perm, probes: int = 32, mass_threshold: float = 0.9, out=None,
               workspace=None):
    """The routed form (``rsc_knn_routed``): ``(idx, dist, route, stats)``."""
    torch = _torch()
    _check_dev(X, offsets, perm)
    n, d = X.shape
    parts = offsets.numel() - 1
    lib = load()
    ws = _ws(workspace, lib.rsc_knn_routed_workspace_bytes(router.handle, n, d, k, parts, probes), X.device)
    idx, dist = _out(n, k, X.device, out)
    route = torch.empty(n, dtype=torch.uint8, device=X.device)
    st = RoutedStats()
    check(lib.rsc_knn_routed(router.handle, _ptr(X), n, d, k, _ptr(offsets), _ptr(perm), parts, probes,
                             mass_threshold, _ptr(idx), _ptr(dist), _ptr(route), ctypes.byref(st), _ptr(ws),
                             ws.numel(), _stream()))
    return idx, dist, route, _stats_dict(st)
