"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

The paper benchmarks its neighbourhood-graph step on the PCA embeddings of
public 10x / CELLxGENE datasets (Performance and reproducibility; Methods,
Benchmarking).  Those datasets are not available here, so every workload is
a seeded Gaussian mixture with the shape of such an embedding: ``d`` PCA
components whose variances fall off as ``1/i`` (a PCA spectrum), cells
grouped around cluster centres.

This module only draws random numbers.  It holds none of the arithmetic of
the method (no distances, no selection, no smoothing), so that both the HIP
path and the CPU oracle can take their inputs from it without sharing code.

Recipe (fixed here so that every consumer draws the same data):

* ``numpy.random.Generator(PCG64(seed))``;
* draw order: centres ``C x d`` from ``N(0, 25 I)`` (standard deviation 5),
  then the cluster label of every cell, then the within-cluster noise
  ``N(0, diag(lambda))`` with ``lambda_i = 1/i`` for ``i = 1..d``;
* cluster weights are either uniform or the finite rank-Zipf law
  ``p_m ~ m^-s`` for ``m = 1..C``;
* ``X = centres[label] + noise`` is formed in float64 and rounded once to
  float32 (round to nearest even).
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "MixtureSpec",
    "cluster_weights",
    "draw_centres",
    "mixture",
    "mixture_from_centres",
    "batched_sizes",
    "batched_samples",
    "WORKLOADS",
    "workload",
    "sample_rows",
    "lattice_1d",
    "random_knn_lists",
    "routed_draws",
    "init_rows",
    "random_probes",
    "random_mask",
    "random_labels",
    "EDIST",
    "perturbation_screen",
    "SPARSE_PCA",
    "sparse_expression",
]

_CHUNK = 1 << 18  # rows drawn per call; the PCG64 stream is identical to one big draw


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def cluster_weights(n_clusters: int, law: str = "uniform", zipf_s: float = 1.1) -> np.ndarray:
    """Mixture weights: ``uniform`` or rank-Zipf ``p_m ~ m**-zipf_s``."""
    if n_clusters < 1:
        raise ValueError("n_clusters must be >= 1")
    if law == "uniform":
        p = np.full(n_clusters, 1.0 / n_clusters)
    elif law == "zipf":
        p = np.arange(1, n_clusters + 1, dtype=np.float64) ** (-zipf_s)
        p /= p.sum()
    else:
        raise ValueError(f"unknown cluster law {law!r}")
    return p


def draw_centres(rng: np.random.Generator, n_clusters: int, d: int, centre_sd: float = 5.0) -> np.ndarray:
    return rng.standard_normal((n_clusters, d)) * centre_sd


def _noise_scale(d: int) -> np.ndarray:
    lam = 1.0 / np.arange(1, d + 1, dtype=np.float64)
    return np.sqrt(lam)


def mixture_from_centres(rng: np.random.Generator, centres: np.ndarray, n: int,
                         weights: np.ndarray, return_labels: bool = False, spread: float = 1.0):
    """Draw ``n`` cells around given ``centres`` (labels first, then noise
    of standard deviation ``spread`` sqrt(1/i) in dimension i)."""
    c, d = centres.shape
    labels = rng.choice(c, size=n, p=weights)
    scale = _noise_scale(d) * spread
    out = np.empty((n, d), dtype=np.float32)
    for s in range(0, n, _CHUNK):
        e = min(n, s + _CHUNK)
        noise = rng.standard_normal((e - s, d)) * scale
        out[s:e] = (centres[labels[s:e]] + noise).astype(np.float32)
    if return_labels:
        return out, labels
    return out


@dataclass(frozen=True)
class MixtureSpec:
    n: int
    d: int = 50
    n_clusters: int = 20
    law: str = "uniform"
    seed: int = 0


def mixture(n: int, d: int = 50, n_clusters: int = 20, law: str = "uniform", seed: int = 0,
            return_labels: bool = False):
    """One seeded Gaussian-mixture embedding, ``n x d`` float32, C-contiguous."""
    rng = _rng(seed)
    centres = draw_centres(rng, n_clusters, d)
    return mixture_from_centres(rng, centres, n, cluster_weights(n_clusters, law), return_labels)


def tight_mixture(n: int, d: int = 50, n_clusters: int = 20, spread: float = 0.2, seed: int = 0):
    """A mixture whose clusters are ``spread`` times as wide as ``mixture``'s:
    the neighbour gaps are then small against the row norms, as they are in
    the 2M-cell workload, at a size the CPU oracle handles."""
    rng = _rng(seed)
    centres = draw_centres(rng, n_clusters, d)
    return mixture_from_centres(rng, centres, n, cluster_weights(n_clusters, "uniform"), spread=spread)


def batched_sizes(n_samples: int = 64, lo: int = 2000, hi: int = 200000, seed: int = 4) -> np.ndarray:
    """Sample sizes log-uniform in ``[lo, hi]`` (rounded to integers)."""
    rng = _rng(seed)
    u = rng.uniform(math.log(lo), math.log(hi), size=n_samples)
    return np.rint(np.exp(u)).astype(np.int64)


def batched_samples(n_samples: int = 64, lo: int = 2000, hi: int = 200000, d: int = 50, seed: int = 4):
    """Concatenated independent samples plus their ``int64`` offsets (``S+1``).

    Sample ``s`` has its own seed ``1000 + s`` and ``C_s ~ U{10..40}`` uniform
    clusters, drawn from that sample's generator before its centres.
    """
    sizes = batched_sizes(n_samples, lo, hi, seed)
    offsets = np.zeros(n_samples + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    X = np.empty((int(offsets[-1]), d), dtype=np.float32)
    for s in range(n_samples):
        rng = _rng(1000 + s)
        c = int(rng.integers(10, 41))
        centres = draw_centres(rng, c, d)
        X[offsets[s]:offsets[s + 1]] = mixture_from_centres(rng, centres, int(sizes[s]), cluster_weights(c))
    return X, offsets


# The paper's benchmark scales, as synthetic stand-ins (d = 50 PCA components, k = 15).
WORKLOADS = {
    "plain_10k": MixtureSpec(n=10_000, n_clusters=20, law="uniform", seed=0),
    "plain_1m": MixtureSpec(n=1_000_000, n_clusters=100, law="zipf", seed=1),
    "precision_2m": MixtureSpec(n=2_000_000, n_clusters=100, law="zipf", seed=2),
}

# Learned-router form: 500 rank-Zipf clusters; the centres come from one seed,
# the base cells and the held-out training cells from two more.
ROUTED = {"n_base": 5_000_000, "n_train": 1_000_000, "n_clusters": 500, "law": "zipf", "centre_seed": 5,
          "base_seed": 50, "train_seed": 51, "parts": 4096}


def routed_draws(n_base: int | None = None, n_train: int | None = None, n_clusters: int | None = None,
                 d: int = 50):
    """``(base, train)`` of the routed form: two draws around the same centres."""
    c = ROUTED["n_clusters"] if n_clusters is None else n_clusters
    centres = draw_centres(_rng(ROUTED["centre_seed"]), c, d)
    w = cluster_weights(c, ROUTED["law"])
    base = mixture_from_centres(_rng(ROUTED["base_seed"]), centres, ROUTED["n_base"] if n_base is None else n_base, w)
    train = mixture_from_centres(_rng(ROUTED["train_seed"]), centres,
                                 ROUTED["n_train"] if n_train is None else n_train, w)
    return base, train


def init_rows(n: int, parts: int, seed: int) -> np.ndarray:
    """Distinct row ids (int32) whose rows seed the partition centroids."""
    return _rng(seed).choice(n, size=parts, replace=False).astype(np.int32)


def random_probes(n: int, parts: int, probes: int, seed: int, own: np.ndarray | None = None,
                  blank: float = 0.05, repeat: float = 0.05) -> np.ndarray:
    """Probe lists (int32 ``n x probes``) of random partitions: slot 0 is the
    row's own partition when ``own`` is given; a fraction of the other slots
    is left empty (-1) or repeats an earlier slot."""
    rng = _rng(seed)
    P = rng.integers(0, parts, size=(n, probes)).astype(np.int32)
    if own is not None:
        P[:, 0] = own
    if probes > 1:
        u = rng.random((n, probes))
        src = rng.integers(0, np.arange(1, probes + 1)[None, :].repeat(n, 0))
        rep = np.take_along_axis(P, src, axis=1)
        P = np.where((u < repeat) & (np.arange(probes) > 0), rep, P)
        P = np.where((u > 1 - blank) & (np.arange(probes) > 0), -1, P)
    return P


def random_mask(n: int, fraction: float, seed: int) -> np.ndarray:
    """A seeded uint8 mask with about ``fraction`` ones."""
    return (_rng(seed).random(n) < fraction).astype(np.uint8)


def random_labels(n: int, parts: int, seed: int) -> np.ndarray:
    return _rng(seed).integers(0, parts, size=n).astype(np.int32)


def workload(name: str, n: int | None = None) -> np.ndarray:
    """Embedding of a named workload; ``n`` overrides the size (same recipe)."""
    spec = WORKLOADS[name]
    return mixture(n if n is not None else spec.n, spec.d, spec.n_clusters, spec.law, spec.seed)


def sample_rows(n: int, count: int, seed: int) -> np.ndarray:
    """A sorted seeded sample of distinct row ids (for sampled parity checks)."""
    rng = _rng(seed)
    count = min(count, n)
    return np.sort(rng.choice(n, size=count, replace=False)).astype(np.int64)


def lattice_1d(n: int, d: int = 1, spacing: float = 1.0) -> np.ndarray:
    """Points ``i * spacing`` on the first axis (other axes zero): exact ties."""
    X = np.zeros((n, d), dtype=np.float32)
    X[:, 0] = np.arange(n, dtype=np.float32) * np.float32(spacing)
    return X


def random_knn_lists(n: int, k: int, seed: int, hub_fraction: float = 0.01):
    """Synthetic kNN-shaped lists (``idx`` int32, ``dist`` float32, self at slot 0).

    Neighbours are distinct, never the row itself; a small set of hub rows is
    over-represented so that some rows receive many reverse edges.  Distances
    are positive and non-decreasing along each row.  Used to exercise the
    graph stage at sizes where a brute-force kNN on the CPU would be too slow.
    """
    if k < 1 or n < k:
        raise ValueError("need 1 <= k <= n")
    rng = _rng(seed)
    idx = np.empty((n, k), dtype=np.int64)
    idx[:, 0] = np.arange(n)
    if k > 1:
        m = 3 * k + 8
        n_hub = max(1, int(n * hub_fraction))
        hubs = rng.choice(n, size=n_hub, replace=False)
        cand = rng.integers(0, n, size=(n, m))
        use_hub = rng.random((n, m)) < 0.3
        cand = np.where(use_hub, hubs[rng.integers(0, n_hub, size=(n, m))], cand)
        cand[cand == np.arange(n)[:, None]] = -1
        cand.sort(axis=1)
        bad = cand < 0
        bad[:, 1:] |= cand[:, 1:] == cand[:, :-1]
        keys = rng.random((n, m))
        keys[bad] = 2.0
        order = np.argsort(keys, axis=1, kind="stable")
        cand = np.take_along_axis(cand, order, axis=1)
        short = np.nonzero((~bad).sum(axis=1) < k - 1)[0]
        for i in short:  # rare: not enough distinct draws, fill deterministically
            row = [int(v) for v in cand[i] if v >= 0]
            row = list(dict.fromkeys(row))
            j = (i + 1) % n
            while len(row) < k - 1:
                if j != i and j not in row:
                    row.append(j)
                j = (j + 1) % n
            cand[i, : k - 1] = row[: k - 1]
        idx[:, 1:] = cand[:, : k - 1]
    gaps = rng.exponential(1.0, size=(n, k)).astype(np.float64)
    gaps[:, 0] = 0.0
    dist = np.cumsum(gaps, axis=1)
    dist[:, 1:] += 0.5
    return idx.astype(np.int32), dist.astype(np.float32)


# Energy-distance workload: a perturbation screen.  One large control group
# and many perturbation groups whose sizes are log-uniform; every cell is
# drawn from the same PCA-like noise N(0, diag(1/i)); perturbation g shifts
# its cells by an effect vector that is 0 for 70% of the groups (no
# phenotype) and N(0, s^2 diag(1/i)) with s log-uniform in [0.2, 2] for the
# rest.  Labels are shuffled so that a group's cells are scattered over X.
EDIST = {"n_groups": 1000, "control": 20_000, "lo": 50, "hi": 350, "seed": 9}


def perturbation_screen(n_groups: int | None = None, control: int | None = None, lo: int | None = None,
                        hi: int | None = None, d: int = 50, seed: int | None = None):
    """``(X float32 n x d, labels int32 n)``; group 0 is the control group."""
    G = EDIST["n_groups"] if n_groups is None else n_groups
    c0 = EDIST["control"] if control is None else control
    lo = EDIST["lo"] if lo is None else lo
    hi = EDIST["hi"] if hi is None else hi
    rng = _rng(EDIST["seed"] if seed is None else seed)
    sizes = np.exp(rng.uniform(np.log(lo), np.log(hi + 1), size=G - 1)).astype(np.int64)
    sizes = np.concatenate([[c0], sizes])
    lam = _noise_scale(d)
    effect = np.zeros((G, d))
    hit = rng.random(G) < 0.3
    hit[0] = False
    s = np.exp(rng.uniform(np.log(0.2), np.log(2.0), size=G))
    effect[hit] = rng.standard_normal((int(hit.sum()), d)) * lam * s[hit, None]
    labels = rng.permutation(np.repeat(np.arange(G, dtype=np.int32), sizes))
    X = np.empty((labels.size, d), dtype=np.float32)
    for r0 in range(0, labels.size, _CHUNK):
        lab = labels[r0:r0 + _CHUNK]
        X[r0:r0 + lab.size] = (effect[lab] + rng.standard_normal((lab.size, d)) * lam).astype(np.float32)
    return X, labels


# Sparse expression matrix for the PCA row: cells x genes in CSR, a stand-in
# for log-normalised counts over highly variable genes.  Gene g is detected in
# a cell with probability q_g = a / (1 + g / 500) (a popularity that falls off
# over the gene list, `a` set for the target density).  A detected entry
# holds log1p(s_c exp(b_g + u_c . v_g)) with a log-normal cell depth s_c, r = 8
# latent programs u_c ~ N(0, I), v_g ~ N(0, 0.35^2 I) and b_g ~ N(0.5, 0.5^2),
# so the matrix has a low-rank structure under noise.  Detected positions are
# drawn in row-major order as geometric gaps at max_g q_g, each kept with
# probability q_g / max q, so the gene indices of a row come out ascending.
SPARSE_PCA = {"n": 1_000_000, "p": 2000, "density": 0.05, "seed": 21}


def sparse_expression(n: int | None = None, p: int | None = None, density: float | None = None,
                      seed: int | None = None, programs: int = 8):
    """``(indptr int64 n+1, indices int32, data float32)``: rows in cell
    order, gene indices ascending within each row."""
    n = SPARSE_PCA["n"] if n is None else n
    p = SPARSE_PCA["p"] if p is None else p
    density = SPARSE_PCA["density"] if density is None else density
    rng = _rng(SPARSE_PCA["seed"] if seed is None else seed)
    w = 1.0 / (1.0 + np.arange(p) / 500.0)
    q = np.minimum(1.0, density * w / w.mean())
    qmax = float(q.max())
    b = rng.normal(0.5, 0.5, size=p)
    V = rng.normal(0.0, 0.35, size=(programs, p))
    Vt = np.ascontiguousarray(V.T)
    depth = np.exp(rng.normal(0.0, 0.3, size=n))
    U = rng.standard_normal((n, programs))
    counts = np.zeros(n, dtype=np.int64)
    ind_parts, val_parts = [], []
    rows_per = max(1, (1 << 26) // p)
    for r0 in range(0, n, rows_per):
        r1 = min(n, r0 + rows_per)
        size = (r1 - r0) * p
        pos = []
        last = -1
        while True:  # candidate positions: geometric gaps at qmax over the chunk's grid
            gaps = rng.geometric(qmax, size=int(qmax * size * 1.05) + 64)
            cand = last + np.cumsum(gaps)
            pos.append(cand[cand < size])
            if cand[-1] >= size:
                break
            last = int(cand[-1])
        pos = np.concatenate(pos)
        g = pos % p
        pos = pos[rng.random(pos.size) < q[g] / qmax]
        cr, g = pos // p, pos % p
        c = cr + r0
        val = np.log1p(depth[c] * np.exp(b[g] + (U[c] * Vt[g]).sum(1)))
        counts[r0:r1] = np.bincount(cr, minlength=r1 - r0)
        ind_parts.append(g.astype(np.int32))
        val_parts.append(val.astype(np.float32))
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=indptr[1:])
    return indptr, np.concatenate(ind_parts), np.concatenate(val_parts)


# Initial embedding for the UMAP layout: UMAP's random initialisation,
# coordinates uniform on [-10, 10].
def umap_init(n: int, dim: int = 2, seed: int = 31) -> np.ndarray:
    """``float32 [n, dim]`` uniform on [-10, 10]."""
    return _rng(seed).uniform(-10.0, 10.0, size=(n, dim)).astype(np.float32)
