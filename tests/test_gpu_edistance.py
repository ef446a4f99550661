"""Energy distance between groups of cells: parity of the HIP path (through
the C ABI) with the float64 oracle.

Tolerance (derived from the arithmetic of the kernels): a distance is
computed as sqrt((|x|^2 + |y|^2) - 2 x.y) in float64 with the dot product on
the float64 matrix cores, so its square is off by at most
e = 2 (d + 4) u (|x|^2 + |y|^2), u = 2^-53, and the distance by at most
min(sqrt(e), e / dist), plus 4 units of roundoff from the square root.  A pair's sum
adds float64 tile partials (at most 64 roundings per value, below 1e-12
relative here) and rounds each tile to 64-bit fixed point (half a unit of
2^-e_p per tile, e_p from the bound count * 2 max|x|).
"""

import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rsc():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_02402_amd as rsc

    global _RSC
    rsc.load()
    _RSC = rsc
    return rsc


def dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


_RSC = None


def groups(labels, G):
    """The oracle's group layout of ``labels`` (host offsets, cells), after
    checking that the library's GPU counting sort gives the same layout."""
    from oracle import edistance as oed

    off, cells = oed.groups_from_labels(np.asarray(labels), G=G)
    if _RSC is not None:
        off_g, cells_g = _RSC.edistance_groups(dev(np.asarray(labels, dtype=np.int32)), G)
        assert np.array_equal(off_g, off) and np.array_equal(cells_g.cpu().numpy(), cells)
    return off, cells


def sum_bounds(X, offsets, cells, pairs):
    """Per-pair bound on |GPU sum - exact sum| (float64, numpy)."""
    Xd = X.astype(np.float64)
    d = X.shape[1]
    nrm = (Xd * Xd).sum(1)
    maxn = np.sqrt(nrm[cells].max()) if cells.size else 0.0
    out = np.zeros(len(pairs))
    for p, (a, b) in enumerate(pairs):
        A = cells[offsets[a]:offsets[a + 1]]
        B = cells[offsets[b]:offsets[b + 1]]
        if A.size == 0 or B.size == 0:
            continue
        tot = 0.0
        s_abs = 0.0
        for i0 in range(0, A.size, 512):
            Ai = A[i0:i0 + 512]
            diff = Xd[Ai][:, None, :] - Xd[B][None, :, :]
            D = np.sqrt((diff * diff).sum(-1))
            e = 2 * (d + 4) * U * (nrm[Ai][:, None] + nrm[B][None, :])
            err = np.where(D > 0, np.minimum(np.sqrt(e), e / np.where(D > 0, D, 1.0)), np.sqrt(e)) + 4 * U * D
            if a == b:
                mask = (np.arange(i0, i0 + Ai.size)[:, None] < np.arange(B.size)[None, :])
                err, D = err * mask, D * mask
            tot += err.sum()
            s_abs += D.sum()
        na, nb = A.size, B.size
        cnt = na * (na - 1) / 2 if a == b else na * nb
        tiles = ((na + 63) // 64) * ((nb + 63) // 64)
        quant = 0.5 * tiles * cnt * 2 * maxn * 2.0 ** -60
        out[p] = tot + 1e-12 * s_abs + quant
    return out


def check_sums(rsc, X, offsets, cells, pairs, label):
    from oracle import edistance as oed

    log(f"[edist] {label}: n={X.shape[0]} d={X.shape[1]} G={offsets.size - 1} pairs={len(pairs)}")
    g = rsc.edistance_sums(dev(X), offsets, dev(cells), pairs).cpu().numpy()
    o = oed.sums(X, offsets, cells, pairs)
    bnd = sum_bounds(X, offsets, cells, pairs)
    err = np.abs(g - o)
    worst = np.max(err / np.maximum(bnd, 1e-300)) if len(pairs) else 0.0
    rel = np.max(err / np.maximum(np.abs(o), 1e-300)) if len(pairs) else 0.0
    log(f"  max |gpu - oracle| / bound = {worst:.3e}, max relative error {rel:.2e}")
    assert (err <= bnd).all(), f"pairs over the bound: {np.flatnonzero(err > bnd)[:10]}"
    return g, o, bnd


def test_sums_ragged_groups(rsc):
    from oracle import edistance as oed

    sizes = [0, 1, 2, 3, 63, 64, 65, 127, 128, 129, 200, 7, 1, 0, 500]
    rng = np.random.default_rng(1)
    labels = rng.permutation(np.repeat(np.arange(len(sizes)), sizes))
    X = (rng.standard_normal((labels.size, 50)) + 3.0).astype(np.float32)
    off, cells = groups(labels, len(sizes))
    check_sums(rsc, X, off, cells, oed.all_pairs(len(sizes)), "ragged groups, all pairs")


def test_sums_explicit_pairs_any_order(rsc):
    sizes = [70, 150, 3, 64]
    rng = np.random.default_rng(2)
    labels = rng.permutation(np.repeat(np.arange(4), sizes))
    X = rng.standard_normal((labels.size, 20)).astype(np.float32)
    off, cells = groups(labels, 4)
    pairs = np.array([[3, 1], [1, 3], [2, 2], [0, 0], [1, 0], [3, 3], [2, 1], [2, 1]], dtype=np.int32)
    g, o, _ = check_sums(rsc, X, off, cells, pairs, "explicit pairs, both orders, repeats")
    assert g[6] == g[7]


@pytest.mark.parametrize("d", [1, 3, 64, 65, 130, 300])
def test_sums_general_d(rsc, d):
    from oracle import edistance as oed

    sizes = [90, 65, 1, 140]
    rng = np.random.default_rng(d)
    labels = rng.permutation(np.repeat(np.arange(4), sizes))
    X = (rng.standard_normal((labels.size, d)) * 2.0).astype(np.float32)
    off, cells = groups(labels, 4)
    check_sums(rsc, X, off, cells, oed.all_pairs(4), f"d={d}")


def test_sums_exact_duplicates(rsc):
    from oracle import edistance as oed

    sizes = [100, 80, 40]
    rng = np.random.default_rng(3)
    labels = np.repeat(np.arange(3), sizes)
    X = (rng.standard_normal((220, 50)) + 10.0).astype(np.float32)
    X[10:30] = X[5]      # duplicates inside group 0
    X[100:110] = X[5]    # and across groups 0 and 1
    X[180:220] = X[181]  # group 2: all cells identical
    off, cells = groups(labels, 3)
    g, o, bnd = check_sums(rsc, X, off, cells, oed.all_pairs(3), "exact duplicates")
    assert o[5] == 0.0  # (2, 2): every distance 0


def pairwise_check(rsc, X, labels, G, label):
    from oracle import edistance as oed

    off, cells = groups(labels, G)
    log(f"[edist] pairwise {label}: n={X.shape[0]} G={G}")
    E, D = rsc.edistance_pairwise(dev(X), off, dev(cells), want_means=True)
    E, D = E.cpu().numpy(), D.cpu().numpy()
    Eo, Do = oed.pairwise(X, off, cells)
    pairs = oed.all_pairs(G)
    sizes = np.diff(off)
    cnt = oed.pair_counts(sizes, pairs)
    bD = np.zeros((G, G))
    with np.errstate(invalid="ignore", divide="ignore"):
        m = np.where(cnt > 0, sum_bounds(X, off, cells, pairs) / cnt, 0.0)
    bD[pairs[:, 0], pairs[:, 1]] = m
    bD[pairs[:, 1], pairs[:, 0]] = m
    assert np.array_equal(np.isnan(D), np.isnan(Do)) and np.array_equal(np.isnan(E), np.isnan(Eo))
    ok = ~np.isnan(Do)
    assert (np.abs(D - Do)[ok] <= bD[ok]).all()
    dd = np.diag(bD)
    bE = 2 * bD + dd[:, None] + dd[None, :] + 4 * U * np.abs(np.nan_to_num(Eo))
    okE = ~np.isnan(Eo)
    errE = np.abs(E - Eo)[okE]
    log(f"  max |E - E_oracle| = {errE.max():.3e} (bound max {bE[okE].max():.3e})")
    assert (errE <= bE[okE]).all()
    assert np.array_equal(E, E.T, equal_nan=True) and (np.diag(E) == 0).all()
    # E is assembled from D exactly as stated: 2 D[a, b] - (D[a, a] + D[b, b])
    dg = np.diag(D)
    np.testing.assert_array_equal(E, 2.0 * D - (dg[:, None] + dg[None, :]))
    return off, cells, E


def test_pairwise_small_screen(rsc):
    X, labels = synth.perturbation_screen(n_groups=40, control=600, lo=5, hi=90, seed=4)
    pairwise_check(rsc, X, labels, 40, "40 groups")


def test_pairwise_singletons_and_empty_groups(rsc):
    sizes = [3, 1, 0, 1, 70]
    rng = np.random.default_rng(5)
    labels = rng.permutation(np.repeat(np.arange(5), sizes))
    X = rng.standard_normal((labels.size, 8)).astype(np.float32)
    pairwise_check(rsc, X, labels, 5, "singletons and an empty group")


def test_onesided(rsc):
    from oracle import edistance as oed

    X, labels = synth.perturbation_screen(n_groups=30, control=800, lo=10, hi=120, seed=6)
    off, cells = groups(labels, 30)
    for ref in (0, 17):
        E = rsc.edistance_onesided(dev(X), off, dev(cells), ref).cpu().numpy()
        Eo = oed.onesided(X, off, cells, ref)
        pairs = oed.onesided_pairs(30, ref)
        cnt = oed.pair_counts(np.diff(off), pairs)
        b = sum_bounds(X, off, cells, pairs) / np.maximum(cnt, 1)
        within = np.empty(30)
        within[ref] = b[ref]
        within[[g for g in range(30) if g != ref]] = b[30:]
        bE = 2 * b[:30] + within + within[ref] + 4 * U * np.abs(Eo)
        log(f"[edist] one-sided ref={ref}: max |E - E_oracle| = {np.abs(E - Eo).max():.3e}")
        assert (np.abs(E - Eo) <= bE).all() and E[ref] == 0.0


def test_deterministic(rsc):
    X, labels = synth.perturbation_screen(n_groups=60, control=3000, lo=20, hi=300, seed=7)
    off, cells = groups(labels, 60)
    Xt, ct = dev(X), dev(cells)
    a = rsc.edistance_pairwise(Xt, off, ct).cpu().numpy()
    b = rsc.edistance_pairwise(Xt, off, ct).cpu().numpy()
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))


def test_full_screen_sampled_parity(rsc):
    """The benchmarked screen (1000 groups, about 174k cells), the full matrix
    on the GPU in the benchmarked launch; the oracle on sampled pairs."""
    from oracle import edistance as oed

    X, labels = synth.perturbation_screen()
    G = synth.EDIST["n_groups"]
    off, cells = groups(labels, G)
    log(f"[edist] full screen: n={X.shape[0]} G={G}, GPU pairwise")
    E, D = rsc.edistance_pairwise(dev(X), off, dev(cells), want_means=True)
    E, D = E.cpu().numpy(), D.cpu().numpy()
    rng = np.random.default_rng(10)
    gs = rng.choice(np.arange(1, G), size=16, replace=False)
    pairs = np.array([[0, g] for g in gs[:6]] + [[g, g] for g in gs[6:10]] + [[gs[i], gs[i + 1]] for i in range(10, 15)],
                     dtype=np.int32)
    log(f"  oracle on {len(pairs)} sampled pairs")
    s = oed.sums(X, off, cells, pairs)
    cnt = oed.pair_counts(np.diff(off), pairs)
    bnd = sum_bounds(X, off, cells, pairs) / cnt
    got = D[pairs[:, 0], pairs[:, 1]]
    err = np.abs(got - s / cnt)
    log(f"  max |D - D_oracle| / bound = {np.max(err / bnd):.3e}")
    assert (err <= bnd).all()
    assert np.array_equal(E, E.T) and (np.diag(E) == 0).all() and np.isfinite(E).all()
    dg = np.diag(D)
    np.testing.assert_array_equal(E, 2.0 * D - (dg[:, None] + dg[None, :]))


@pytest.mark.parametrize("scale", [2.0 ** -70, 2.0 ** 60])
def test_sums_extreme_scales(rsc, scale):
    """Squared distances far below 1e-30 or above 1e30 take the correctly
    rounded square root; power-of-two scaling is exact in the inputs."""
    from oracle import edistance as oed

    sizes = [40, 70, 2]
    rng = np.random.default_rng(12)
    labels = rng.permutation(np.repeat(np.arange(3), sizes))
    X = (rng.standard_normal((labels.size, 16)) * scale).astype(np.float32)
    off, cells = groups(labels, 3)
    check_sums(rsc, X, off, cells, oed.all_pairs(3), f"scale 2^{int(np.log2(scale))}")


def test_group_layout_and_bad_labels(rsc):
    from oracle import edistance as oed

    rng = np.random.default_rng(13)
    labels = rng.integers(0, 37, size=5000).astype(np.int32)
    labels[labels == 5] = 6  # an empty group
    off_g, cells_g = rsc.edistance_groups(dev(labels), 37)
    off_o, cells_o = oed.groups_from_labels(labels, G=37)
    assert np.array_equal(off_g, off_o) and np.array_equal(cells_g.cpu().numpy(), cells_o)
    bad = labels.copy()
    bad[100] = 37
    with pytest.raises(rsc.RscError):
        rsc.edistance_groups(dev(bad), 37)
    bad[100] = -1
    with pytest.raises(rsc.RscError):
        rsc.edistance_groups(dev(bad), 37)
