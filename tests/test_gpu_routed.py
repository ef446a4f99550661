"""Parity of the routed form's HIP path (through the C ABI) with the CPU oracle:
k-means partitions, the probed search, and the router network's BF16
inference and training kernels."""

import struct
import sys

import numpy as np
import pytest

import synth
from tests.parity import compare_knn

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


def dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    import torch

    torch.cuda.synchronize()
    return t.cpu().numpy()


# ---------------------------------------------------------------------------
# Partitions
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,d,P", [(20000, 50, 64),    # brute-force assignment (d <= 64, P <= 2048)
                                   (4000, 80, 16),      # the exact k = 1 search (d > 64)
                                   (12000, 20, 2100)])  # the exact k = 1 search (P > 2048)
def test_kmeans_matches_oracle(rsc, oracle_mod, n, d, P):
    from oracle import partition

    X = synth.mixture(n, d=d, n_clusters=30, law="zipf", seed=21)
    iters = 6
    init = synth.init_rows(X.shape[0], P, seed=22)
    log(f"[kmeans] n={X.shape[0]} P={P} iters={iters}")
    C_g, a_g, off_g, perm_g, rel_g = rsc.partition_kmeans(dev(X), P, dev(init), iters)
    C_g, a_g, off_g, perm_g = host(C_g), host(a_g), host(off_g), host(perm_g)
    C_o, a_o, rel_o = partition.kmeans(X, init, iters)
    log(f"  relocated gpu={rel_g} oracle={rel_o}; labels differ on {(a_g != a_o).sum()} rows; "
        f"max centroid ulps {np.max(np.abs(C_g.view(np.int32) - C_o.view(np.int32)))}")
    assert rel_g == rel_o
    assert np.array_equal(a_g, a_o)
    # fixed-point sums are exact for all but the tiniest values: centroids
    # agree to the last bit, at worst one float32 ulp
    assert np.max(np.abs(C_g.view(np.int32).astype(np.int64) - C_o.view(np.int32))) <= 1
    off_o, perm_o = partition.inverted_lists(a_o, P)
    assert np.array_equal(off_g, off_o)
    for p in range(P):
        assert np.array_equal(np.sort(perm_g[off_g[p]:off_g[p + 1]]), perm_o[off_o[p]:off_o[p + 1]])


def test_kmeans_relocates_empty_partition(rsc):
    # the hand-derived case of the oracle's pin: rows 0, 0, 5, 5.5, 6 with
    # initial centroids rows 0, 1, 2 -> centroid 1 is empty and takes row 4
    X = np.array([[0.0], [0.0], [5.0], [5.5], [6.0]], dtype=np.float32)
    C, a, off, perm, rel = rsc.partition_kmeans(dev(X), 3, dev(np.array([0, 1, 2], dtype=np.int32)), 1)
    assert rel == 1
    assert host(C)[:, 0].tolist() == [0.0, 6.0, 5.25]
    assert host(a).tolist() == [0, 0, 2, 2, 1]
    assert host(off).tolist() == [0, 2, 3, 5]


def test_partition_lists_and_labels(rsc):
    from oracle import partition

    labels = synth.random_labels(30011, 97, seed=3)
    labels[labels == 40] = 41  # an empty partition
    off, perm = rsc.partition_lists(dev(labels), 97)
    off, perm = host(off), host(perm)
    off_o, perm_o = partition.inverted_lists(labels, 97)
    assert np.array_equal(off, off_o)
    for p in range(97):
        assert np.array_equal(np.sort(perm[off[p]:off[p + 1]]), perm_o[off_o[p]:off_o[p + 1]])
    idx = synth.random_labels(500 * 7, 30011, seed=4).reshape(500, 7)
    idx[3, 2] = -1
    idx[7, 0] = 30011
    lab = host(rsc.partition_labels(dev(idx), dev(labels)))
    exp = np.where((idx >= 0) & (idx < 30011), labels[np.clip(idx, 0, 30010)], -1)
    assert np.array_equal(lab, exp)


# ---------------------------------------------------------------------------
# Probed search
# ---------------------------------------------------------------------------

def probed_case(rsc, oracle_mod, X, P, probes, k, seed, mark_fraction=0.03):
    from oracle import partition

    n = X.shape[0]
    labels = synth.random_labels(n, P, seed) if P > 1 else np.zeros(n, np.int32)
    off, perm = partition.inverted_lists(labels, P)
    pr = synth.random_probes(n, P, probes, seed + 1, own=labels)
    mark = synth.random_mask(n, mark_fraction, seed + 2)
    log(f"[probed] n={n} P={P} probes={probes} k={k} marked={int(mark.sum())}")
    idx_g, dist_g, route, stats = rsc.knn_probed(dev(X), k, dev(off), dev(perm.astype(np.int32)), dev(pr),
                                                 exact_rows=dev(mark))
    idx_g, dist_g, route = host(idx_g), host(dist_g), host(route)
    log(f"  stats {stats}")
    assert np.array_equal(route == 1, mark == 1)
    # probed rows: exact within their partitions; rows sent to exact search
    # (marked, or not certified inside their partitions): exact over all rows
    exact = route != 0
    idx_o, _, dist_o = partition.routed_knn(X, k, off, perm, pr, exact_rows=exact)
    res = compare_knn(X, np.arange(n), idx_g, dist_g, idx_o, dist_o, oracle_mod, k)
    log(f"  {res['exact_rows']}/{n} rows identical, near-tie rows {res['near_tie_rows']}")
    assert stats["uncertified_rows"] == int((route == 2).sum()) <= max(5, n // 100)
    assert stats["low_mass_rows"] == int(mark.sum())
    assert stats["routed_rows"] + stats["low_mass_rows"] + stats["uncertified_rows"] == n
    return res, stats


def test_probed_matches_oracle(rsc, oracle_mod):
    X = synth.mixture(12000, n_clusters=12, seed=31)
    probed_case(rsc, oracle_mod, X, 97, 6, 15, seed=32)


def test_probed_ragged_wide_k(rsc, oracle_mod):
    # k > 16 (64-wide screen), partitions smaller than k-1 (candidate shortfall)
    X = synth.mixture(3001, d=33, n_clusters=5, seed=41)
    probed_case(rsc, oracle_mod, X, 611, 3, 20, seed=42, mark_fraction=0.1)


def test_probed_all_partitions_is_exact(rsc, oracle_mod):
    X = synth.mixture(5000, n_clusters=8, seed=51)
    P = 40
    labels = synth.random_labels(5000, P, 52)
    from oracle import partition

    off, perm = partition.inverted_lists(labels, P)
    pr = np.tile(np.arange(P, dtype=np.int32), (5000, 1))
    idx_g, dist_g, route, stats = rsc.knn_probed(dev(X), 15, dev(off), dev(perm), dev(pr))
    idx_o, _, dist_o = oracle_mod.knn(X, 15)
    compare_knn(X, np.arange(5000), host(idx_g), host(dist_g), idx_o, dist_o, oracle_mod, 15)


def test_probed_rejects_bad_layouts(rsc):
    from paper_2603_02402_amd import RscError

    X = synth.mixture(1000, n_clusters=3, seed=61)
    off = np.array([0, 500, 999], dtype=np.int64)  # sizes add up to 999, not 1000
    perm = np.arange(1000, dtype=np.int32)
    pr = np.zeros((1000, 2), dtype=np.int32)
    with pytest.raises(RscError, match="partition"):
        rsc.knn_probed(dev(X), 5, dev(off), dev(perm), dev(pr))
    off = np.array([0, 500, 1000], dtype=np.int64)
    pr[5, 1] = 2  # partition 2 does not exist
    with pytest.raises(RscError, match="probe"):
        rsc.knn_probed(dev(X), 5, dev(off), dev(perm), dev(pr))


# ---------------------------------------------------------------------------
# Router network
# ---------------------------------------------------------------------------

MAGIC = 0x52435352


def write_router_file(path, params, d, H, P, step=0, seed=0, moments=None):
    """The router file format: header, weights, then the two Adam moments."""
    with open(path, "wb") as f:
        f.write(struct.pack("<5i", MAGIC, 1, d, H, P))
        f.write(struct.pack("<qQ", step, seed))
        for part in [params] + (moments or [[np.zeros_like(p) for p in params]] * 2):
            for a in part:
                f.write(np.ascontiguousarray(a, dtype=np.float32).tobytes())


def read_router_file(path, d, H, P):
    raw = open(path, "rb").read()
    hdr = struct.unpack("<5i", raw[:20])
    step, seed = struct.unpack("<qQ", raw[20:36])
    assert hdr == (MAGIC, 1, d, H, P)
    arr = np.frombuffer(raw[36:], dtype=np.float32)
    shapes = [(H, d), (H,), (H, H), (H,), (P, H), (P,)]
    sizes = [int(np.prod(s)) for s in shapes]
    total = sum(sizes)
    assert arr.size == 3 * total
    out = []
    for part in range(3):
        o = part * total
        cur = []
        for s, z in zip(shapes, sizes):
            cur.append(arr[o:o + z].reshape(s).astype(np.float64))
            o += z
        out.append(cur)
    return out, step, seed


def f32_params(params):
    return [np.asarray(p, dtype=np.float32).astype(np.float64) for p in params]


def router_case(tmp_path, d, H, P, seed):
    from oracle import mlp

    rng = np.random.default_rng(seed)
    params = mlp.init_params(d, H, P, seed=seed)
    params = [p + (0.1 * rng.standard_normal(p.shape) if p.ndim == 1 else 0.0) for p in params]
    params = f32_params(params)
    path = tmp_path / f"router_{seed}.bin"
    write_router_file(path, params, d, H, P)
    return params, path


def make_router(rsc, path, d, H, P):
    r = rsc.Router(d, H, P, seed=0)
    r.load_file(path)
    return r


def rel_fro(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("d,H,P,n,m", [(50, 64, 128, 300, 5), (50, 256, 4096, 200, 15), (7, 128, 64, 64, 1)])
def test_router_gradients_match_oracle(rsc, tmp_path, d, H, P, n, m):
    from oracle import mlp

    params, path = router_case(tmp_path, d, H, P, seed=d + H + P)
    rng = np.random.default_rng(n)
    X = rng.standard_normal((n, d)).astype(np.float32) * 2
    labels = rng.integers(0, P, size=(n, m)).astype(np.int32)
    r = make_router(rsc, path, d, H, P)
    grad, loss = r.gradients(dev(X), dev(labels))
    grad, loss = host(grad), float(host(loss)[0])
    t = mlp.soft_targets(labels, P)
    emu = mlp.backward_bf16(params, X.astype(np.float64), t)
    exact = mlp.backward(params, X.astype(np.float64), t)
    names = ["W1", "b1", "W2", "b2", "W3", "b3"]
    o = 0
    log(f"[router grads] d={d} H={H} P={P} n={n} m={m}")
    for name, ge, gx in zip(names, emu, exact):
        g = grad[o:o + ge.size].reshape(ge.shape)
        o += ge.size
        re, rx = rel_fro(g, ge), rel_fro(g, gx)
        cos = float((g * gx).sum() / (np.linalg.norm(g) * np.linalg.norm(gx)))
        log(f"  {name}: rel err vs BF16-emulated {re:.2e}, vs float64 {rx:.2e}, cosine {cos:.6f}")
        # same roundings as the kernels: only float32 accumulation order and
        # the rare bfloat16 rounding flip it causes remain
        assert re < 1e-2, name
        # the bfloat16 roundings themselves (bound pinned in the oracle's tests)
        assert rx < 2**-4, name
        assert cos > 0.998, name
    assert o == grad.size
    (x, h1, h2), z = mlp.forward_bf16(params, X.astype(np.float64))
    ls = mlp.log_softmax(z)
    loss_o = float(-(t * ls).sum(axis=1).mean())
    log(f"  loss gpu {loss:.6f} oracle {loss_o:.6f}")
    assert abs(loss - loss_o) <= 1e-4 * abs(loss_o)
    r.close()


def test_router_logits_and_probes_match_oracle(rsc, tmp_path):
    from oracle import mlp

    d, H, P = 50, 256, 4096
    params, path = router_case(tmp_path, d, H, P, seed=5)
    X = synth.mixture(16384 + 77, n_clusters=10, seed=71)  # two inference chunks, ragged tail
    r = make_router(rsc, path, d, H, P)
    z_g = host(r.logits(dev(X)))
    rows = synth.sample_rows(X.shape[0], 600, seed=72)
    rows = np.union1d(rows, np.arange(X.shape[0] - 80, X.shape[0]))
    _, z_o = mlp.forward_bf16(params, X[rows].astype(np.float64))
    scale = np.abs(z_o).max(axis=1, keepdims=True)
    err = np.abs(z_g[rows] - z_o) / scale
    log(f"[router logits] max |dz| / max|z| = {err.max():.2e}")
    assert err.max() < 1e-3
    probes = 32
    parts_g, mass_g = r.probe(dev(X), probes)
    parts_g, mass_g = host(parts_g), host(mass_g)
    # the selection is taken on the kernels' own (bfloat16-rounded) logits:
    # the oracle's top set of those, except where two logits at the cut lie
    # closer than twice the logit tolerance asserted above
    zb = z_o
    order = np.lexsort((np.broadcast_to(np.arange(P), zb.shape), -zb), axis=1)[:, :probes]
    tol = 2 * 1e-3 * scale
    swaps = 0
    for i, r_ in enumerate(rows):
        g, o_ = parts_g[r_], order[i]
        assert len(set(g.tolist())) == probes
        if set(g.tolist()) != set(o_.tolist()):
            cut = zb[i, o_[-1]]
            for j in set(g.tolist()) ^ set(o_.tolist()):
                assert abs(zb[i, j] - cut) < tol[i, 0], (r_, j)
            swaps += 1
        # descending logits along the list
        zl = zb[i, g]
        assert (np.diff(zl) <= tol[i, 0]).all()
    log(f"  probe sets equal on {len(rows) - swaps}/{len(rows)} sampled rows (others: near-ties at the cut)")
    # softmax mass over the GPU's chosen set, from the oracle's logits
    ls = mlp.log_softmax(zb)
    mass_chk = np.exp(np.take_along_axis(ls, parts_g[rows].astype(np.int64), axis=1)).sum(axis=1)
    assert np.abs(mass_g[rows] - mass_chk).max() < 1e-3
    r.close()


def test_router_adam_first_step(rsc, tmp_path):
    from oracle import mlp

    d, H, P, n = 50, 64, 128, 256
    params, path = router_case(tmp_path, d, H, P, seed=9)
    rng = np.random.default_rng(10)
    X = rng.standard_normal((n, d)).astype(np.float32)
    labels = rng.integers(0, P, size=(n, 3)).astype(np.int32)
    r = make_router(rsc, path, d, H, P)
    lr = 1e-3
    r.train(dev(X), dev(labels), epochs=1, batch=n, lr=lr)  # one step over the whole set
    out = tmp_path / "after.bin"
    r.save(out)
    (w1, m1, m2), step, _ = read_router_file(out, d, H, P)
    assert step == 1
    g_o = mlp.backward(params, X.astype(np.float64), mlp.soft_targets(labels, P))
    for name, w0, w, g, a, b in zip(["W1", "b1", "W2", "b2", "W3", "b3"], params, w1, g_o, m1, m2):
        dw = w - w0
        # first Adam step: lr * g / (|g| + eps), so |dw| <= lr everywhere and
        # dw = -lr sign(g) wherever the gradient is clearly non-zero
        assert np.abs(dw).max() <= lr * (1 + 1e-3) + 1e-6 * np.abs(w0).max(), name
        big = np.abs(g) > 0.1 * np.abs(g).max()
        assert np.allclose(dw[big], -lr * np.sign(g[big]), rtol=1e-2, atol=1e-6 * max(1.0, np.abs(w0).max())), name
        # moments: (1 - beta1) g and (1 - beta2) g^2
        assert rel_fro(a, 0.1 * g) < 2**-4, name
        assert rel_fro(np.sqrt(b / 0.001), np.abs(g)) < 2**-4, name
    r.close()


def test_router_training_lowers_loss_and_roundtrips(rsc, tmp_path):
    from oracle import partition

    X = synth.mixture(8192, n_clusters=16, seed=81)
    C, labels, _ = partition.kmeans(X, synth.init_rows(8192, 64, 82), 3)
    lab = np.repeat(labels[:, None], 4, axis=1).astype(np.int32)
    r = rsc.Router(50, 128, 64, seed=7)
    losses = r.train(dev(X), dev(lab), epochs=12, batch=512, lr=3e-3)
    log(f"[router train] epoch losses {['%.4f' % v for v in losses]}")
    # each epoch's loss is the mean over its steps, so the first already
    # includes learning; it must start below the uniform guess log(64)
    assert losses[0] < np.log(64)
    assert losses[-1] < 0.5 * losses[0]
    assert all(b <= a * 1.02 for a, b in zip(losses, losses[1:]))
    p = tmp_path / "trained.bin"
    r.save(p)
    r2 = rsc.Router(50, 128, 64, seed=99)
    r2.load_file(p)
    z1, z2 = host(r.logits(dev(X[:500]))), host(r2.logits(dev(X[:500])))
    assert np.array_equal(z1, z2)
    assert r2.info()["steps"] == r.info()["steps"] == 12 * 16
    # top-1 partition of the trained router agrees with the partition labels on most cells
    parts, mass = r.probe(dev(X), 1)
    acc = float((host(parts)[:, 0] == labels).mean())
    log(f"  top-1 agreement with the partition labels {acc:.3f}")
    assert acc > 0.5  # chance is 1/64
    r.close()
    r2.close()


def test_router_rejects_bad_arguments(rsc, tmp_path):
    from paper_2603_02402_amd import RscError

    with pytest.raises(RscError):
        rsc.Router(50, 100, 64)  # hidden not a multiple of 64
    r = rsc.Router(50, 64, 64)
    with pytest.raises(RscError):
        r.load_file(tmp_path / "missing.bin")
    other = rsc.Router(50, 64, 128)
    other.save(tmp_path / "other.bin")
    with pytest.raises(RscError, match="shape"):
        r.load_file(tmp_path / "other.bin")
    r.close()
    other.close()


# ---------------------------------------------------------------------------
# End to end: partitions, labels, training, routed search; and the ablation
# ---------------------------------------------------------------------------

def test_routed_end_to_end_and_ablation(rsc, oracle_mod):
    """What the trained router gains over probing the nearest centroids,
    measured like against like at the same number of probes:
      * the network alone (no fallback) against the nearest centroids (no
        fallback): the network ranks the partitions no better than the
        centroid distances do (measured: 0.969 against 0.971), and is held
        within one point of them;
      * the routed form (router + exact search for its low-mass rows) must
        reach recall@15 >= 0.99, and is compared with the nearest centroids
        given the same exact-search budget: exact search for the same number
        of rows, chosen by the centroids' own signal of doubt, the smallest
        gap between the squared distances to the (probes+1)-th and the
        probes-th (or the first) nearest centroid.  The network's softmax
        mass beats the first gap (0.994 against 0.987) and only matches the
        second (0.9936 against 0.9938): held within 0.3 points of the best.
    So the trained network's gain over the method without it is its
    confidence signal, not its ranking, and a plain geometric signal does as
    well; the benchmark reports the same comparison at 5M cells."""
    from oracle import partition

    k, P, probes = 15, 128, 6
    base, train = synth.routed_draws(n_base=40000, n_train=12000, n_clusters=40)
    n = base.shape[0]
    Xb, Xt = dev(base), dev(train)
    C, assign, off, perm, _ = rsc.partition_kmeans(Xb, P, dev(synth.init_rows(n, P, 91)), 10)
    tidx, _ = rsc.knn(Xb, k, Q=Xt)                     # exact neighbours of the held-out cells
    labels = rsc.partition_labels(tidx, assign)        # their partitions: the soft targets
    router = rsc.Router(50, 256, P, seed=3)
    losses = router.train(Xt, labels, epochs=30, batch=512, lr=2e-3)
    log(f"[routed e2e] n={n} P={P} probes={probes}; loss {losses[0]:.3f} -> {losses[-1]:.3f}")

    rows = synth.sample_rows(n, 1500, seed=92)
    exact_idx, _, _ = oracle_mod.knn_rows(base, rows, k)

    def recall(idx):
        return partition.recall(host(idx)[rows][:, 1:], exact_idx[:, 1:])

    r_idx, r_dist, route, st = rsc.knn_routed(router, Xb, k, off, perm, probes=probes, mass_threshold=0.9)
    rec_routed = recall(r_idx)
    nr_idx, _, _, st0 = rsc.knn_routed(router, Xb, k, off, perm, probes=probes, mass_threshold=0.0)
    rec_router_only = recall(nr_idx)
    nc_parts, _ = rsc.knn(C, probes, Q=Xb)             # nearest centroids, in order
    nc_idx, _, _, st_nc = rsc.knn_probed(Xb, k, off, perm, nc_parts)
    rec_nc = recall(nc_idx)
    import torch

    nc_d = rsc.knn(C, probes + 1, Q=Xb)[1].double() ** 2
    low = int(st["low_mass_rows"])
    rec_gap = {}
    for name, (a, b) in {"next": (probes, probes - 1), "first": (probes, 0)}.items():
        mask = torch.zeros(n, dtype=torch.uint8, device="cuda")
        mask[torch.argsort(nc_d[:, a] - nc_d[:, b])[:low]] = 1
        g_idx, _, _, _ = rsc.knn_probed(Xb, k, off, perm, nc_parts[:, :probes].contiguous(), exact_rows=mask)
        rec_gap[name] = recall(g_idx)
    log(f"  recall@15: routed+fallback {rec_routed:.4f} (exact rows {low}, "
        f"uncertified {st['uncertified_rows']}, mean candidates {st['mean_probed_rows']:.0f}); "
        f"router only {rec_router_only:.4f}; nearest centroids {rec_nc:.4f} "
        f"(mean candidates {st_nc['mean_probed_rows']:.0f}); nearest centroids + exact search for the same "
        f"{low} rows by gap to the next centroid {rec_gap['next']:.4f}, to the first {rec_gap['first']:.4f}")
    assert rec_routed >= 0.99
    assert rec_routed > rec_gap["next"]
    assert rec_routed >= max(rec_gap.values()) - 0.003
    assert rec_router_only >= rec_nc - 0.01
    # the routed answer itself: exact within the probed partitions for routed
    # rows (the oracle on the router's own probe lists), exact over every cell
    # for rows sent to exact search
    pr, _ = router.probe(Xb, probes)
    sub = rows[:300]
    route_h = host(route)
    idx_o, _, dist_o = partition.routed_knn(base, k, host(off), host(perm), host(pr)[sub],
                                            exact_rows=route_h[sub] != 0, rows=sub)
    compare_knn(base, sub, host(r_idx)[sub], host(r_dist)[sub], idx_o, dist_o, oracle_mod, k)
    router.close()
