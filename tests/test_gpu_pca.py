"""Sparse PCA: parity of the HIP path (through the C ABI) with the float64
oracle.

Tolerances (derived): the Gram matrix is summed in float64 from exact
float32 products, so |S_gpu - S| <= n u sum |x_i x_j| with u = 2^-53 (a
different summation order), and the covariance inherits that over n - 1.
The eigensolver is float64 on both sides: eigenvalues agree within a few
units of roundoff of ||C||, and a loading within (roundoff of ||C||) / gap to
its nearest eigenvalue; the scores inherit the loadings' error times the
row norms.
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

    rsc.load()
    return rsc


def dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def csr(n, p, density, seed):
    return synth.sparse_expression(n=n, p=p, density=density, seed=seed)


def abs_gram(ip, ix, v, p):
    """sum over cells of |x_i x_j| (float64), for the Gram's error bound."""
    from oracle import pca as opca

    _, S = opca.gram(ip, ix, np.abs(v), p)
    return S


@pytest.mark.parametrize("n,p,density", [(700, 40, 0.2), (3000, 129, 0.08), (2500, 300, 0.05), (130, 63, 0.5)])
def test_covariance_parity(rsc, n, p, density):
    from oracle import pca as opca

    ip, ix, v = csr(n, p, density, seed=n + p)
    log(f"[pca] covariance n={n} p={p} nnz={ip[-1]}")
    mu, C = rsc.pca_covariance(dev(ip), dev(ix), dev(v), p)
    mu, C = mu.cpu().numpy(), C.cpu().numpy()
    mu_o, C_o = opca.covariance(ip, ix, v, p)
    A = abs_gram(ip, ix, v, p)
    bS = 4 * n * U * A
    bC = (bS + n * 4 * U * np.abs(np.outer(mu_o, mu_o)) * n) / (n - 1) + 4 * U * np.abs(C_o)
    np.testing.assert_allclose(mu, mu_o, rtol=4 * n * U, atol=1e-300)
    err = np.abs(C - C_o)
    log(f"  max |C - C_oracle| / bound = {np.max(err / bC):.3e}")
    assert (err <= bC).all()
    assert np.array_equal(C, C.T)


def check_pca(rsc, ip, ix, v, p, k, label):
    from oracle import pca as opca

    n = len(ip) - 1
    log(f"[pca] {label}: n={n} p={p} k={k} nnz={ip[-1]}")
    mu, ev, V, Z = rsc.pca(dev(ip), dev(ix), dev(v), p, k)
    mu, ev, V, Z = mu.cpu().numpy(), ev.cpu().numpy(), V.cpu().numpy(), Z.cpu().numpy()
    mu_o, C_o, ev_o, V_o, Z_o = opca.pca(ip, ix, v, p, k)
    cn = np.abs(np.linalg.eigvalsh(C_o)).max()
    tol_ev = 64 * p * U * cn + 4 * n * U * np.abs(C_o).max()
    log(f"  max |evals - oracle| = {np.abs(ev - ev_o).max():.3e} (tol {tol_ev:.3e})")
    assert (np.abs(ev - ev_o) <= tol_ev).all()
    w_all = np.sort(np.linalg.eigvalsh(C_o))[::-1]
    # |dZ[c, t]| <= (||x_c||_1 + ||mu||_1) max_g |dV[g, t]| + the float32 rounding of Z
    l1 = np.array([np.abs(v[ip[c]:ip[c + 1]]).astype(np.float64).sum() for c in range(n)])
    scale = l1.max() + np.abs(mu_o).sum()
    for t in range(k):
        gap = min(abs(w_all[t] - w_all[t - 1]) if t > 0 else np.inf, abs(w_all[t] - w_all[t + 1]))
        tol_v = 10 * tol_ev / max(gap, 1e-300)
        err_v = np.abs(V[:, t] - V_o[:, t]).max()
        assert err_v <= tol_v, f"component {t}: loading error {err_v:.3e} > {tol_v:.3e} (gap {gap:.3e})"
        zt = np.abs(Z[:, t] - Z_o[:, t])
        zb = scale * err_v + 2.0 ** -24 * np.abs(Z_o[:, t]) + 64 * U * scale
        assert (zt <= zb).all(), f"scores of component {t}: {zt.max():.3e}"
    log(f"  evals {ev[:4]} ...; max loading error {np.abs(V - V_o).max():.3e}")
    return ev, ev_o


def test_pca_small(rsc):
    ip, ix, v = csr(2000, 80, 0.15, seed=5)
    check_pca(rsc, ip, ix, v, 80, 10, "small")


def test_pca_ragged_tiles_and_empty_rows(rsc):
    ip, ix, v = csr(1500, 191, 0.05, seed=6)  # 191 + 1 columns: a ragged last tile
    ip = np.concatenate([ip, [ip[-1]], [ip[-1]]])  # two empty cells at the end
    check_pca(rsc, ip, ix, v, 191, 20, "ragged tiles, empty rows")


def test_pca_bad_gene_index(rsc):
    ip, ix, v = csr(300, 40, 0.2, seed=7)
    ix = ix.copy()
    ix[5] = 40
    with pytest.raises(rsc.RscError):
        rsc.pca_covariance(dev(ip), dev(ix), dev(v), 40)


def test_pca_deterministic(rsc):
    ip, ix, v = csr(5000, 200, 0.05, seed=8)
    a = rsc.pca(dev(ip), dev(ix), dev(v), 200, 16)
    b = rsc.pca(dev(ip), dev(ix), dev(v), 200, 16)
    for x, y in zip(a, b):
        assert np.array_equal(x.cpu().numpy(), y.cpu().numpy())


def test_pca_two_chunks(rsc):
    """300k cells x 2000 genes: more than one 2 GiB dense chunk (262,144
    cells at 2048 padded columns), the benchmarked gene count."""
    from oracle import pca as opca

    n, p, k = 300_000, 2000, 12
    ip, ix, v = csr(n, p, 0.05, seed=9)
    log(f"[pca] two chunks: n={n} p={p} nnz={ip[-1]}")
    mu, ev, V, Z = rsc.pca(dev(ip), dev(ix), dev(v), p, k)
    mu, ev, V, Z = mu.cpu().numpy(), ev.cpu().numpy(), V.cpu().numpy(), Z.cpu().numpy()
    log("  oracle (float64)")
    mu_o, C_o, ev_o, V_o, Z_o = opca.pca(ip, ix, v, p, k)
    np.testing.assert_allclose(mu, mu_o, rtol=4 * n * U)
    w_all = np.sort(np.linalg.eigvalsh(C_o))[::-1]
    tol_ev = 64 * p * U * np.abs(w_all).max() + 4 * n * U * np.abs(C_o).max()
    log(f"  max |evals - oracle| = {np.abs(ev - ev_o).max():.3e} (tol {tol_ev:.3e})")
    assert (np.abs(ev - ev_o) <= tol_ev).all()
    rows = synth.sample_rows(n, 2000, seed=3)
    l1 = np.array([np.abs(v[ip[c]:ip[c + 1]]).astype(np.float64).sum() for c in rows])
    scale = l1.max() + np.abs(mu_o).sum()
    for t in range(k):
        gap = min(abs(w_all[t] - w_all[t - 1]) if t > 0 else np.inf, abs(w_all[t] - w_all[t + 1]))
        err_v = np.abs(V[:, t] - V_o[:, t]).max()
        assert err_v <= 10 * tol_ev / gap, f"component {t}: {err_v:.3e} (gap {gap:.3e})"
        zb = scale * err_v + 2.0 ** -24 * np.abs(Z_o[rows, t]) + 64 * U * scale
        assert (np.abs(Z[rows, t] - Z_o[rows, t]) <= zb).all()
    log(f"  loadings within {np.abs(V - V_o).max():.3e}")
