"""GPU checks of whole workloads on the inputs their definitions name.

* The real n = 8192 workload (nbw = 64, nev = 4096): band N(0,1) plus the
  diagonal shift 4i/n (seed 1002), reflectors from bulge chasing that band
  (Sec. 2.2.1, Eq. 2stage_fwd2), Z_in = the eigenvectors of the lowest 4096
  eigenvalues of T (Eq. 2stage_solve), back-transformed (Eq. 2stage_bkwd1):
  all three steps on the GPU, in the launch configuration the benchmark
  times (prepare + apply).  Checks: the oracle's one-reflector-at-a-time
  back-transformation of 64 sampled columns from the same reflectors and
  Z_in (relative error <= 1e-12); the eigen-residual of every column against
  the band matrix (a banded product on the host); the whole Gram matrix.
* The tridiagonal step at the n = 32768 complex workload (nev = 8192): the
  T of the GPU chase of its band (seed 1003), eigenvalues of 512 indices
  against LAPACK's bisection, residuals of all 8192 vectors, orthogonality
  of every adjacent pair and of 512 sampled vectors against all others.

Bounds (FP64, eps = 2.2e-16): eigen-residuals and orthogonality are held to
1e-12 n (relative Frobenius), the end-to-end bound; a column of the
back-transformation is a unitary image, so its parity is 1e-12 relative.
Inverse iteration places a vector within eps ||T|| / gap of the true one,
and eigenvalues closer than 1e-6 ||T|| are orthonormalised together, so an
adjacent pair's inner product is below ~2 eps / 1e-6 = 4.4e-10 (asserted:
1e-9).
"""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _band_matmul(ab, Y):
    """B Y for the Hermitian band matrix in lower band layout ab[d, k] =
    B[k+d, k] (test helper, one diagonal at a time)."""
    nb1, n = ab.shape
    out = ab[0][:, None] * Y
    for d in range(1, nb1):
        a = ab[d, : n - d][:, None]
        out[d:] += a * Y[: n - d]
        out[: n - d] += np.conj(a) * Y[d:]
    return out


def _band_norm1(ab):
    """Largest column sum of |B| (an upper bound of the 2-norm)."""
    nb1, n = ab.shape
    s = np.abs(ab[0]).copy()
    for d in range(1, nb1):
        s[: n - d] += np.abs(ab[d, : n - d])
        s[d:] += np.abs(ab[d, : n - d])
    return float(s.max())


@pytest.mark.timeout(900)
def test_real_workload_as_defined(oracle_mod):
    import torch
    import synth
    import paper_2002_10991_amd as T
    n, nbw, nev = 8192, 64, 4096
    ab = synth.band_matrix(n, nbw, 1002, "d", diag_shift=True)
    dev = torch.device("cuda:0")
    print(f"[gpu] chase + tridiag + back-transform n={n} nbw={nbw} nev={nev}", flush=True)
    d, e, hv, ht = T.band_to_tridiagonal(torch.from_numpy(np.ascontiguousarray(ab.T)).to(dev),
                                         nbw)
    w, Zt = T.tridiagonal_eigh(d, e, nev)
    buf = torch.empty((nev, n), dtype=torch.float64, device=dev)
    buf.copy_(Zt.T)
    Zin = buf.cpu().numpy().T.copy(order="F")
    work = T.alloc_workspace(n, nbw, nev, False, dev)
    wb = work.numel()
    assert T.trbt_prepare_d(n, nbw, hv, ht, work, wb) == 0
    assert T.trbt_apply_d(n, nbw, nev, hv, ht, buf, n, work, wb) == 0
    torch.cuda.synchronize()
    assert T.trbt_work_check(work) == 0
    assert bool(torch.isfinite(d).all())
    Y = buf.cpu().numpy().T
    V, tau, w = hv.cpu().numpy(), ht.cpu().numpy(), w.cpu().numpy()

    # parity on sampled columns: the same reflectors and Z_in through the oracle
    cols = np.unique(np.concatenate([[0, 15, 16, nev // 2, nev - 1],
                                     np.random.default_rng(11).choice(nev, 59, replace=False)]))
    ref = oracle_mod.back_transform(Zin[:, cols], V, tau, nbw)
    err = np.linalg.norm(Y[:, cols] - ref) / np.linalg.norm(ref)
    print(f"[gpu] {len(cols)} columns vs oracle: rel err {err:.2e}", flush=True)
    assert err <= 1e-12

    # eigenpairs of the band matrix B: residual of every column, whole Gram
    nrm = _band_norm1(ab)
    R = _band_matmul(ab, Y) - Y * w
    res_col = np.linalg.norm(R, axis=0) / nrm
    res = np.linalg.norm(R) / np.linalg.norm(synth.band_matrix(n, nbw, 1002, "d", True))
    G = Y.T @ Y
    G[np.diag_indices(nev)] -= 1.0
    orth, orth_max = np.linalg.norm(G), np.abs(G).max()
    print(f"[gpu] residual max/col {res_col.max():.2e}, rel Frobenius {res:.2e}; "
          f"||Y^T Y - I||_F {orth:.2e} (max entry {orth_max:.2e})", flush=True)
    assert res <= 1e-12 * n and res_col.max() <= 1e-12 * np.sqrt(n)
    assert orth <= 1e-12 * n
    # the eigenvalues are the lowest half of B's (LAPACK on the band)
    import scipy.linalg as sl
    lam = sl.eig_banded(ab, lower=True, eigvals_only=True, select="i",
                        select_range=(0, nev - 1))
    assert np.max(np.abs(w - lam)) <= 1e-12 * nrm


def _tnorm(d, e):
    ae = np.abs(e)
    r = np.abs(d).copy()
    r[:-1] += ae
    r[1:] += ae
    return float(r.max())


@pytest.mark.timeout(900)
def test_tridiagonal_at_complex_workload_size():
    import scipy.linalg as sl
    import torch
    import synth
    import paper_2002_10991_amd as T
    n, nbw, nev = 32768, 64, 8192
    ab = synth.band_matrix(n, nbw, 1003, "z")
    dev = torch.device("cuda:0")
    print(f"[gpu] chase n={n} nbw={nbw} complex, then tridiag nev={nev}", flush=True)
    d, e, _, _ = T.band_to_tridiagonal(torch.from_numpy(np.ascontiguousarray(ab.T)).to(dev),
                                       nbw)
    er = e.real.clone()
    er[-1] = e[-1].abs()
    er = er.contiguous()
    w, Zt = T.tridiagonal_eigh(d, er, nev)
    torch.cuda.synchronize()
    d, er, w = d.cpu().numpy(), er.cpu().numpy(), w.cpu().numpy()
    assert np.all(np.isfinite(d))
    Z = Zt.cpu().numpy()
    tn = _tnorm(d, er)
    assert np.all(np.diff(w) >= 0)

    # eigenvalues: the first and last 64 and 384 seeded indices in between,
    # against LAPACK's bisection on the same T
    rng = np.random.default_rng(21)
    mid = np.sort(rng.choice(np.arange(64, nev - 64), 384, replace=False))
    ref_lo = sl.eigvalsh_tridiagonal(d, er, select="i", select_range=(0, 63))
    ref_hi = sl.eigvalsh_tridiagonal(d, er, select="i", select_range=(nev - 64, nev - 1))
    ref_mid = np.array([sl.eigvalsh_tridiagonal(d, er, select="i", select_range=(i, i))[0]
                        for i in mid])
    err_w = max(np.abs(w[:64] - ref_lo).max(), np.abs(w[nev - 64:] - ref_hi).max(),
                np.abs(w[mid] - ref_mid).max())
    # every vector's residual
    R = d[:, None] * Z - Z * w
    R[:-1] += er[:, None] * Z[1:]
    R[1:] += er[:, None] * Z[:-1]
    res = np.linalg.norm(R, axis=0).max()
    del R
    # orthogonality: every adjacent pair, and 512 sampled vectors against all
    adj = np.abs(np.einsum("ij,ij->j", Z[:, :-1], Z[:, 1:])).max()
    nrm = np.abs(np.linalg.norm(Z, axis=0) - 1).max()
    cols = np.sort(rng.choice(nev, 512, replace=False))
    Gs = Z[:, cols].T @ Z
    Gs[np.arange(512), cols] -= 1.0
    orth = np.linalg.norm(Gs)
    print(f"[gpu] eigenvalues {err_w:.2e} (||T|| {tn:.1f}), residual {res:.2e}, adjacent pairs "
          f"{adj:.2e}, norms {nrm:.2e}, sampled Gram {orth:.2e}", flush=True)
    assert err_w <= 1e-13 * tn
    assert res <= 1e-13 * tn * np.sqrt(n) / 10
    assert adj <= 1e-9 and nrm <= 1e-13
    assert orth <= 1e-12 * n
