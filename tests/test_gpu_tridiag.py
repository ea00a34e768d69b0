"""GPU tridiagonal eigenpairs (bisection + inverse iteration, the step of
Eq. 2stage_solve) through the C ABI, against the oracle's implicit QL (pinned
by the Toeplitz closed form, Jacobi and LAPACK), closed forms and
invariants, and the whole stage 2 on the GPU (chase, tridiagonal solve,
back-transformation).

Bounds (FP64, eps = 2.2e-16, ||T|| the largest row sum):
  * eigenvalues: |w - w_QL| <= 1e-13 ||T|| (bisection stops at a few ulps of
    the eigenvalue; QL is accurate to O(eps ||T||));
  * eigenvectors: residual ||T z - w z|| <= 1e-13 ||T||, and the angle to the
    QL vector <= 1e-9 (inverse iteration's error is eps ||T|| / gap, gaps of
    these random matrices are >= 1e-5 ||T||);
  * orthogonality ||Z^T Z - I||_F <= 1e-12 n (the end-to-end bound).
"""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _gpu(d, e, nev, label=""):
    import torch
    import paper_2002_10991_amd as T
    n = len(d)
    print(f"[gpu] tridiag_eigh {label} n={n} nev={nev}", flush=True)
    dd = torch.from_numpy(np.ascontiguousarray(d, dtype=np.float64)).to("cuda")
    ee = torch.from_numpy(np.ascontiguousarray(e if n > 1 else np.zeros(1),
                                               dtype=np.float64)).to("cuda")
    w, Z = T.tridiagonal_eigh(dd, ee, nev)
    torch.cuda.synchronize()
    return w.cpu().numpy(), Z.cpu().numpy()


def _tnorm(d, e):
    ae = np.abs(e)
    r = np.abs(d).copy()
    r[:-1] += ae
    r[1:] += ae
    return float(r.max())


def _tmul(d, e, Z):
    Y = d[:, None] * Z
    Y[:-1] += e[:, None] * Z[1:]
    Y[1:] += e[:, None] * Z[:-1]
    return Y


def _check(d, e, w, Z, wref=None, Zref=None):
    n, nev = Z.shape
    tn = _tnorm(d, e)
    if wref is not None:
        assert np.max(np.abs(w - wref[:nev])) <= 1e-13 * tn
    assert np.all(np.diff(w) >= 0)
    R = _tmul(d, e, Z) - Z * w
    assert np.max(np.linalg.norm(R, axis=0)) <= 1e-13 * tn * max(1.0, np.sqrt(n) / 10)
    assert np.linalg.norm(Z.T @ Z - np.eye(nev)) <= 1e-12 * n
    if Zref is not None:
        cos = np.abs(np.sum(Z * Zref[:, :nev], axis=0))
        assert np.all(1 - cos <= 1e-9)


@pytest.mark.parametrize("n,nev", [(1, 1), (2, 2), (3, 1), (50, 50), (300, 150), (1000, 333),
                                   (513, 17)])
def test_tridiag_vs_oracle_ql(oracle_mod, n, nev):
    rng = np.random.default_rng(100 + n)
    d = rng.standard_normal(n)
    e = rng.standard_normal(max(n - 1, 0))
    wq, Xq = oracle_mod.tridiagonal_eigh(d, e)
    w, Z = _gpu(d, e, nev, "random")
    _check(d, e, w, Z, wq, Xq)


def test_tridiag_of_a_chased_band(oracle_mod):
    import synth
    n, nbw, nev = 600, 16, 300
    ab = synth.band_matrix(n, nbw, 61, "d", diag_shift=True)
    r = oracle_mod.band_to_tridiagonal(ab, nbw)
    wq, Xq = oracle_mod.tridiagonal_eigh(r["d"], r["e"])
    w, Z = _gpu(r["d"], r["e"], nev, "chased band")
    _check(r["d"], r["e"], w, Z, wq, Xq)


def test_tridiag_toeplitz_closed_form():
    n, a, b = 200, 2.0, -1.0
    d, e = np.full(n, a), np.full(n - 1, b)
    w, Z = _gpu(d, e, n, "toeplitz")
    k = np.arange(1, n + 1)
    lam = np.sort(a + 2 * b * np.cos(k * np.pi / (n + 1)))
    assert np.max(np.abs(w - lam)) <= 1e-13 * 4
    # eigenvector of lambda_k ~ sin(j k pi / (n+1)); lambda ascending <-> k ascending for b < 0
    j = np.arange(1, n + 1)
    for col in (0, 1, 57, n - 1):
        kk = col + 1
        v = np.sin(j * kk * np.pi / (n + 1))
        v /= np.linalg.norm(v)
        assert 1 - abs(v @ Z[:, col]) <= 1e-10


def test_tridiag_diagonal_and_degenerate_shapes():
    import torch
    import paper_2002_10991_amd as T
    d = np.array([3.0, -1.0, 2.0, 0.5, -4.0])
    w, Z = _gpu(d, np.zeros(4), 5, "diagonal")
    order = np.argsort(d)
    assert np.max(np.abs(w - d[order])) <= 8 * 2.2e-16 * 4.0   # bisection: a few ulps
    assert np.allclose(np.abs(Z), np.eye(5)[:, order], atol=1e-15)
    # nev = 0 and n = 0: nothing to do
    z = torch.zeros(0, dtype=torch.float64, device="cuda")
    w0, Z0 = T.tridiagonal_eigh(torch.ones(3, dtype=torch.float64, device="cuda"),
                                torch.ones(2, dtype=torch.float64, device="cuda"), 0)
    assert w0.numel() == 0 and Z0.shape == (3, 0)
    w0, Z0 = T.tridiagonal_eigh(z, z, 0)
    assert w0.numel() == 0


def test_tridiag_degenerate_clusters():
    """Two identical blocks: every eigenvalue is double.  The vectors of each
    cluster (inverse iterates from different starts) come out orthonormal
    after the cluster's modified Gram-Schmidt pass (one workgroup per
    cluster) and span the two blocks' eigenvectors."""
    rng = np.random.default_rng(12)
    m = 60
    d1, e1 = rng.standard_normal(m), rng.standard_normal(m - 1)
    d = np.concatenate([d1, d1])
    e = np.concatenate([e1, [0.0], e1])
    n = 2 * m
    w, Z = _gpu(d, e, n, "two equal blocks")
    w1 = np.linalg.eigvalsh(np.diag(d1) + np.diag(e1, 1) + np.diag(e1, -1))
    assert np.max(np.abs(w - np.repeat(w1, 2))) <= 1e-13 * _tnorm(d, e)
    R = _tmul(d, e, Z) - Z * w
    assert np.max(np.linalg.norm(R, axis=0)) <= 1e-13 * _tnorm(d, e)
    assert np.linalg.norm(Z.T @ Z - np.eye(n)) <= 1e-12 * n
    # each pair spans the pair of block eigenvectors
    _, V1 = np.linalg.eigh(np.diag(d1) + np.diag(e1, 1) + np.diag(e1, -1))
    for k in range(0, m, 7):
        S = Z[:, 2 * k: 2 * k + 2]
        B = np.zeros((n, 2))
        B[:m, 0] = V1[:, k]
        B[m:, 1] = V1[:, k]
        assert np.linalg.norm(B.T @ S @ S.T @ B - np.eye(2)) <= 1e-10


@pytest.mark.timeout(120)
def test_tridiag_large_clusters():
    """256 identical 2x2 blocks: two eigenvalues, each 256-fold, so the
    orthonormalisation pass gets two clusters of 256 vectors (one workgroup
    each).  The vectors come out orthonormal, in the right eigenspaces, and
    the pass finishes in seconds at this n (its cost is m^2 n per cluster on
    one workgroup)."""
    import time
    nb = 256
    d = np.tile([1.0, 3.0], nb)
    e = np.zeros(2 * nb - 1)
    e[0::2] = 0.5                      # couple within each block only
    n = 2 * nb
    t0 = time.perf_counter()
    w, Z = _gpu(d, e, n, "256 equal 2x2 blocks")
    dt = time.perf_counter() - t0
    lo, hi = 2.0 - np.sqrt(1.25), 2.0 + np.sqrt(1.25)   # eigenvalues of [[1, .5], [.5, 3]]
    tn = _tnorm(d, e)
    assert np.max(np.abs(w[:nb] - lo)) <= 1e-13 * tn and np.max(np.abs(w[nb:] - hi)) <= 1e-13 * tn
    R = _tmul(d, e, Z) - Z * w
    assert np.max(np.linalg.norm(R, axis=0)) <= 1e-13 * tn
    assert np.linalg.norm(Z.T @ Z - np.eye(n)) <= 1e-12 * n
    print(f"[gpu] two clusters of {nb}: {dt:.2f} s", flush=True)
    assert dt < 30.0


@pytest.mark.timeout(120)
def test_tridiag_large_clusters_long_vectors():
    """256 identical random 64x64 blocks (n = 16384): every eigenvalue is
    256-fold, and nev = 512 takes the two lowest, two clusters of 256
    vectors of length 16384 for the orthonormalisation pass."""
    import time
    rng = np.random.default_rng(31)
    m, copies = 64, 256
    d1, e1 = rng.standard_normal(m), rng.standard_normal(m - 1)
    d = np.tile(d1, copies)
    e = np.concatenate([np.concatenate([e1, [0.0]]) for _ in range(copies)])[:-1]
    n, nev = m * copies, 512
    t0 = time.perf_counter()
    w, Z = _gpu(d, e, nev, "256 equal 64x64 blocks")
    dt = time.perf_counter() - t0
    w1 = np.linalg.eigvalsh(np.diag(d1) + np.diag(e1, 1) + np.diag(e1, -1))
    tn = _tnorm(d, e)
    assert np.max(np.abs(w - np.repeat(w1[:2], copies))) <= 1e-13 * tn
    R = _tmul(d, e, Z) - Z * w
    # the residual bound of the other checks (it grows like sqrt(n))
    assert np.max(np.linalg.norm(R, axis=0)) <= 1e-13 * tn * max(1.0, np.sqrt(n) / 10)
    assert np.linalg.norm(Z.T @ Z - np.eye(nev)) <= 1e-12 * nev
    print(f"[gpu] two clusters of {copies} at n={n}: {dt:.2f} s", flush=True)
    assert dt < 60.0


def test_tridiag_c2_shape_against_lapack():
    """n = 8192, lowest 4096 (the real workload's tridiagonal size): the
    tridiagonal comes from the GPU chase of that workload's band."""
    import scipy.linalg as sl
    import synth
    import torch
    import paper_2002_10991_amd as T
    n, nbw, nev = 8192, 64, 4096
    ab = synth.band_matrix(n, nbw, 1002, "d", diag_shift=True)
    d, e, _, _ = T.band_to_tridiagonal(torch.from_numpy(np.ascontiguousarray(ab.T)).to("cuda"),
                                       nbw)
    torch.cuda.synchronize()
    d, e = d.cpu().numpy(), e.cpu().numpy()
    w, Z = _gpu(d, e, nev, "C2 shape")
    wl = sl.eigvalsh_tridiagonal(d, e, select="i", select_range=(0, nev - 1))
    tn = _tnorm(d, e)
    assert np.max(np.abs(w - wl)) <= 1e-13 * tn
    R = _tmul(d, e, Z) - Z * w
    assert np.max(np.linalg.norm(R, axis=0)) <= 1e-13 * tn * np.sqrt(n) / 10
    # the whole Gram matrix, and every adjacent pair on its own (inverse
    # iteration's error eps ||T|| / gap is largest there; pairs closer than
    # 1e-6 ||T|| are orthonormalised together, so |z_i . z_i+1| <~ 4.4e-10)
    Gm = Z.T @ Z - np.eye(nev)
    assert np.linalg.norm(Gm) <= 1e-12 * n
    assert np.abs(np.diagonal(Gm, 1)).max() <= 1e-9


@pytest.mark.parametrize("dtype", ["d", "z"])
def test_stage2_entirely_on_gpu(dtype):
    """Chase, tridiagonal eigenpairs and back-transformation all on the GPU:
    the result are eigenvectors of the band matrix B."""
    import torch
    import synth
    import paper_2002_10991_amd as T
    n, nbw, nev = 1024, 32, 256
    ab = synth.band_matrix(n, nbw, 808, dtype)
    d, e, hv, ht = T.band_to_tridiagonal(torch.from_numpy(np.ascontiguousarray(ab.T)).to("cuda"),
                                         nbw)
    if dtype == "z":   # every subdiagonal but the last is a real beta: keep its sign
        ea = e.real.clone()
        ea[-1] = e[-1].abs()
    else:
        ea = e
    w, Zr = T.tridiagonal_eigh(d, ea.to(torch.float64).contiguous(), nev)
    if dtype == "z":
        Zc = Zr.to(torch.complex128)
        Zc[-1, :] *= (e[-1] / e[-1].abs())   # T = D T_r D^H, D = diag(1, .., 1, phase)
    else:
        Zc = Zr
    buf = torch.empty((nev, n), dtype=Zc.dtype, device="cuda")
    buf.copy_(Zc.T)
    print(f"[gpu] back_transform stage-2 n={n} nbw={nbw} nev={nev} {dtype}", flush=True)
    T.back_transform(buf.T, hv, ht, nbw)
    torch.cuda.synchronize()
    Y = buf.cpu().numpy().T
    w = w.cpu().numpy()
    B = synth.dense_from_band(ab)
    res = np.linalg.norm(B @ Y - Y * w) / (np.linalg.norm(B) * np.sqrt(nev))
    orth = np.linalg.norm(Y.conj().T @ Y - np.eye(nev))
    assert res <= 1e-13 and orth <= 1e-12 * n
