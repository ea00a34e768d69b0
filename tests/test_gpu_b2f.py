"""GPU parity of the band-to-full back-transformation C = P^* Y (Sec. 2.1,
Eq. 2stage_bkwd2) through the C ABI, against the oracle's one-reflector-at-a-
time application on identical inputs.

Tolerance: relative Frobenius error <= 1e-12 (FP64).  Both sides apply the
same unitary product; the GPU merges 64 reflectors into one compact-WY
factor and sums in a different order (measured ~1e-15).

Inputs: seeded synthetic unitary reflectors with the shape of full-to-band
output (column j holds v_j in rows [j+nbw, n), v_j[0] = 1, tau unitary), and
at n <= 1024 the oracle's own reduction of a dense Hermitian matrix; the
entries the header says are never read (above each reflector's start, rows
n .. ldv-1) are filled with NaN so that reading one would show.
"""
import time

import numpy as np
import pytest

from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

TOL = 1e-12


def _relerr(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _dev_v(V, nbw, ldv, poison=True):
    """(n, J) reflectors -> device buffer (J, ldv) whose transpose view is
    column-major; unread entries NaN."""
    import torch
    n, J = V.shape
    host = np.full((max(J, 1), ldv), np.nan if poison else 0.0, V.dtype)
    for j in range(J):
        host[j, j + nbw: n] = V[j + nbw:, j]
    buf = torch.from_numpy(host).to("cuda")
    return buf, buf.T[:n, :J]


def gpu_b2f(Y, V, tau, nbw, ldv=None, ldz=None, poison=True):
    import torch
    import paper_2002_10991_amd as T
    n, nev = Y.shape
    ldv = ldv or max(n, 1)
    ldz = ldz or max(n, 1)
    print(f"[gpu] band_to_full n={n} nbw={nbw} nev={nev} ldv={ldv} ldz={ldz} "
          f"{'z' if np.iscomplexobj(Y) else 'd'}", flush=True)
    vb, vv = _dev_v(V, nbw, ldv, poison)
    host = np.full((max(nev, 1), ldz), 777.0, Y.dtype)
    host[:nev, :n] = Y.T
    zb = torch.from_numpy(host).to("cuda")
    td = torch.from_numpy(np.ascontiguousarray(tau)).to("cuda")
    T.band_to_full(zb.T[:n, :nev], vv, td, nbw)
    torch.cuda.synchronize()
    out = zb.cpu().numpy()
    assert np.all(out[:, n:] == 777.0)        # rows n .. ldz-1 untouched
    return out[:nev, :n].T


SHAPES = [(40, 4, 7), (100, 16, 33), (130, 64, 20), (300, 32, 65), (257, 7, 100),
          (500, 64, 17), (70, 1, 5), (66, 64, 3), (200, 128, 40), (600, 64, 1)]


@pytest.mark.parametrize("dtype", ["d", "z"])
@pytest.mark.parametrize("n,nbw,nev", SHAPES)
def test_b2f_parity_shapes(oracle_mod, dtype, n, nbw, nev):
    import synth
    V, tau = synth.full_unitary_reflectors(n, nbw, 900 + n + nbw, dtype)
    Y = synth.gaussian(n, nev, 901 + n, dtype)
    ref = oracle_mod.back_transform_full(Y, V, tau, nbw)
    got = gpu_b2f(Y, V, tau, nbw, ldv=n + 3, ldz=n + 5)
    assert _relerr(got, ref) <= TOL


@pytest.mark.parametrize("dtype", ["d", "z"])
def test_b2f_v0_not_one(oracle_mod, dtype):
    """v_j scaled by alpha (v_j[0] = alpha != 1) and tau by 1/|alpha|^2: the
    same reflectors, and the kernel reads v_j[0]."""
    import synth
    n, nbw, nev = 300, 16, 40
    V, tau = synth.full_unitary_reflectors(n, nbw, 31, dtype)
    rng = np.random.default_rng(32)
    J = V.shape[1]
    mag = rng.uniform(0.5, 2.0, J) * rng.choice([-1.0, 1.0], J)
    alpha = mag * np.exp(1j * rng.uniform(0, 2 * np.pi, J)) if dtype == "z" else mag
    V2, t2 = V * alpha[None, :], tau / np.abs(alpha) ** 2
    Y = synth.gaussian(n, nev, 33, dtype)
    got = gpu_b2f(Y, V2, t2, nbw)
    assert _relerr(got, oracle_mod.back_transform_full(Y, V2, t2, nbw)) <= TOL
    assert _relerr(got, oracle_mod.back_transform_full(Y, V, tau, nbw)) <= TOL


@pytest.mark.parametrize("dtype", ["d", "z"])
def test_b2f_reduction_reflectors_end_to_end(oracle_mod, dtype):
    """The oracle's full-to-band reduction of a dense Hermitian A (n = 1024,
    nbw = 64), then stage 2 entirely on the GPU (chase, tridiagonal
    eigenpairs, tridiagonal-to-banded back-transformation) and the
    band-to-full step on the GPU: the columns are eigenvectors of A.
    Also the oracle's back-transformation of the same Y (parity)."""
    import torch
    import synth
    import paper_2002_10991_amd as T
    n, nbw, nev = 1024, 64, 200
    A = synth.hermitian_matrix(n, 4040, dtype)
    r = oracle_mod.full_to_band(A, nbw)
    B = r["B"]
    ab = np.zeros((nbw + 1, n), B.dtype)
    for d in range(nbw + 1):
        ab[d, : n - d] = np.diagonal(B, -d)
    dev = torch.device("cuda:0")
    d, e, hv, ht = T.band_to_tridiagonal(torch.from_numpy(np.ascontiguousarray(ab.T)).to(dev),
                                         nbw)
    if dtype == "z":
        er = e.real.clone()
        er[-1] = e[-1].abs()
    else:
        er = e
    w, Zr = T.tridiagonal_eigh(d, er.to(torch.float64).contiguous(), nev)
    Zc = Zr.to(torch.complex128) if dtype == "z" else Zr
    if dtype == "z":
        Zc[-1, :] *= (e[-1] / e[-1].abs())
    buf = torch.empty((nev, n), dtype=Zc.dtype, device=dev)
    buf.copy_(Zc.T)
    T.back_transform(buf.T, hv, ht, nbw)
    torch.cuda.synchronize()
    Y = buf.cpu().numpy().T.copy()
    C = gpu_b2f(Y, r["hh_v"], r["hh_tau"], nbw)
    ref = oracle_mod.back_transform_full(Y, r["hh_v"], r["hh_tau"], nbw)
    assert _relerr(C, ref) <= TOL
    w = w.cpu().numpy()
    nrm = np.linalg.norm(A)
    assert np.max(np.abs(w - np.linalg.eigvalsh(A)[:nev])) <= 1e-12 * nrm
    res = np.linalg.norm(A @ C - C * w) / nrm
    orth = np.linalg.norm(C.conj().T @ C - np.eye(nev))
    print(f"[gpu] eigen-residual {res:.2e}, orthogonality {orth:.2e}", flush=True)
    assert res <= 1e-12 * n and orth <= 1e-12 * n
    assert res <= 1e-13


def test_b2f_deterministic_and_noops(oracle_mod):
    import torch
    import synth
    import paper_2002_10991_amd as T
    n, nbw, nev = 257, 32, 50
    V, tau = synth.full_unitary_reflectors(n, nbw, 8, "z")
    Y = synth.gaussian(n, nev, 9, "z")
    a = gpu_b2f(Y, V, tau, nbw)
    b = gpu_b2f(Y, V, tau, nbw)
    assert np.array_equal(np.ascontiguousarray(a).view(np.uint8),
                          np.ascontiguousarray(b).view(np.uint8))
    # J = 0 and nev = 0 leave Z alone
    Z = torch.randn(4, 20, dtype=torch.float64, device="cuda")
    Z0 = Z.clone()
    assert T.trans_ev_band_to_full_d(20, 19, 4, None, 20, None, Z, 20, None, 0) == 0
    assert T.trans_ev_band_to_full_d(20, 3, 0, None, 20, None, None, 20, None, 0) == 0
    torch.cuda.synchronize()
    assert torch.equal(Z, Z0)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("dtype", ["d", "z"])
def test_b2f_full_size_sampled(oracle_mod, dtype):
    """The benchmarked shapes: real n = 8192, nbw = 64, nev = 4096 (256
    columns against the oracle) and complex n = 32768, nbw = 64, nev = 8192
    (64 columns against the oracle, the rest by norm preservation)."""
    import torch
    import synth
    import paper_2002_10991_amd as T
    n, nev, ncheck = (8192, 4096, 256) if dtype == "d" else (32768, 8192, 64)
    nbw = 64
    t0 = time.perf_counter()
    V, tau = synth.full_unitary_reflectors(n, nbw, 5005 if dtype == "d" else 5006, dtype)
    Y = synth.gaussian(n, nev, 5007, dtype)
    print(f"[gpu] inputs {V.shape} {V.dtype} + {Y.shape} in {time.perf_counter() - t0:.1f} s",
          flush=True)
    dev = torch.device("cuda:0")
    print(f"[gpu] band_to_full full size n={n} nev={nev} {dtype}", flush=True)
    vb = torch.from_numpy(np.ascontiguousarray(V.T)).to(dev)   # (J, n): column-major V
    td = torch.from_numpy(tau).to(dev)
    zb = torch.from_numpy(np.ascontiguousarray(Y.T)).to(dev)
    T.band_to_full(zb.T, vb.T, td, nbw)
    torch.cuda.synchronize()
    del vb
    out = zb.cpu().numpy().T
    edge = [0, 1, 15, 16, 31, 32, nev // 2, nev - 1]
    rest = np.setdiff1d(np.arange(nev), edge)
    cols = np.unique(np.concatenate([edge, np.random.default_rng(3).choice(rest, ncheck - len(edge),
                                                                            replace=False)]))
    t0 = time.perf_counter()
    ref = oracle_mod.back_transform_full(Y, V, tau, nbw, cols=cols)
    err = _relerr(out[:, cols], ref)
    print(f"[gpu] {len(cols)} columns vs oracle ({time.perf_counter() - t0:.1f} s): "
          f"rel err {err:.2e}", flush=True)
    assert err <= TOL
    ny, nz = np.linalg.norm(out, axis=0), np.linalg.norm(Y, axis=0)
    assert np.max(np.abs(ny - nz) / nz) <= 1e-12
