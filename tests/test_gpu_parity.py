"""GPU parity: the HIP back-transformation (through the C ABI) against the CPU
oracle on identical seeded inputs.

Tolerance: relative Frobenius error <= 1e-12 in FP64 (the target accuracy
of the workload definition).  Both sides apply exactly the same unitary
transformation; they differ only in rounding order (the blocked GPU path
merges 16 reflectors into one compact-WY factor), and the measured
difference is ~1e-15.
"""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

TOL = 1e-12


def _torch():
    import torch
    return torch


def _dev_tensor(a: np.ndarray):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _dev_z(Z: np.ndarray, ldz: int):
    """Column-major device copy of Z (n x nev) with leading dimension ldz;
    returns (buffer (nev, ldz), view (n, nev))."""
    torch = _torch()
    n, nev = Z.shape
    host = np.zeros((nev, ldz), Z.dtype)
    host[:, :n] = Z.T
    buf = torch.from_numpy(host).to("cuda")
    return buf, buf.T[:n]


def gpu_back_transform(Z, V, tau, nbw, ldz=None, check_err=True):
    import paper_2002_10991_amd as T
    torch = _torch()
    n, nev = Z.shape
    ldz = ldz or max(n, 1)
    buf, Zd = _dev_z(Z, ldz)
    Vd, td = _dev_tensor(V), _dev_tensor(tau)
    work = T.alloc_workspace(n, nbw, nev, np.iscomplexobj(Z))
    print(f"[gpu] back_transform n={n} nbw={nbw} nev={nev} ldz={ldz} "
          f"dtype={'z' if np.iscomplexobj(Z) else 'd'}", flush=True)
    T.back_transform(Zd, Vd, td, nbw, work=work)
    torch.cuda.synchronize()
    if check_err and work is not None:
        assert T.trbt_work_check(work) == 0, "device wait timeout flag set"
    return buf.cpu().numpy(), work


def _inputs(n, nbw, nev, dtype, seed, oracle_mod):
    import synth
    lengths = oracle_mod.reflector_table(n, nbw)[3]
    V, tau = synth.unitary_reflectors(lengths, nbw, seed, dtype)
    Z = synth.gaussian(n, nev, seed + 1, dtype)
    return Z, V, tau


def _relerr(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


SHAPES = [
    # (n, nbw, nev): blocked path (nbw a multiple of 16 up to 128; above 64
    # with 4 waves per strip) and unblocked path
    (40, 16, 17), (100, 16, 33), (150, 32, 65), (200, 48, 16), (300, 64, 64),
    (301, 64, 63), (517, 64, 100), (130, 32, 1), (100, 128, 10),
    (400, 80, 50), (500, 96, 70), (700, 112, 33), (1000, 128, 100), (1301, 128, 17),
    (50, 2, 7), (61, 3, 20), (90, 8, 31), (129, 31, 64), (140, 33, 65), (300, 100, 20),
]


@pytest.mark.parametrize("dtype", ["d", "z"])
@pytest.mark.parametrize("n,nbw,nev", SHAPES)
def test_parity_shapes(oracle_mod, dtype, n, nbw, nev):
    Z, V, tau = _inputs(n, nbw, nev, dtype, 1000 + n + nbw, oracle_mod)
    ref = oracle_mod.back_transform(Z, V, tau, nbw)
    out, _ = gpu_back_transform(Z, V, tau, nbw)
    assert _relerr(out[:, :n].T, ref) <= TOL


@pytest.mark.parametrize("dtype", ["d", "z"])
def test_ldz_padding_untouched_and_nan_isolated(oracle_mod, dtype):
    n, nbw, nev, ldz = 150, 32, 40, 163
    Z, V, tau = _inputs(n, nbw, nev, dtype, 77, oracle_mod)
    Z = Z.copy()
    Z[5, 3] = np.nan
    import paper_2002_10991_amd as T
    torch = _torch()
    host = np.full((nev, ldz), 12345.0, Z.dtype)
    host[:, :n] = Z.T
    buf = torch.from_numpy(host).to("cuda")
    T.back_transform(buf.T[:n], _dev_tensor(V), _dev_tensor(tau), nbw)
    torch.cuda.synchronize()
    out = buf.cpu().numpy()
    assert np.all(out[:, n:] == 12345.0)
    assert np.all(np.isnan(out[3, :n]) | np.isfinite(out[3, :n]))
    good = [c for c in range(nev) if c != 3]
    ref = oracle_mod.back_transform(Z[:, good], V, tau, nbw)
    assert _relerr(out[good, :n].T, ref) <= TOL
    assert np.all(np.isfinite(out[good, :n]))


@pytest.mark.parametrize("dtype", ["d", "z"])
@pytest.mark.parametrize("n,nbw,nev", [(2000, 16, 50), (3000, 32, 100), (1500, 64, 300),
                                       (2500, 48, 17), (3000, 128, 40), (1024, 32, 1024)])
def test_parity_slot_groups(oracle_mod, dtype, n, nbw, nev):
    """Few column strips and many slots: several workgroups share each strip
    (slot groups, up to 8), handing tiles across workgroups through Z."""
    Z, V, tau = _inputs(n, nbw, nev, dtype, 6000 + n + nbw, oracle_mod)
    ref = oracle_mod.back_transform(Z, V, tau, nbw)
    out, _ = gpu_back_transform(Z, V, tau, nbw)
    assert _relerr(out[:, :n].T, ref) <= TOL
    again, _ = gpu_back_transform(Z, V, tau, nbw)
    assert np.array_equal(out.view(np.uint8), again.view(np.uint8))


@pytest.mark.parametrize("nbw", [32, 7])
def test_deterministic_bitwise(oracle_mod, nbw):
    Z, V, tau = _inputs(257, nbw, 50, "z", 5, oracle_mod)
    a, _ = gpu_back_transform(Z, V, tau, nbw)
    b, _ = gpu_back_transform(Z, V, tau, nbw)
    assert np.array_equal(a.view(np.uint8), b.view(np.uint8))


def test_degenerate_shapes_are_noops(oracle_mod):
    import paper_2002_10991_amd as T
    torch = _torch()
    for n, nbw, nev in [(2, 4, 2), (1, 1, 1), (10, 1, 5), (30, 8, 0)]:
        Z = torch.randn(max(nev, 1), max(n, 1), dtype=torch.float64, device="cuda")
        Z0 = Z.clone()
        K = T.trbt_num_reflectors(n, nbw)
        V = torch.zeros(max(K, 1), nbw, dtype=torch.float64, device="cuda")
        tau = torch.zeros(max(K, 1), dtype=torch.float64, device="cuda")
        rc = T.trans_ev_tridi_to_band_d(n, nbw, nev, V, tau, Z, max(n, 1), None, 0)
        torch.cuda.synchronize()
        assert rc == 0 and torch.equal(Z, Z0)


def test_workspace_too_small_rejected(oracle_mod):
    import paper_2002_10991_amd as T
    torch = _torch()
    n, nbw, nev = 100, 32, 10
    need = T.trbt_workspace_bytes(n, nbw, nev, False)
    assert need > 0
    Z = torch.zeros(nev, n, dtype=torch.float64, device="cuda")
    V = torch.zeros(T.trbt_num_reflectors(n, nbw), nbw, dtype=torch.float64, device="cuda")
    tau = torch.zeros(V.shape[0], dtype=torch.float64, device="cuda")
    work = T.alloc_workspace(n, nbw, nev, False)
    rc = T.trans_ev_tridi_to_band_d(n, nbw, nev, V, tau, Z, n, work, need - 8)
    assert rc == -101


@pytest.mark.parametrize("dtype", ["d", "z"])
def test_c1_pipeline_end_to_end(oracle_mod, dtype):
    """C1 shape (n=1024, nbw=32, all eigenvectors) with reflectors from the
    oracle's bulge chase and Z_in from its QL solve: GPU output matches the
    oracle back-transform and the result is an eigenbasis of B."""
    import synth
    n, nbw = 1024, 32
    ab = synth.band_matrix(n, nbw, 1001, dtype)
    p = oracle_mod.stage2_pipeline(ab, nbw, n)
    ref = oracle_mod.back_transform(p["Z_in"], p["hh_v"], p["hh_tau"], nbw)
    out, _ = gpu_back_transform(p["Z_in"], p["hh_v"], p["hh_tau"], nbw)
    Y = out.T
    assert _relerr(Y, ref) <= TOL
    B = synth.dense_from_band(ab)
    nrm = np.linalg.norm(B)
    assert np.linalg.norm(B @ Y - Y * p["w"]) / nrm <= 1e-12 * n
    assert np.linalg.norm(np.conj(Y.T) @ Y - np.eye(n)) <= 1e-12 * n


def _rescaled_nan_tail(V, tau, lengths, dtype, seed):
    """The same reflectors H = I - tau v v^H written with v' = alpha v
    (v'[0] = alpha != 1) and tau' = tau / |alpha|^2, and every stored entry
    at a position >= len filled with NaN.  The header promises v[0] is read
    and the tail is never read, so the product of reflectors is unchanged."""
    rng = np.random.default_rng(seed)
    K = len(tau)
    mag = rng.uniform(0.5, 2.0, K) * rng.choice([-1.0, 1.0], K)
    alpha = mag * np.exp(1j * rng.uniform(0, 2 * np.pi, K)) if dtype == "z" else mag
    V2 = V * alpha[:, None]
    t2 = tau / np.abs(alpha) ** 2
    Vz = V2.copy()                       # zero tail: the oracle's own layout
    tail = np.arange(V.shape[1])[None, :] >= np.asarray(lengths)[:, None]
    V2[tail] = np.nan
    return V2, t2, Vz


@pytest.mark.parametrize("dtype", ["d", "z"])
@pytest.mark.parametrize("n,nbw,nev", [(300, 64, 40), (200, 32, 33), (150, 16, 20),
                                       (150, 24, 20), (97, 7, 10), (100, 128, 9),
                                       (600, 96, 20), (300, 100, 9)])
def test_parity_v0_not_one_nan_tail(oracle_mod, dtype, n, nbw, nev):
    """v[0] != 1 and NaN beyond each reflector's length, on the blocked
    (nbw in {16, 32, 64, 96, 128}) and the streaming path (24, 7, 100)."""
    Z, V, tau = _inputs(n, nbw, nev, dtype, 3000 + n + nbw, oracle_mod)
    lengths = oracle_mod.reflector_table(n, nbw)[3]
    V2, t2, Vz = _rescaled_nan_tail(V, tau, lengths, dtype, 5 + n)
    assert np.all(np.abs(V2[:, 0]) != 1.0)
    out, _ = gpu_back_transform(Z, V2, t2, nbw)
    got = out[:, :n].T
    assert np.all(np.isfinite(got))
    assert _relerr(got, oracle_mod.back_transform(Z, Vz, t2, nbw)) <= TOL
    # the same operator as the unscaled reflectors
    assert _relerr(got, oracle_mod.back_transform(Z, V, tau, nbw)) <= TOL
