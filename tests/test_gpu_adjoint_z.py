"""GPU parity of the adjoint of the complex back-transformation (conjugate-
Wirtinger gradients of a real loss, PyTorch's convention), through the C ABI,
against the CPU oracle's complex adjoint and torch.autograd.gradcheck.

Tolerance: relative Frobenius error <= 1e-12 for grad Z_in, grad v and
grad tau, each compared as a whole array.  The GPU runs the same per-column
recurrences as the oracle (one lane per column, the same summation order
inside a column); only the column sums behind grad v and grad tau are taken
in a different order (64 columns of a wave, then waves in order, against
the oracle's per-thread blocks), which moves them by ~1e-15 relative.
"""
import numpy as np
import pytest

import oracle_cache
from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

TOL = 1e-12


def _relerr(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _inputs(n, nbw, nev, seed, general_tau=False):
    import synth
    lengths = synth.reflector_lengths(n, nbw)
    V, tau = synth.unitary_reflectors(lengths, nbw, seed, "z")
    if general_tau:
        rng = np.random.default_rng(seed + 7)
        tau = rng.uniform(0.3, 1.7, len(tau)) + 1j * rng.uniform(-0.8, 0.8, len(tau))
    Z = synth.gaussian(n, nev, seed + 1, "z")
    G = synth.gaussian(n, nev, seed + 2, "z")
    return Z, G, V, tau


def gpu_adjoint_z(Z, G, V, tau, nbw):
    import torch
    import paper_2002_10991_amd as T
    n, nev = Z.shape
    print(f"[gpu] adjoint_z n={n} nbw={nbw} nev={nev}", flush=True)
    zb = torch.from_numpy(np.ascontiguousarray(Z.T)).to("cuda")
    gb = torch.from_numpy(np.ascontiguousarray(G.T)).to("cuda")
    g, dv, dt = T.adjoint(zb.T, gb.T, torch.from_numpy(V).to("cuda"),
                          torch.from_numpy(tau).to("cuda"), nbw)
    torch.cuda.synchronize()
    return g.cpu().numpy(), dv.cpu().numpy(), dt.cpu().numpy()


# nbw in {16, 32, 48, 64}: the blocked (compact-WY, MFMA) form; the others:
# the stage-parallel streaming form
SHAPES = [(40, 16, 17), (100, 16, 33), (150, 32, 65), (300, 64, 64), (301, 64, 63),
          (200, 48, 40), (530, 64, 47), (61, 3, 20), (90, 8, 31), (129, 31, 64), (100, 128, 10),
          (70, 2, 5)]


@pytest.mark.parametrize("n,nbw,nev", SHAPES)
def test_complex_adjoint_vs_oracle(oracle_mod, n, nbw, nev):
    Z, G, V, tau = _inputs(n, nbw, nev, 500 + n + nbw)
    rZ, rv, rt = oracle_mod.adjoint(Z, G, V, tau, nbw)
    gZ, gv, gt = gpu_adjoint_z(Z, G, V, tau, nbw)
    assert _relerr(gZ, rZ) <= TOL
    assert _relerr(gv, rv) <= TOL
    assert _relerr(gt, rt) <= TOL


@pytest.mark.parametrize("n,nbw,nev", [(120, 16, 40), (97, 7, 10)])
def test_complex_adjoint_general_tau(oracle_mod, n, nbw, nev):
    Z, G, V, tau = _inputs(n, nbw, nev, 900 + n, general_tau=True)
    rZ, rv, rt = oracle_mod.adjoint(Z, G, V, tau, nbw)
    gZ, gv, gt = gpu_adjoint_z(Z, G, V, tau, nbw)
    assert _relerr(gZ, rZ) <= TOL and _relerr(gv, rv) <= TOL and _relerr(gt, rt) <= TOL


def test_complex_adjoint_deterministic():
    Z, G, V, tau = _inputs(200, 32, 70, 31)
    a = gpu_adjoint_z(Z, G, V, tau, 32)
    b = gpu_adjoint_z(Z, G, V, tau, 32)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_complex_adjoint_degenerate(oracle_mod):
    import torch
    import paper_2002_10991_amd as T
    # nev = 0: zero parameter gradients
    Z, G, V, tau = _inputs(50, 8, 3, 41)
    vd, td = torch.from_numpy(V).to("cuda"), torch.from_numpy(tau).to("cuda")
    z0 = torch.zeros((0, 50), dtype=torch.complex128, device="cuda")
    _, dv, dt = T.adjoint(z0.T, z0.clone().T, vd, td, 8)
    torch.cuda.synchronize()
    assert dv.shape == V.shape and not dv.abs().any() and not dt.abs().any()
    # nbw = 1: no reflectors, grad Z_in = G
    gb = torch.from_numpy(np.ascontiguousarray(G.T)).to("cuda")
    zb = torch.from_numpy(np.ascontiguousarray(Z.T)).to("cuda")
    e = torch.zeros((0, 1), dtype=torch.complex128, device="cuda")
    g, dv, dt = T.adjoint(zb.T, gb.T, e, e[:, 0], 1)
    torch.cuda.synchronize()
    assert np.array_equal(g.cpu().numpy(), G) and dv.numel() == 0


def _split_pair_z(Z, G, V, tau, nbw):
    """The complex split pair on device copies: (forward result, grad Z_in,
    dv, dtau, status of the two calls)."""
    import torch
    import paper_2002_10991_amd as T
    n, nev = Z.shape
    Vd = torch.from_numpy(V).to("cuda")
    td = torch.from_numpy(tau).to("cuda")
    zb = torch.from_numpy(np.ascontiguousarray(Z.T)).to("cuda")
    gb = torch.from_numpy(np.ascontiguousarray(G.T)).to("cuda")
    K = len(tau)
    dv = torch.empty(K, nbw, dtype=torch.complex128, device="cuda")
    dt = torch.empty(K, dtype=torch.complex128, device="cuda")
    nb = T.trbt_adjoint_workspace_bytes_z(n, nbw, nev)
    w = torch.empty(nb + 256, dtype=torch.uint8, device="cuda")
    w = w[(-w.data_ptr()) % 256:][:nb]
    r1 = T.trans_ev_tridi_to_band_fwd_ckpt_z(n, nbw, nev, Vd, td, zb, n, 16, w, nb)
    r2 = T.trans_ev_tridi_to_band_bwd_ckpt_z(n, nbw, nev, Vd, td, gb, n, dv, dt, 16, w, nb)
    torch.cuda.synchronize()
    if (r1, r2) == (0, 0):
        assert T.trbt_work_check(w) == 0
    return zb.cpu().numpy(), gb.cpu().numpy(), dv.cpu().numpy(), dt.cpu().numpy(), (r1, r2)


# the last three run the checkpointing forward and the sweep with slot
# groups (enough slots per strip, few strips)
@pytest.mark.parametrize("n,nbw,nev", [(301, 64, 63), (150, 32, 40), (200, 48, 17),
                                       (100, 16, 33), (1100, 64, 40), (700, 16, 33),
                                       (1500, 48, 70)])
def test_complex_split_pair(oracle_mod, n, nbw, nev):
    """trans_ev_tridi_to_band_{fwd,bwd}_ckpt_z: the forward result bitwise
    the plain complex forward's, the gradients bitwise the one-call complex
    adjoint's, and both against the oracle."""
    import torch
    import paper_2002_10991_amd as T
    Z, G, V, tau = _inputs(n, nbw, nev, 640 + n + nbw)
    print(f"[gpu] complex split pair n={n} nbw={nbw} nev={nev}", flush=True)
    fz, gz, dv, dt, rcs = _split_pair_z(Z, G, V, tau, nbw)
    assert rcs == (0, 0)
    zb = torch.from_numpy(np.ascontiguousarray(Z.T)).to("cuda")
    T.back_transform(zb.T, torch.from_numpy(V).to("cuda"), torch.from_numpy(tau).to("cuda"), nbw)
    torch.cuda.synchronize()
    assert np.array_equal(fz, zb.cpu().numpy())
    oZ, ov, ot = gpu_adjoint_z(Z, G, V, tau, nbw)
    assert np.array_equal(gz.T, oZ) and np.array_equal(dv, ov) and np.array_equal(dt, ot)
    rZ, rv, rt = oracle_mod.adjoint(Z, G, V, tau, nbw)
    assert _relerr(gz.T, rZ) <= TOL and _relerr(dv, rv) <= TOL and _relerr(dt, rt) <= TOL


def test_complex_split_pair_other_band_widths():
    """Band widths without blocked kernels: status -2 from both halves
    (before any launch); the autograd wrapper then takes the one-call
    adjoint."""
    Z, G, V, tau = _inputs(90, 8, 10, 5)
    *_, rcs = _split_pair_z(Z, G, V, tau, 8)
    assert rcs == (-2, -2)


def test_complex_autograd_gradcheck_blocked():
    """gradcheck through the split pair (nbw = 16)."""
    import torch
    import paper_2002_10991_amd as T
    n, nbw, nev = 36, 16, 2
    Z, _, V, tau = _inputs(n, nbw, nev, 78, general_tau=True)
    print(f"[gpu] gradcheck complex n={n} nbw={nbw} nev={nev}", flush=True)
    args = [torch.from_numpy(np.ascontiguousarray(a)).to("cuda").requires_grad_(True)
            for a in (Z, V, tau)]
    assert torch.autograd.gradcheck(lambda z, v, t: T.back_transform_autograd(z, v, t, nbw),
                                    args, eps=1e-6, atol=1e-7, rtol=1e-6)


def test_complex_autograd_gradcheck():
    import torch
    import paper_2002_10991_amd as T
    n, nbw, nev = 10, 3, 2
    Z, _, V, tau = _inputs(n, nbw, nev, 77, general_tau=True)
    print(f"[gpu] gradcheck complex n={n} nbw={nbw} nev={nev}", flush=True)
    args = [torch.from_numpy(np.ascontiguousarray(a)).to("cuda").requires_grad_(True)
            for a in (Z, V, tau)]
    assert torch.autograd.gradcheck(lambda z, v, t: T.back_transform_autograd(z, v, t, nbw),
                                    args, eps=1e-6, atol=1e-7, rtol=1e-6)


def test_complex_autograd_matches_oracle(oracle_mod):
    import torch
    import paper_2002_10991_amd as T
    n, nbw, nev = 150, 32, 20
    Z, G, V, tau = _inputs(n, nbw, nev, 88)
    Zt, Vt, tt = (torch.from_numpy(np.ascontiguousarray(a)).to("cuda").requires_grad_(True)
                  for a in (Z, V, tau))
    Gt = torch.from_numpy(G).to("cuda")
    # L = Re sum conj(G) Y: its gradient with respect to Y is G
    torch.real(torch.sum(torch.conj(Gt) * T.back_transform_autograd(Zt, Vt, tt, nbw))).backward()
    rZ, rv, rt = oracle_mod.adjoint(Z, G, V, tau, nbw)
    for got, ref in ((Zt.grad, rZ), (Vt.grad, rv), (tt.grad, rt)):
        assert _relerr(got.cpu().numpy(), ref) <= TOL


def test_complex_adjoint_full_n_column_subset(oracle_mod):
    # n and nbw of the differentiation workload, 64 columns (the oracle's
    # cost grows with the columns; the GPU runs them as one wave)
    n, nbw, nev = 4096, 64, 64
    Z, G, V, tau = _inputs(n, nbw, nev, 2005)
    rZ, rv, rt = oracle_mod.adjoint(Z, G, V, tau, nbw)
    gZ, gv, gt = gpu_adjoint_z(Z, G, V, tau, nbw)
    assert _relerr(gZ, rZ) <= TOL and _relerr(gv, rv) <= TOL and _relerr(gt, rt) <= TOL


def test_complex_adjoint_c5_shape_512_columns(oracle_mod):
    """n=4096, nbw=64 with 512 columns (32 strips of the column sums behind
    grad v and grad tau): every output against the oracle."""
    n, nbw, nev = 4096, 64, 512
    Z, G, V, tau = _inputs(n, nbw, nev, 1005)
    gZ, gv, gt = gpu_adjoint_z(Z, G, V, tau, nbw)

    def compute():
        rZ, rv, rt = oracle_mod.adjoint(Z, G, V, tau, nbw)
        return {"dZ": rZ, "dv": rv, "dtau": rt}
    r = oracle_cache.cached("adjoint", dict(n=n, nbw=nbw, nev=nev, dtype="z", seed=1005),
                            compute)
    rZ, rv, rt = r["dZ"], r["dv"], r["dtau"]
    e = (_relerr(gZ, rZ), _relerr(gv, rv), _relerr(gt, rt))
    print(f"[gpu] complex adjoint nev=512 rel errors {e}", flush=True)
    assert max(e) <= TOL


@pytest.mark.timeout(900)
def test_complex_adjoint_c5_full_nev(oracle_mod):
    """The complex differentiation workload at its full width (n=4096,
    nbw=64, nev=2048: 128 column strips behind grad v and grad tau, the
    shape the benchmark times): every output against the oracle."""
    n, nbw, nev = 4096, 64, 2048
    Z, G, V, tau = _inputs(n, nbw, nev, 2005)
    gZ, gv, gt = gpu_adjoint_z(Z, G, V, tau, nbw)

    def compute():
        rZ, rv, rt = oracle_mod.adjoint(Z, G, V, tau, nbw)
        return {"dZ": rZ, "dv": rv, "dtau": rt}
    r = oracle_cache.cached("adjoint", dict(n=n, nbw=nbw, nev=nev, dtype="z", seed=2005),
                            compute)
    e = (_relerr(gZ, r["dZ"]), _relerr(gv, r["dv"]), _relerr(gt, r["dtau"]))
    print(f"[gpu] complex adjoint nev=2048 rel errors {e}", flush=True)
    assert max(e) <= TOL


@pytest.mark.parametrize("n,nbw,nev", [(300, 64, 40), (97, 7, 10)])
def test_complex_adjoint_v0_not_one_nan_tail(oracle_mod, n, nbw, nev):
    """Complex v[0] != 1 (v scaled by alpha, tau by 1/|alpha|^2) and NaN beyond
    each reflector's length."""
    import synth
    Z, G, V, tau = _inputs(n, nbw, nev, 4200 + n)
    lengths = synth.reflector_lengths(n, nbw)
    rng = np.random.default_rng(n + 1)
    alpha = rng.uniform(0.5, 2.0, len(tau)) * np.exp(1j * rng.uniform(0, 2 * np.pi, len(tau)))
    V2 = V * alpha[:, None]
    t2 = tau / np.abs(alpha) ** 2
    Vn = V2.copy()
    Vn[np.arange(nbw)[None, :] >= lengths[:, None]] = np.nan
    rZ, rv, rt = oracle_mod.adjoint(Z, G, V2, t2, nbw)
    gZ, gv, gt = gpu_adjoint_z(Z, G, Vn, t2, nbw)
    mask = np.arange(nbw)[None, :] < lengths[:, None]
    assert _relerr(gZ, rZ) <= TOL and _relerr(gt, rt) <= TOL
    assert _relerr(gv[mask], rv[mask]) <= TOL and np.all(gv[~mask] == 0)
