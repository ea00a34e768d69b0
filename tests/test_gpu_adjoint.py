"""GPU parity of the adjoint (reverse-mode derivative) of the real
back-transformation, through the C ABI, against the CPU oracle's adjoint,
the dense-Q gradient on tiny problems and central finite differences.

Tolerance: relative Frobenius error <= 1e-12 for dL/dZ_in, dL/dv and
dL/dtau (each compared as a whole array).  The blocked path sums the
column contributions in a different order than the oracle (per 16-column
strip, then over strips), which moves results by ~1e-15 relative.
"""
import numpy as np
import pytest

import oracle_cache
from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

TOL = 1e-12


def _torch():
    import torch
    return torch


def _relerr(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _inputs(n, nbw, nev, seed, general_tau=False):
    import synth
    lengths = synth.reflector_lengths(n, nbw)
    V, tau = synth.unitary_reflectors(lengths, nbw, seed, "d")
    if general_tau:
        tau = np.random.default_rng(seed + 7).uniform(0.3, 1.7, len(tau))
    Z = synth.gaussian(n, nev, seed + 1, "d")
    G = synth.gaussian(n, nev, seed + 2, "d")
    return Z, G, V, tau


def _dev_colmajor(A, ld, fill=0.0):
    torch = _torch()
    n, m = A.shape
    host = np.full((max(m, 1), ld), fill)
    host[:m, :n] = A.T
    buf = torch.from_numpy(host).to("cuda")
    return buf, buf.T[:n, :m]


def gpu_adjoint(Z, G, V, tau, nbw, ldz=None, ldg=None, pad_fill=0.0):
    import paper_2002_10991_amd as T
    torch = _torch()
    n, nev = Z.shape
    ldz = ldz or max(n, 1)
    ldg = ldg or max(n, 1)
    print(f"[gpu] adjoint n={n} nbw={nbw} nev={nev} ldz={ldz} ldg={ldg}", flush=True)
    zb, zv = _dev_colmajor(Z, ldz, pad_fill)
    gb, gv = _dev_colmajor(G, ldg, pad_fill)
    Vd = torch.from_numpy(np.ascontiguousarray(V)).to("cuda")
    td = torch.from_numpy(np.ascontiguousarray(tau)).to("cuda")
    K = len(tau)
    dv = torch.full((max(K, 1), nbw), np.nan, dtype=torch.float64, device="cuda")
    dt = torch.full((max(K, 1),), np.nan, dtype=torch.float64, device="cuda")
    nb = T.trbt_adjoint_workspace_bytes_d(n, nbw, nev)
    work = None
    if nb:
        w = torch.empty(nb + 256, dtype=torch.uint8, device="cuda")
        work = w[(-w.data_ptr()) % 256:][:nb]
    rc = T.trans_ev_tridi_to_band_adjoint_d(n, nbw, nev, Vd if K else None, td if K else None,
                                            zb if nev else None, ldz, gb if nev else None, ldg,
                                            dv if K else None, dt if K else None, 16, work, nb)
    torch.cuda.synchronize()
    assert rc == 0, rc
    if work is not None:
        assert T.trbt_work_check(work) == 0, "device wait timeout flag set"
    return (gb.cpu().numpy(), zb.cpu().numpy(), dv.cpu().numpy()[:K], dt.cpu().numpy()[:K])


SHAPES = [
    # blocked compact-WY adjoint (nbw in {16, 32, 48, 64}), ragged nev
    (40, 16, 17), (100, 16, 33), (150, 32, 65), (200, 48, 16), (300, 64, 64),
    (301, 64, 63), (517, 64, 100), (130, 32, 1),
    # streaming adjoint (other nbw)
    (50, 2, 7), (61, 3, 20), (90, 8, 31), (129, 31, 64), (140, 33, 65), (100, 24, 70),
]


@pytest.mark.parametrize("n,nbw,nev", SHAPES)
def test_adjoint_vs_oracle(oracle_mod, n, nbw, nev):
    Z, G, V, tau = _inputs(n, nbw, nev, 2000 + n + nbw)
    rZ, rv, rt = oracle_mod.adjoint(Z, G, V, tau, nbw)
    gb, zb, dv, dt = gpu_adjoint(Z, G, V, tau, nbw)
    assert _relerr(gb[:nev, :n].T, rZ) <= TOL
    assert _relerr(dv, rv) <= TOL
    assert _relerr(dt, rt) <= TOL
    assert np.array_equal(zb[:nev, :n].T, Z)     # Z_in is read only


@pytest.mark.parametrize("n,nbw,nev", [(150, 32, 40), (90, 8, 31)])
def test_adjoint_general_tau_and_padding(oracle_mod, n, nbw, nev):
    """tau off the Householder value (non-orthogonal H) and ldz, ldg > n:
    the padding rows are never touched."""
    Z, G, V, tau = _inputs(n, nbw, nev, 77, general_tau=True)
    rZ, rv, rt = oracle_mod.adjoint(Z, G, V, tau, nbw)
    gb, zb, dv, dt = gpu_adjoint(Z, G, V, tau, nbw, ldz=n + 5, ldg=n + 3, pad_fill=4321.0)
    assert np.all(gb[:, n:] == 4321.0) and np.all(zb[:, n:] == 4321.0)
    assert _relerr(gb[:nev, :n].T, rZ) <= TOL
    assert _relerr(dv, rv) <= TOL
    assert _relerr(dt, rt) <= TOL


def _dense_grad(n, nbw, V, tau, Z, G, oracle_mod):
    st, sl, r0, ln = oracle_mod.reflector_table(n, nbw)
    K = len(tau)
    H, vh = [], []
    for k in range(K):
        v = np.zeros(n)
        v[r0[k]: r0[k] + ln[k]] = V[k, : ln[k]]
        vh.append(v)
        H.append(np.eye(n) - tau[k] * np.outer(v, v))
    pre = [np.eye(n)]
    for k in range(K):
        pre.append(pre[-1] @ H[k])
    suf = [None] * (K + 1)
    suf[K] = Z.copy()
    for k in range(K - 1, -1, -1):
        suf[k] = H[k] @ suf[k + 1]
    dv = np.zeros((K, nbw))
    dt = np.zeros(K)
    for k in range(K):
        D = pre[k].T @ G @ suf[k + 1].T
        dt[k] = -vh[k] @ D @ vh[k]
        full = -tau[k] * (D + D.T) @ vh[k]
        dv[k, : ln[k]] = full[r0[k]: r0[k] + ln[k]]
    return pre[K].T @ G, dv, dt


@pytest.mark.parametrize("n,nbw,nev", [(17, 4, 5), (40, 16, 9), (45, 32, 20)])
def test_adjoint_dense_q(oracle_mod, n, nbw, nev):
    Z, G, V, tau = _inputs(n, nbw, nev, 11 + n, general_tau=True)
    rZ, rv, rt = _dense_grad(n, nbw, V, tau, Z, G, oracle_mod)
    gb, _, dv, dt = gpu_adjoint(Z, G, V, tau, nbw)
    assert _relerr(gb[:nev, :n].T, rZ) <= 1e-12
    assert _relerr(dv, rv) <= 1e-12
    assert _relerr(dt, rt) <= 1e-12


def _gpu_loss(Z, G, V, tau, nbw):
    import paper_2002_10991_amd as T
    torch = _torch()
    n, nev = Z.shape
    zb = torch.from_numpy(np.ascontiguousarray(Z.T)).to("cuda")
    T.back_transform(zb.T, torch.from_numpy(np.ascontiguousarray(V)).to("cuda"),
                     torch.from_numpy(np.ascontiguousarray(tau)).to("cuda"), nbw)
    torch.cuda.synchronize()
    return float(np.sum(G * zb.cpu().numpy().T))


@pytest.mark.parametrize("nbw", [8, 16])
def test_adjoint_central_differences(oracle_mod, nbw):
    """The n=64, nev=16 case from the stage-2 pipeline (band matrix, bulge
    chase, QL eigenvectors); directional derivatives of L = <G, Z_out> from
    the GPU adjoint against central differences of the GPU forward."""
    import synth
    n, nev = 64, 16
    ab = synth.band_matrix(n, nbw, 3005, "d")
    p = oracle_mod.stage2_pipeline(ab, nbw, nev)
    V, tau, Z = p["hh_v"], p["hh_tau"], p["Z_in"]
    G = synth.gaussian(n, nev, 3006, "d")
    gb, _, dv, dt = gpu_adjoint(Z, G, V, tau, nbw)
    dZ = gb[:nev, :n].T
    lengths = synth.reflector_lengths(n, nbw)
    mask = np.arange(nbw)[None, :] < lengths[:, None]
    rng = np.random.default_rng(3007)
    h = 1e-6
    for trial in range(3):
        dV = rng.standard_normal(V.shape) * mask
        dT = rng.standard_normal(tau.shape)
        dZi = rng.standard_normal(Z.shape)
        fd = (_gpu_loss(Z + h * dZi, G, V + h * dV, tau + h * dT, nbw)
              - _gpu_loss(Z - h * dZi, G, V - h * dV, tau - h * dT, nbw)) / (2 * h)
        an = np.sum(dZ * dZi) + np.sum(dv * dV) + np.sum(dt * dT)
        assert abs(fd - an) <= 1e-7 * max(abs(an), 1.0), (trial, fd, an)


@pytest.mark.parametrize("nbw", [64, 7])
def test_adjoint_deterministic(oracle_mod, nbw):
    Z, G, V, tau = _inputs(257, nbw, 50, 5)
    a = gpu_adjoint(Z, G, V, tau, nbw)
    b = gpu_adjoint(Z, G, V, tau, nbw)
    for x, y in zip(a, b):
        assert np.array_equal(x.view(np.uint8), y.view(np.uint8))


def test_adjoint_degenerate(oracle_mod):
    import paper_2002_10991_amd as T
    torch = _torch()
    # nev = 0: dv and dtau are zeroed, nothing else is touched
    n, nbw = 100, 32
    K = T.trbt_num_reflectors(n, nbw)
    V = torch.randn(K, nbw, dtype=torch.float64, device="cuda")
    tau = torch.randn(K, dtype=torch.float64, device="cuda")
    dv = torch.full((K, nbw), 7.0, dtype=torch.float64, device="cuda")
    dt = torch.full((K,), 7.0, dtype=torch.float64, device="cuda")
    rc = T.trans_ev_tridi_to_band_adjoint_d(n, nbw, 0, V, tau, None, n, None, n, dv, dt, 16,
                                            None, 0)
    torch.cuda.synchronize()
    assert rc == 0 and torch.all(dv == 0) and torch.all(dt == 0)
    # no reflectors: G is dL/dZ_in already
    G = torch.randn(5, 10, dtype=torch.float64, device="cuda")
    G0 = G.clone()
    rc = T.trans_ev_tridi_to_band_adjoint_d(10, 1, 5, None, None, G, 10, G, 10, None, None, 16,
                                            None, 0)
    torch.cuda.synchronize()
    assert rc == 0 and torch.equal(G, G0)
    # workspace too small
    Z = torch.zeros(4, n, dtype=torch.float64, device="cuda")
    need = T.trbt_adjoint_workspace_bytes_d(n, nbw, 4)
    w = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    w = w[(-w.data_ptr()) % 256:]
    rc = T.trans_ev_tridi_to_band_adjoint_d(n, nbw, 4, V, tau, Z, n, Z.clone(), n, dv, dt, 16,
                                            w, need - 8)
    assert rc == -101


def test_autograd_function(oracle_mod):
    """torch.autograd through BackTransform (forward kernel + hand-written
    adjoint) against the oracle adjoint."""
    import paper_2002_10991_amd as T
    torch = _torch()
    n, nbw, nev = 200, 32, 30
    Z, G, V, tau = _inputs(n, nbw, nev, 91)
    Zt = torch.from_numpy(Z).to("cuda").requires_grad_(True)
    Vt = torch.from_numpy(V).to("cuda").requires_grad_(True)
    tt = torch.from_numpy(tau).to("cuda").requires_grad_(True)
    Z0 = Zt.detach().clone()
    out = T.back_transform_autograd(Zt, Vt, tt, nbw)
    torch.cuda.synchronize()
    assert torch.equal(Zt.detach(), Z0)          # the input is never written
    loss = (out * torch.from_numpy(G).to("cuda")).sum()
    loss.backward()
    ref_out = oracle_mod.back_transform(Z, V, tau, nbw)
    assert _relerr(out.detach().cpu().numpy(), ref_out) <= TOL
    rZ, rv, rt = oracle_mod.adjoint(Z, G, V, tau, nbw)
    assert _relerr(Zt.grad.cpu().numpy(), rZ) <= TOL
    assert _relerr(Vt.grad.cpu().numpy(), rv) <= TOL
    assert _relerr(tt.grad.cpu().numpy(), rt) <= TOL


def test_c5_full_n_exact_columns(oracle_mod):
    """n=4096, nbw=64 (the differentiation workload's reflectors) on 256
    columns: every output against the oracle adjoint."""
    import synth
    n, nbw, nev = 4096, 64, 256
    lengths = synth.reflector_lengths(n, nbw)
    V, tau = synth.unitary_reflectors(lengths, nbw, 1005, "d")
    Z = synth.gaussian(n, nev, 1006, "d")
    G = synth.gaussian(n, nev, 2005, "d")
    rZ, rv, rt = oracle_mod.adjoint(Z, G, V, tau, nbw)
    gb, _, dv, dt = gpu_adjoint(Z, G, V, tau, nbw)
    assert _relerr(gb[:nev, :n].T, rZ) <= TOL
    assert _relerr(dv, rv) <= TOL
    assert _relerr(dt, rt) <= TOL


def test_c5_full_size_properties(oracle_mod):
    """n=4096, nbw=64, nev=2048 (the benchmarked shape): properties that hold
    at any size.  <G, Q Z> = <dL/dZ_in, Z>; ||dL/dZ_in|| = ||G|| (Q
    orthogonal); sampled columns of dL/dZ_in equal the oracle's (columns of
    dL/dZ_in are independent); the directional derivative along (dv, dtau)
    matches central differences of the GPU forward."""
    import paper_2002_10991_amd as T
    import synth
    torch = _torch()
    n, nbw, nev = 4096, 64, 2048
    lengths = synth.reflector_lengths(n, nbw)
    V, tau = synth.unitary_reflectors(lengths, nbw, 1005, "d")
    Z = synth.gaussian(n, nev, 1006, "d")
    G = synth.gaussian(n, nev, 2005, "d")
    gb, _, dv, dt = gpu_adjoint(Z, G, V, tau, nbw)
    dZ = gb[:nev, :n].T
    QZ = oracle_mod.back_transform(Z, V, tau, nbw, cols=np.arange(0, nev, 64))
    cols = np.arange(0, nev, 64)
    lhs = np.sum(G[:, cols] * QZ)
    rhs = np.sum(dZ[:, cols] * Z[:, cols])
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(G[:, cols]) * np.linalg.norm(Z[:, cols])
    assert abs(np.linalg.norm(dZ) - np.linalg.norm(G)) <= 1e-12 * np.linalg.norm(G)
    rZ, _, _ = oracle_mod.adjoint(Z[:, cols[:4]], G[:, cols[:4]], V, tau, nbw)
    assert _relerr(dZ[:, cols[:4]], rZ) <= TOL
    mask = np.arange(nbw)[None, :] < lengths[:, None]
    assert np.all(dv[~mask] == 0.0)
    rng = np.random.default_rng(2006)
    dV = rng.standard_normal(V.shape) * mask
    dT = rng.standard_normal(tau.shape)
    h = 1e-6
    fd = (_gpu_loss(Z, G, V + h * dV, tau + h * dT, nbw)
          - _gpu_loss(Z, G, V - h * dV, tau - h * dT, nbw)) / (2 * h)
    an = np.sum(dv * dV) + np.sum(dt * dT)
    assert abs(fd - an) <= 1e-6 * max(abs(an), 1.0), (fd, an)


def _split_adjoint(Z, G, V, tau, nbw):
    """The split pair on device copies: returns (forward result, dL/dZ_in,
    dv, dtau, fault word)."""
    import paper_2002_10991_amd as T
    torch = _torch()
    n, nev = Z.shape
    Vd = torch.from_numpy(V).to("cuda")
    td = torch.from_numpy(tau).to("cuda")
    zb = torch.from_numpy(np.ascontiguousarray(Z.T)).to("cuda")
    gb = torch.from_numpy(np.ascontiguousarray(G.T)).to("cuda")
    K = len(tau)
    dv = torch.empty(K, nbw, dtype=torch.float64, device="cuda")
    dt = torch.empty(K, dtype=torch.float64, device="cuda")
    nb = T.trbt_adjoint_workspace_bytes_d(n, nbw, nev)
    w = torch.empty(nb + 256, dtype=torch.uint8, device="cuda")
    w = w[(-w.data_ptr()) % 256:][:nb]
    assert T.trans_ev_tridi_to_band_fwd_ckpt_d(n, nbw, nev, Vd, td, zb, n, 16, w, nb) == 0
    assert T.trans_ev_tridi_to_band_bwd_ckpt_d(n, nbw, nev, Vd, td, gb, n, dv, dt, 16, w, nb) == 0
    torch.cuda.synchronize()
    return (zb.cpu().numpy(), gb.cpu().numpy(), dv.cpu().numpy(), dt.cpu().numpy(),
            int(w[:4].view(torch.int32).cpu()[0]))


# the last four run the checkpointing forward and the gradient sweep with
# slot groups (several workgroups per column strip: enough slots per strip
# and few strips; G = 3, 4, 4, 4)
@pytest.mark.parametrize("n,nbw,nev", [(301, 64, 63), (150, 32, 40), (90, 8, 31), (100, 24, 17),
                                       (1100, 64, 40), (2100, 32, 100), (700, 16, 33),
                                       (1500, 48, 70)])
def test_split_adjoint(oracle_mod, n, nbw, nev):
    """Checkpointing forward + backward from the checkpoints: the forward
    result is bitwise the plain forward call's, the gradients bitwise the
    one-call adjoint's, and both match the oracle."""
    import paper_2002_10991_amd as T
    torch = _torch()
    Z, G, V, tau = _inputs(n, nbw, nev, 333 + n)
    print(f"[gpu] split adjoint n={n} nbw={nbw} nev={nev}", flush=True)
    Vd = torch.from_numpy(V).to("cuda")
    td = torch.from_numpy(tau).to("cuda")
    zb = torch.from_numpy(np.ascontiguousarray(Z.T)).to("cuda")
    gb = torch.from_numpy(np.ascontiguousarray(G.T)).to("cuda")
    K = len(tau)
    dv = torch.empty(K, nbw, dtype=torch.float64, device="cuda")
    dt = torch.empty(K, dtype=torch.float64, device="cuda")
    nb = T.trbt_adjoint_workspace_bytes_d(n, nbw, nev)
    w = torch.empty(nb + 256, dtype=torch.uint8, device="cuda")
    w = w[(-w.data_ptr()) % 256:][:nb]
    assert T.trans_ev_tridi_to_band_fwd_ckpt_d(n, nbw, nev, Vd, td, zb, n, 16, w, nb) == 0
    assert T.trans_ev_tridi_to_band_bwd_ckpt_d(n, nbw, nev, Vd, td, gb, n, dv, dt, 16, w, nb) == 0
    torch.cuda.synchronize()
    assert int(w[:4].view(torch.int32).cpu()[0]) == 0
    fwd_plain, _ = _plain_forward(Z, V, tau, nbw)
    assert np.array_equal(zb.cpu().numpy(), fwd_plain)
    one = gpu_adjoint(Z, G, V, tau, nbw)
    assert np.array_equal(gb.cpu().numpy(), one[0][:nev, :n])
    assert np.array_equal(dv.cpu().numpy(), one[2])
    assert np.array_equal(dt.cpu().numpy(), one[3])
    rZ, rv, rt = oracle_mod.adjoint(Z, G, V, tau, nbw)
    assert _relerr(gb.cpu().numpy().T, rZ) <= TOL
    assert _relerr(dv.cpu().numpy(), rv) <= TOL
    assert _relerr(dt.cpu().numpy(), rt) <= TOL


def _plain_forward(Z, V, tau, nbw):
    import paper_2002_10991_amd as T
    torch = _torch()
    zb = torch.from_numpy(np.ascontiguousarray(Z.T)).to("cuda")
    T.back_transform(zb.T, torch.from_numpy(V).to("cuda"), torch.from_numpy(tau).to("cuda"), nbw)
    torch.cuda.synchronize()
    return zb.cpu().numpy(), None


@pytest.mark.parametrize("n,nbw,nev", [(300, 64, 40), (150, 32, 20), (90, 8, 31)])
def test_adjoint_v0_not_one_nan_tail(oracle_mod, n, nbw, nev):
    """v[0] != 1 (v scaled by alpha, tau by 1/alpha^2: the same H) and NaN
    beyond each reflector's length: the adjoint reads v[0] and never the tail;
    gradients against the oracle's on the zero-tail layout."""
    import synth
    Z, G, V, tau = _inputs(n, nbw, nev, 4100 + n)
    lengths = synth.reflector_lengths(n, nbw)
    rng = np.random.default_rng(n)
    alpha = rng.uniform(0.5, 2.0, len(tau)) * rng.choice([-1.0, 1.0], len(tau))
    V2 = V * alpha[:, None]
    t2 = tau / alpha ** 2
    Vn = V2.copy()
    Vn[np.arange(nbw)[None, :] >= lengths[:, None]] = np.nan
    rZ, rv, rt = oracle_mod.adjoint(Z, G, V2, t2, nbw)
    gb, _, dv, dt = gpu_adjoint(Z, G, Vn, t2, nbw)
    assert _relerr(gb[:nev, :n].T, rZ) <= TOL
    mask = np.arange(nbw)[None, :] < lengths[:, None]
    assert _relerr(dv[mask], rv[mask]) <= TOL
    assert np.all(dv[~mask] == 0.0)
    assert _relerr(dt, rt) <= TOL


def test_c5_full_nev_vs_oracle(oracle_mod):
    """The differentiation workload at its full size (n=4096, nbw=64,
    nev=2048, the shape the benchmark times): dL/dZ_in, dL/dv and dL/dtau
    against the oracle's adjoint over all 2048 columns.  dv and dtau are sums
    over every column, so this covers the 128-strip reduction."""
    import synth
    n, nbw, nev = 4096, 64, 2048
    lengths = synth.reflector_lengths(n, nbw)
    V, tau = synth.unitary_reflectors(lengths, nbw, 1005, "d")
    Z = synth.gaussian(n, nev, 1006, "d")
    G = synth.gaussian(n, nev, 2005, "d")
    gb, _, dv, dt = gpu_adjoint(Z, G, V, tau, nbw)

    def compute():
        rZ, rv, rt = oracle_mod.adjoint(Z, G, V, tau, nbw)
        return {"dZ": rZ, "dv": rv, "dtau": rt}
    r = oracle_cache.cached("adjoint", dict(n=n, nbw=nbw, nev=nev, dtype="d", v_seed=1005,
                                            z_seed=1006, g_seed=2005), compute)
    rZ, rv, rt = r["dZ"], r["dv"], r["dtau"]
    e = (_relerr(gb[:nev, :n].T, rZ), _relerr(dv, rv), _relerr(dt, rt))
    print(f"[gpu] C5 full nev rel errors dZ {e[0]:.2e} dv {e[1]:.2e} dtau {e[2]:.2e}", flush=True)
    assert max(e) <= TOL


def test_c5_split_pair_full_size(oracle_mod):
    """The split pair at the benchmarked shape (n=4096, nbw=64, nev=2048:
    128 strips, so both strip kernels run with two workgroups per strip):
    forward result bitwise the plain forward's, gradients bitwise the
    one-call adjoint's, and all of them against the oracle."""
    import synth
    n, nbw, nev = 4096, 64, 2048
    lengths = synth.reflector_lengths(n, nbw)
    V, tau = synth.unitary_reflectors(lengths, nbw, 1005, "d")
    Z = synth.gaussian(n, nev, 1006, "d")
    G = synth.gaussian(n, nev, 2005, "d")
    print(f"[gpu] split adjoint n={n} nbw={nbw} nev={nev}", flush=True)
    fz, gz, dv, dt, fault = _split_adjoint(Z, G, V, tau, nbw)
    assert fault == 0
    fwd_plain, _ = _plain_forward(Z, V, tau, nbw)
    assert np.array_equal(fz, fwd_plain)
    one = gpu_adjoint(Z, G, V, tau, nbw)
    assert np.array_equal(gz, one[0][:nev, :n])
    assert np.array_equal(dv, one[2]) and np.array_equal(dt, one[3])

    def compute():
        rZ, rv, rt = oracle_mod.adjoint(Z, G, V, tau, nbw)
        return {"dZ": rZ, "dv": rv, "dtau": rt}
    r = oracle_cache.cached("adjoint", dict(n=n, nbw=nbw, nev=nev, dtype="d", v_seed=1005,
                                            z_seed=1006, g_seed=2005), compute)
    assert _relerr(gz.T, r["dZ"]) <= TOL
    assert _relerr(dv, r["dv"]) <= TOL and _relerr(dt, r["dtau"]) <= TOL
