"""Pins for the oracle's adjoint of the complex back-transformation
Z_out = H_0 ... H_{K-1} Z_in, H_k = I - tau_k v_k v_k^H (Eq. 2stage_bkwd1),
for the real loss L = Re <G, Z_out> = Re sum conj(G) Z_out, in the
conjugate-Wirtinger convention (dL = Re sum conj(grad_x) dx for every complex
perturbation dx; PyTorch's convention).

Independent checks (none re-runs the oracle's per-column recurrences):
  * dense brute force on tiny problems with explicit n x n matrices: with
    A_k = H_0..H_{k-1}, C_k = H_{k+1}..H_{K-1} Z_in and D = A_k^H G C_k^H
    (the gradient with respect to H_k), dH_k = -dtau v v^H - tau dv v^H -
    tau v dv^H gives grad_tau = -v^H D v, grad_v = -conj(tau) D v - tau D^H v,
    and grad_Z_in = Q^H G;
  * central differences of the forward oracle along random complex directions;
  * real data carried in complex arrays reproduces the real adjoint exactly.
"""
import numpy as np
import pytest


def _inputs(n, nbw, nev, seed, general_tau=False):
    import synth
    lengths = synth.reflector_lengths(n, nbw)
    V, tau = synth.unitary_reflectors(lengths, nbw, seed, "z")
    if general_tau:   # the formulas hold for any complex tau
        rng = np.random.default_rng(seed + 7)
        tau = rng.uniform(0.3, 1.7, len(tau)) + 1j * rng.uniform(-0.8, 0.8, len(tau))
    Z = synth.gaussian(n, nev, seed + 1, "z")
    G = synth.gaussian(n, nev, seed + 2, "z")
    return Z, G, V, tau


def _dense_grad(n, nbw, V, tau, Z, G, oracle_mod):
    st, sl, r0, ln = oracle_mod.reflector_table(n, nbw)
    K = len(tau)
    H, vh = [], []
    for k in range(K):
        v = np.zeros(n, complex)
        v[r0[k]: r0[k] + ln[k]] = V[k, : ln[k]]
        vh.append(v)
        H.append(np.eye(n) - tau[k] * np.outer(v, v.conj()))
    pre = [np.eye(n, dtype=complex)]
    for k in range(K):
        pre.append(pre[-1] @ H[k])
    suf = [None] * (K + 1)
    suf[K] = Z.copy()
    for k in range(K - 1, -1, -1):
        suf[k] = H[k] @ suf[k + 1]
    dv = np.zeros((K, nbw), complex)
    dt = np.zeros(K, complex)
    for k in range(K):
        D = pre[k].conj().T @ G @ suf[k + 1].conj().T
        v = vh[k]
        dt[k] = -(v.conj() @ D @ v)
        full = -np.conj(tau[k]) * (D @ v) - tau[k] * (D.conj().T @ v)
        dv[k, : ln[k]] = full[r0[k]: r0[k] + ln[k]]
    return pre[K].conj().T @ G, dv, dt


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("n,nbw,nev,general", [(12, 3, 4, False), (17, 4, 5, True),
                                               (9, 8, 2, True), (14, 2, 3, False)])
def test_complex_adjoint_matches_dense_q(oracle_mod, n, nbw, nev, general):
    Z, G, V, tau = _inputs(n, nbw, nev, 30 + n, general)
    dZ, dv, dt = oracle_mod.adjoint(Z, G, V, tau, nbw)
    rZ, rv, rt = _dense_grad(n, nbw, V, tau, Z, G, oracle_mod)
    assert _rel(dZ, rZ) < 1e-13
    assert _rel(dv, rv) < 1e-13
    assert _rel(dt, rt) < 1e-13


def test_complex_adjoint_central_differences(oracle_mod):
    n, nbw, nev = 64, 8, 16
    Z, G, V, tau = _inputs(n, nbw, nev, 3005, general_tau=True)
    K = len(tau)
    _, _, r0, ln = oracle_mod.reflector_table(n, nbw)
    dZ, dv, dt = oracle_mod.adjoint(Z, G, V, tau, nbw)

    def loss(Zx, Vx, tx):
        Y = oracle_mod.back_transform(Zx, Vx, tx, nbw)
        return float(np.real(np.sum(np.conj(G) * Y)))

    rng = np.random.default_rng(11)
    mask = np.arange(nbw)[None, :] < ln[:, None]
    for _ in range(3):
        eZ = rng.standard_normal(Z.shape) + 1j * rng.standard_normal(Z.shape)
        eV = (rng.standard_normal(V.shape) + 1j * rng.standard_normal(V.shape)) * mask
        et = rng.standard_normal(K) + 1j * rng.standard_normal(K)
        h = 1e-6
        fd = (loss(Z + h * eZ, V + h * eV, tau + h * et)
              - loss(Z - h * eZ, V - h * eV, tau - h * et)) / (2 * h)
        an = np.real(np.sum(np.conj(dZ) * eZ) + np.sum(np.conj(dv) * eV)
                     + np.sum(np.conj(dt) * et))
        assert abs(fd - an) <= 1e-7 * max(abs(an), 1.0), (fd, an)


def test_complex_adjoint_of_real_data_is_the_real_adjoint(oracle_mod):
    import synth
    n, nbw, nev = 70, 6, 9
    lengths = synth.reflector_lengths(n, nbw)
    V, tau = synth.unitary_reflectors(lengths, nbw, 5, "d")
    Z = synth.gaussian(n, nev, 6, "d")
    G = synth.gaussian(n, nev, 7, "d")
    rZ, rv, rt = oracle_mod.adjoint(Z, G, V, tau, nbw)
    cZ, cv, ct = oracle_mod.adjoint(Z.astype(complex), G.astype(complex), V.astype(complex),
                                    tau.astype(complex), nbw)
    for c, r in ((cZ, rZ), (cv, rv), (ct, rt)):
        assert np.all(c.imag == 0)
        assert _rel(c.real, r) < 1e-15


def test_complex_adjoint_padding_and_degenerate(oracle_mod):
    n, nbw, nev = 20, 6, 3
    Z, G, V, tau = _inputs(n, nbw, nev, 77)
    _, dv, _ = oracle_mod.adjoint(Z, G, V, tau, nbw)
    _, _, _, ln = oracle_mod.reflector_table(n, nbw)
    for k in range(len(ln)):
        assert np.all(dv[k, ln[k]:] == 0)
    # nev = 0: zero parameter gradients
    dZ0, dv0, dt0 = oracle_mod.adjoint(Z[:, :0], G[:, :0], V, tau, nbw)
    assert dZ0.shape == (n, 0) and np.all(dv0 == 0) and np.all(dt0 == 0)
