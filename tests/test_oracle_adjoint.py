"""Pins for the oracle's adjoint of the real back-transformation
Z_out = H_0 ... H_{K-1} Z_in (Eq. 2stage_bkwd1, real reflectors),
L = <G, Z_out>, so dL/dZ_out = G.

Independent checks (none re-runs the oracle's own recurrences):
  * dense-Q brute force on tiny problems: explicit n x n matrices H_k,
    dL/dH_k = A_k^T G C_k^T with A_k = H_0..H_{k-1}, C_k = H_{k+1}..H_{K-1} Z_in,
    then dtau_k = -v^T (dL/dH_k) v and dv_k = -tau_k (dL/dH_k + dL/dH_k^T) v;
  * central finite differences of the forward map on the n=64, nbw=8, nev=16
    case built by the stage-2 pipeline (band matrix, bulge chase, QL);
  * the transpose identity <G, Q Z> = <Q^T G, Z> against the forward oracle;
  * linearity in G, and zero derivative entries beyond each reflector's length.
"""
import numpy as np
import pytest


def _inputs(n, nbw, nev, seed, oracle_mod, general_tau=False):
    import synth
    lengths = synth.reflector_lengths(n, nbw)
    V, tau = synth.unitary_reflectors(lengths, nbw, seed, "d")
    if general_tau:   # the derivative formulas hold for any tau, not only 2/|v|^2
        tau = np.random.default_rng(seed + 7).uniform(0.3, 1.7, len(tau))
    Z = synth.gaussian(n, nev, seed + 1, "d")
    G = synth.gaussian(n, nev, seed + 2, "d")
    return Z, G, V, tau, lengths


def _dense_grad(n, nbw, V, tau, Z, G, oracle_mod):
    st, sl, r0, ln = oracle_mod.reflector_table(n, nbw)
    K = len(tau)
    H, vh = [], []
    for k in range(K):
        v = np.zeros(n)
        v[r0[k]: r0[k] + ln[k]] = V[k, : ln[k]]
        vh.append(v)
        H.append(np.eye(n) - tau[k] * np.outer(v, v))
    pre = [np.eye(n)]                     # pre[k] = H_0 ... H_{k-1}
    for k in range(K):
        pre.append(pre[-1] @ H[k])
    suf = [None] * (K + 1)                # suf[k] = H_k ... H_{K-1} Z
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


@pytest.mark.parametrize("n,nbw,nev,general", [(12, 3, 4, False), (17, 4, 5, True),
                                               (9, 8, 2, True), (14, 2, 3, False)])
def test_adjoint_matches_dense_q(oracle_mod, n, nbw, nev, general):
    Z, G, V, tau, _ = _inputs(n, nbw, nev, 10 + n, oracle_mod, general)
    dZ, dv, dt = oracle_mod.adjoint(Z, G, V, tau, nbw)
    rZ, rv, rt = _dense_grad(n, nbw, V, tau, Z, G, oracle_mod)
    assert np.allclose(dZ, rZ, rtol=0, atol=1e-12 * np.abs(rZ).max())
    assert np.allclose(dv, rv, rtol=0, atol=1e-12 * np.abs(rv).max())
    assert np.allclose(dt, rt, rtol=0, atol=1e-12 * np.abs(rt).max())


def _loss(oracle_mod, Z, G, V, tau, nbw):
    return float(np.sum(G * oracle_mod.back_transform(Z, V, tau, nbw)))


def test_adjoint_central_differences_fd_case(oracle_mod):
    """n=64, nbw=8, nev=16: reflectors from the bulge chase of a seeded band
    matrix, Z_in = the lowest 16 QL eigenvectors, G ~ N(0,1).  Directional
    derivatives along seeded random directions agree with central
    differences (h = 1e-6) to 1e-7 relative."""
    import synth
    n, nbw, nev = 64, 8, 16
    ab = synth.band_matrix(n, nbw, 3005, "d")
    p = oracle_mod.stage2_pipeline(ab, nbw, nev)
    V, tau, Z = p["hh_v"], p["hh_tau"], p["Z_in"]
    G = synth.gaussian(n, nev, 3006, "d")
    lengths = synth.reflector_lengths(n, nbw)
    dZ, dv, dt = oracle_mod.adjoint(Z, G, V, tau, nbw)
    rng = np.random.default_rng(3007)
    mask = np.arange(nbw)[None, :] < lengths[:, None]
    h = 1e-6
    for trial in range(3):
        dV = rng.standard_normal(V.shape) * mask
        dT = rng.standard_normal(tau.shape)
        dZi = rng.standard_normal(Z.shape)
        fd = (_loss(oracle_mod, Z + h * dZi, G, V + h * dV, tau + h * dT, nbw)
              - _loss(oracle_mod, Z - h * dZi, G, V - h * dV, tau - h * dT, nbw)) / (2 * h)
        an = np.sum(dZ * dZi) + np.sum(dv * dV) + np.sum(dt * dT)
        assert abs(fd - an) <= 1e-7 * max(abs(an), 1.0), (trial, fd, an)
    # a few single entries as well
    for k, i in [(0, 0), (5, 3), (len(tau) - 1, 1), (100, 7)]:
        e = np.zeros_like(V)
        e[k, i] = 1.0
        fd = (_loss(oracle_mod, Z, G, V + h * e, tau, nbw)
              - _loss(oracle_mod, Z, G, V - h * e, tau, nbw)) / (2 * h)
        assert abs(fd - dv[k, i]) <= 1e-7 * max(abs(dv[k, i]), 1.0)
        et = np.zeros_like(tau)
        et[k] = 1.0
        fd = (_loss(oracle_mod, Z, G, V, tau + h * et, nbw)
              - _loss(oracle_mod, Z, G, V, tau - h * et, nbw)) / (2 * h)
        assert abs(fd - dt[k]) <= 1e-7 * max(abs(dt[k]), 1.0)


def test_adjoint_transpose_identity_and_padding(oracle_mod):
    n, nbw, nev = 300, 16, 7
    Z, G, V, tau, lengths = _inputs(n, nbw, nev, 31, oracle_mod)
    dZ, dv, dt = oracle_mod.adjoint(Z, G, V, tau, nbw)
    QZ = oracle_mod.back_transform(Z, V, tau, nbw)
    lhs, rhs = np.sum(G * QZ), np.sum(dZ * Z)
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(G) * np.linalg.norm(Z)
    mask = np.arange(nbw)[None, :] >= lengths[:, None]
    assert np.all(dv[mask] == 0.0)
    # Z_in -> dL/dZ_in is Q^T G: orthogonal, so the norm is kept
    assert abs(np.linalg.norm(dZ) - np.linalg.norm(G)) <= 1e-12 * np.linalg.norm(G)


def test_adjoint_linear_in_g_and_degenerate(oracle_mod):
    n, nbw, nev = 120, 8, 5
    Z, G1, V, tau, _ = _inputs(n, nbw, nev, 41, oracle_mod)
    G2 = np.random.default_rng(5).standard_normal(G1.shape)
    a = oracle_mod.adjoint(Z, G1, V, tau, nbw)
    b = oracle_mod.adjoint(Z, G2, V, tau, nbw)
    c = oracle_mod.adjoint(Z, 2.0 * G1 - 3.0 * G2, V, tau, nbw)
    for x, y, w in zip(a, b, c):
        assert np.allclose(w, 2.0 * x - 3.0 * y, rtol=0, atol=1e-12 * max(np.abs(w).max(), 1))
    # no reflectors: dL/dZ_in = G, nothing else
    dZ, dv, dt = oracle_mod.adjoint(Z, G1, np.zeros((0, 1)), np.zeros(0), 1)
    assert np.array_equal(dZ, G1) and dv.size == 0 and dt.size == 0
