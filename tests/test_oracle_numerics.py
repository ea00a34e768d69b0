"""Pins for the oracle's numerical routines against mathematics that does
not depend on the oracle: closed forms, LAPACK via numpy/scipy, brute force
with explicit dense matrices, invariants of unitary transformations."""
import numpy as np
import pytest
import scipy.linalg as sl

import synth

EPS = np.finfo(np.float64).eps


# ---------------------------------------------------------------- larfg
@pytest.mark.parametrize("m", [1, 2, 5, 64])
@pytest.mark.parametrize("cplx", [False, True])
def test_larfg_identity(oracle_mod, m, cplx):
    rng = np.random.default_rng(m + 10 * cplx)
    for trial in range(20):
        x = rng.standard_normal(m) + (1j * rng.standard_normal(m) if cplx else 0)
        if trial == 0 and m > 1:
            x[1:] = 0                      # nothing to annihilate (real alpha)
            if cplx:
                x[0] = x[0].real
        v, tau, beta = oracle_mod.larfg(x)
        assert v[0] == 1
        H = np.eye(m) - tau * np.outer(v, np.conj(v))
        r = np.conj(H.T) @ x
        e1 = np.zeros(m); e1[0] = 1
        assert np.linalg.norm(r - beta * e1) <= 8 * EPS * np.linalg.norm(x)
        assert np.linalg.norm(np.conj(H.T) @ H - np.eye(m)) <= 16 * EPS * m
        if tau != 0:
            if cplx:
                assert 1 - 1e-14 <= tau.real <= 2 + 1e-14 and abs(tau - 1) <= 1 + 1e-14
            else:
                assert 1 - 1e-14 <= tau <= 2 + 1e-14
        assert abs(abs(beta) - np.linalg.norm(x)) <= 8 * EPS * np.linalg.norm(x)


# ---------------------------------------------------------------- QL
@pytest.mark.parametrize("n", [1, 2, 3, 10, 100, 257])
def test_ql_toeplitz_closed_form(oracle_mod, n):
    a, b = 0.7, -1.3
    w, X = oracle_mod.tridiagonal_eigh(np.full(n, a), np.full(n - 1, b))
    k = np.arange(1, n + 1)
    lam = np.sort(a + 2 * b * np.cos(k * np.pi / (n + 1)))
    assert np.max(np.abs(w - lam)) <= 64 * EPS * (abs(a) + 2 * abs(b)) * max(n, 1) ** 0.5
    # eigenvector of lambda_k is proportional to sin(j k pi / (n+1))
    for kk in [1, n // 2 + 1, n]:
        lam_k = a + 2 * b * np.cos(kk * np.pi / (n + 1))
        i = int(np.argmin(np.abs(w - lam_k)))
        u = np.sin(np.arange(1, n + 1) * kk * np.pi / (n + 1))
        u /= np.linalg.norm(u)
        assert abs(abs(u @ X[:, i]) - 1) <= 1e-10
    assert np.linalg.norm(X.T @ X - np.eye(n)) <= 64 * EPS * n


def test_ql_vs_jacobi_and_lapack(oracle_mod):
    rng = np.random.default_rng(7)
    for n in [5, 17, 64]:
        d, e = rng.standard_normal(n), rng.standard_normal(n - 1)
        w, X = oracle_mod.tridiagonal_eigh(d, e)
        T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
        wj, Vj = oracle_mod.jacobi_eigh(T)
        wl = sl.eigh_tridiagonal(d, e, eigvals_only=True)
        assert np.max(np.abs(w - wj)) <= 1e-13 * np.abs(w).max()
        assert np.max(np.abs(w - wl)) <= 1e-13 * np.abs(w).max()
        assert np.linalg.norm(T @ X - X * w) <= 1e-13 * n * np.linalg.norm(T)
        # eigenvectors agree with Jacobi's up to sign (spectrum is simple)
        s = np.sign(np.sum(X * Vj, axis=0))
        assert np.max(np.abs(X - Vj * s)) <= 1e-9


def test_ql_with_zero_subdiagonal_splits(oracle_mod):
    d = np.array([3.0, 1.0, 2.0, -1.0, 5.0])
    e = np.array([0.5, 0.0, 0.25, 0.0])
    w, X = oracle_mod.tridiagonal_eigh(d, e)
    T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    assert np.allclose(w, np.linalg.eigvalsh(T), atol=1e-14, rtol=0)
    assert np.linalg.norm(T @ X - X * w) <= 1e-14 * 10


# ---------------------------------------------------------------- Jacobi
def test_jacobi_2x2_closed_form(oracle_mod):
    a, b, c = 2.0, 0.75, -1.0
    w, V = oracle_mod.jacobi_eigh(np.array([[a, b], [b, c]]))
    m, r = (a + c) / 2, np.hypot((a - c) / 2, b)
    assert np.allclose(w, [m - r, m + r], atol=1e-15, rtol=0)


def test_jacobi_vs_lapack(oracle_mod):
    rng = np.random.default_rng(3)
    A = rng.standard_normal((40, 40)); A = A + A.T
    w, V = oracle_mod.jacobi_eigh(A)
    assert np.max(np.abs(w - np.linalg.eigvalsh(A))) <= 1e-13 * np.abs(w).max()
    assert np.linalg.norm(A @ V - V * w) <= 1e-12 * np.linalg.norm(A)


# ---------------------------------------------------------------- bulge chase
@pytest.mark.parametrize("dtype", ["d", "z"])
@pytest.mark.parametrize("n,b", [(17, 4), (64, 8), (130, 16), (97, 3), (40, 39), (6, 2)])
def test_chase_preserves_spectrum_and_reconstructs(oracle_mod, dtype, n, b):
    ab = synth.band_matrix(n, b, 100 + n + b, dtype)
    r = oracle_mod.band_to_tridiagonal(ab, b)
    assert r["dropped"] == 0.0                  # fill stays within 2b subdiagonals
    nrm = np.linalg.norm(synth.dense_from_band(ab))
    assert r["offband"] <= 1e-14 * nrm
    ev_lapack = sl.eig_banded(ab, lower=True, eigvals_only=True)
    T = np.diag(r["d"]).astype(complex) + np.diag(r["e"], -1) + np.diag(np.conj(r["e"]), 1)
    assert np.max(np.abs(np.linalg.eigvalsh(T) - ev_lapack)) <= 1e-13 * nrm
    # B = Y T Y^H with Y = back-transform of the identity (Q^* of Eq. 2stage_bkwd1)
    Y = oracle_mod.back_transform(np.eye(n), r["hh_v"], r["hh_tau"], b)
    B = synth.dense_from_band(ab)
    assert np.linalg.norm(B - Y @ T @ np.conj(Y.T)) <= 1e-13 * nrm
    if dtype == "z":
        # every annihilated column gets a real beta: only e[n-2] stays complex
        assert np.max(np.abs(r["e"][:-1].imag)) == 0.0


def test_chase_on_tridiagonal_input_is_identity(oracle_mod):
    n, b = 40, 6
    ab = np.zeros((b + 1, n))
    rng = np.random.default_rng(1)
    ab[0] = rng.standard_normal(n)
    ab[1, : n - 1] = rng.standard_normal(n - 1)
    r = oracle_mod.band_to_tridiagonal(ab, b)
    assert np.all(r["hh_tau"] == 0)
    Z = rng.standard_normal((n, 5))
    Y = oracle_mod.back_transform(Z, r["hh_v"], r["hh_tau"], b)
    assert np.array_equal(Y, Z)
    assert np.array_equal(r["d"], ab[0]) and np.array_equal(r["e"], ab[1, : n - 1])


# ---------------------------------------------------------------- back-transform
def _dense_product(n, b, V, tau, table):
    """Q^* = H_0 H_1 ... H_{K-1} from explicit n x n reflector matrices."""
    st, sl_, r0, ln = table
    Q = np.eye(n, dtype=np.result_type(V, tau))
    for k in range(len(tau)):
        H = np.eye(n, dtype=Q.dtype)
        v = np.zeros(n, Q.dtype)
        v[r0[k]: r0[k] + ln[k]] = V[k, : ln[k]]
        H -= tau[k] * np.outer(v, np.conj(v))
        Q = Q @ H
    return Q


@pytest.mark.parametrize("dtype", ["d", "z"])
@pytest.mark.parametrize("n,b", [(17, 4), (40, 8), (23, 5)])
def test_back_transform_equals_dense_product(oracle_mod, dtype, n, b):
    table = oracle_mod.reflector_table(n, b)
    V, tau = synth.unitary_reflectors(table[3], b, 11, dtype)
    Z = synth.gaussian(n, 7, 12, dtype)
    Y = oracle_mod.back_transform(Z, V, tau, b)
    Q = _dense_product(n, b, V, tau, table)
    assert np.linalg.norm(Y - Q @ Z) <= 1e-14 * np.linalg.norm(Z) * n


@pytest.mark.parametrize("dtype", ["d", "z"])
def test_back_transform_unitary_invariants_and_inverse(oracle_mod, dtype):
    n, b = 300, 16
    table = oracle_mod.reflector_table(n, b)
    V, tau = synth.unitary_reflectors(table[3], b, 21, dtype)
    Z = synth.gaussian(n, 9, 22, dtype)
    Y = oracle_mod.back_transform(Z, V, tau, b)
    G0, G1 = np.conj(Z.T) @ Z, np.conj(Y.T) @ Y
    assert np.linalg.norm(G1 - G0) <= 1e-13 * np.linalg.norm(G0)
    Zb = oracle_mod.apply_q(Y, V, tau, b)
    assert np.linalg.norm(Zb - Z) <= 1e-13 * np.linalg.norm(Z)
    # column subset equals the full computation, bit for bit
    Ys = oracle_mod.back_transform(Z, V, tau, b, cols=[0, 4, 8])
    assert np.array_equal(Ys, Y[:, [0, 4, 8]])


def test_back_transform_is_linear(oracle_mod):
    n, b = 90, 8
    table = oracle_mod.reflector_table(n, b)
    V, tau = synth.unitary_reflectors(table[3], b, 31, "z")
    A, B = synth.gaussian(n, 3, 1, "z"), synth.gaussian(n, 3, 2, "z")
    a = 0.3 - 1.7j
    lhs = oracle_mod.back_transform(A + a * B, V, tau, b)
    rhs = oracle_mod.back_transform(A, V, tau, b) + a * oracle_mod.back_transform(B, V, tau, b)
    assert np.linalg.norm(lhs - rhs) <= 1e-13 * np.linalg.norm(lhs)


# ---------------------------------------------------------------- end to end
@pytest.mark.parametrize("dtype", ["d", "z"])
def test_stage2_pipeline_eigenpairs(oracle_mod, dtype):
    n, b, nev = 256, 16, 128
    ab = synth.band_matrix(n, b, 55, dtype, diag_shift=True)
    p = oracle_mod.stage2_pipeline(ab, b, nev)
    B = synth.dense_from_band(ab)
    Y = oracle_mod.back_transform(p["Z_in"], p["hh_v"], p["hh_tau"], b)
    nrm = np.linalg.norm(B)
    assert np.linalg.norm(B @ Y - Y * p["w"]) / nrm <= 1e-12 * n
    assert np.linalg.norm(np.conj(Y.T) @ Y - np.eye(nev)) <= 1e-12 * n
    w_lapack = sl.eig_banded(ab, lower=True, eigvals_only=True)[:nev]
    assert np.max(np.abs(p["w"] - w_lapack)) <= 1e-12 * nrm


def test_long_double_error_estimate(oracle_mod):
    """The oracle's own rounding error, measured against an extended
    precision (numpy longdouble) replay of the same reflector sequence."""
    n, b = 200, 16
    table = oracle_mod.reflector_table(n, b)
    V, tau = synth.unitary_reflectors(table[3], b, 41, "d")
    Z = synth.gaussian(n, 4, 42, "d")
    Y = oracle_mod.back_transform(Z, V, tau, b)
    L = Z.astype(np.longdouble)
    st, sl_, r0, ln = table
    Vl, tl = V.astype(np.longdouble), tau.astype(np.longdouble)
    for k in range(len(tau) - 1, -1, -1):
        v = Vl[k, : ln[k]]
        seg = L[r0[k]: r0[k] + ln[k]]
        seg -= tl[k] * np.outer(v, v @ seg)
    err = np.linalg.norm((Y - L).astype(np.float64)) / np.linalg.norm(Z)
    assert err <= 1e-14
