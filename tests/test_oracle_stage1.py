"""Pins of the oracle's stage-1 pair: the full-to-band reduction B = P A P^*
(Sec. 2.1, Eq. 2stage_fwd1) and the band-to-full back-transformation
C = P^* Y (Eq. 2stage_bkwd2), against things other than the oracle itself:

* brute force with explicit n x n reflector matrices: P^* = H_0 ... H_{J-1}
  built densely from the stored (v, tau); the oracle's back-transformation
  equals P^* Y and its reduction equals P A P^* (both as dense products);
* LAPACK: the eigenvalues of B equal those of A;
* the band structure (exact zeros outside the band; complex: the entry
  left in each annihilated column is a real beta);
* an already banded real input: every tau is 0 and B = A bitwise;
* the whole two-stage pipeline: full -> band -> tridiagonal -> eigenpairs
  -> Eq. 2stage_bkwd1 -> Eq. 2stage_bkwd2 gives eigenvectors of A.
"""
import numpy as np
import pytest


def _dense_p_star(V, tau, nbw):
    n, J = V.shape
    P = np.eye(n, dtype=np.result_type(V, tau))
    for j in range(J):          # P^* = H_0 H_1 ... H_{J-1}
        v = np.zeros(n, P.dtype)
        v[j + nbw:] = V[j + nbw:, j]
        H = np.eye(n, dtype=P.dtype) - tau[j] * np.outer(v, v.conj())
        P = P @ H
    return P


@pytest.mark.parametrize("dtype", ["d", "z"])
@pytest.mark.parametrize("n,nbw", [(2, 1), (5, 1), (17, 4), (30, 3), (40, 8), (48, 16), (20, 19)])
def test_brute_force_dense_products(oracle_mod, dtype, n, nbw):
    import synth
    A = synth.hermitian_matrix(n, 100 + n, dtype)
    r = oracle_mod.full_to_band(A, nbw)
    V, tau, B = r["hh_v"], r["hh_tau"], r["B"]
    assert V.shape == (n, max(n - nbw - 1, 0)) and len(tau) == V.shape[1]
    Ps = _dense_p_star(V, tau, nbw)
    # reduction: B = P A P^* with P = (P^*)^H
    nrm = np.linalg.norm(A)
    assert np.linalg.norm(Ps.conj().T @ A @ Ps - B) <= 1e-13 * nrm
    # back-transformation: the dense product
    Y = synth.gaussian(n, 7, 5, dtype)
    C = oracle_mod.back_transform_full(Y, V, tau, nbw)
    assert np.linalg.norm(C - Ps @ Y) <= 1e-13 * np.linalg.norm(Y)
    # P^* is unitary; v_j[0] = 1 at row j+nbw, nothing above it
    assert np.linalg.norm(Ps.conj().T @ Ps - np.eye(n)) <= 1e-13 * n
    for j in range(V.shape[1]):
        assert V[j + nbw, j] == 1.0 and np.all(V[: j + nbw, j] == 0)


@pytest.mark.parametrize("dtype", ["d", "z"])
@pytest.mark.parametrize("n,nbw", [(300, 16), (257, 32), (200, 64)])
def test_band_structure_and_eigenvalues(oracle_mod, dtype, n, nbw):
    import synth
    A = synth.hermitian_matrix(n, n + nbw, dtype)
    r = oracle_mod.full_to_band(A, nbw)
    B = r["B"]
    i, j = np.indices(B.shape)
    assert np.all(B[np.abs(i - j) > nbw] == 0)
    assert np.linalg.norm(B - B.conj().T) <= 1e-14 * n * np.linalg.norm(A)
    la, lb = np.linalg.eigvalsh(A), np.linalg.eigvalsh((B + B.conj().T) / 2)
    assert np.max(np.abs(la - lb)) <= 1e-13 * np.max(np.abs(la)) * np.sqrt(n)
    # complex: the last subdiagonal of each annihilated column is a real beta
    if dtype == "z":
        J = r["hh_v"].shape[1]
        assert np.all(np.diagonal(B, -nbw)[:J].imag == 0)
    if n <= 200:   # B = P A P^* as a dense product
        Ps = _dense_p_star(r["hh_v"], r["hh_tau"], nbw)
        assert np.linalg.norm(Ps.conj().T @ A @ Ps - B) <= 1e-13 * np.linalg.norm(A) * n


def test_banded_real_input_is_left_alone(oracle_mod):
    import synth
    n, nbw = 60, 5
    A = synth.hermitian_matrix(n, 9, "d")
    i, j = np.indices(A.shape)
    A[np.abs(i - j) > nbw] = 0.0
    r = oracle_mod.full_to_band(A, nbw)
    assert np.all(r["hh_tau"] == 0.0)
    assert np.array_equal(r["B"], A)
    Y = synth.gaussian(n, 4, 1, "d")
    assert np.array_equal(oracle_mod.back_transform_full(Y, r["hh_v"], r["hh_tau"], nbw), Y)


@pytest.mark.parametrize("dtype", ["d", "z"])
def test_two_stage_pipeline_eigenvectors(oracle_mod, dtype):
    """Eq. 2stage end to end on the oracle: A -> B -> T -> (Lambda, X) ->
    Y = Q^* X -> C = P^* Y; C holds eigenvectors of A."""
    import synth
    n, nbw, nev = 200, 16, 60
    A = synth.hermitian_matrix(n, 77, dtype)
    r = oracle_mod.full_to_band(A, nbw)
    B = r["B"]
    ab = np.zeros((nbw + 1, n), B.dtype)
    for d in range(nbw + 1):
        ab[d, : n - d] = np.diagonal(B, -d)
    p = oracle_mod.stage2_pipeline(ab, nbw, nev)
    Y = oracle_mod.back_transform(p["Z_in"], p["hh_v"], p["hh_tau"], nbw)
    C = oracle_mod.back_transform_full(Y, r["hh_v"], r["hh_tau"], nbw)
    la = np.linalg.eigvalsh(A)[:nev]
    nrm = np.linalg.norm(A)
    assert np.max(np.abs(p["w"] - la)) <= 1e-13 * nrm
    assert np.linalg.norm(A @ C - C * p["w"]) / nrm <= 1e-12 * n
    assert np.linalg.norm(C.conj().T @ C - np.eye(nev)) <= 1e-12 * n
    # tighter than the stated bound: the measured level
    assert np.linalg.norm(A @ C - C * p["w"]) / nrm <= 1e-13


def test_back_transform_column_subsets_and_norms(oracle_mod):
    import synth
    n, nbw = 130, 8
    V, tau = synth.full_unitary_reflectors(n, nbw, 3, "z")
    Y = synth.gaussian(n, 20, 4, "z")
    C = oracle_mod.back_transform_full(Y, V, tau, nbw)
    Cs = oracle_mod.back_transform_full(Y, V, tau, nbw, cols=[3, 11, 19])
    assert np.array_equal(C[:, [3, 11, 19]], Cs)
    # synthetic reflectors are unitary: column norms are preserved
    assert np.allclose(np.linalg.norm(C, axis=0), np.linalg.norm(Y, axis=0), rtol=1e-13)
    Ps = _dense_p_star(V, tau, nbw)
    assert np.linalg.norm(C - Ps @ Y) <= 1e-13 * np.linalg.norm(Y)
