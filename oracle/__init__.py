"""CPU FP64 oracle for the tridiagonal-to-banded eigenvector back-transformation.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark import this package; the product library
neither links nor calls it, and it shares no code with the GPU path.

The arithmetic lives in ``oracle.c`` (plain C, built with gcc); this module is
argument marshalling plus the two small pipeline steps that are pure
bookkeeping (the complex phase fix of the last subdiagonal and column
selection).  Every routine cites the passage of Yu et al. (CPC, 2020,
"GPU-Acceleration of the ELPA2 Distributed Eigensolver") it follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64 = C.c_int64
_dp = C.POINTER(C.c_double)
_i64p = C.POINTER(C.c_int64)


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (plain -O2, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-std=gnu11", "-shared", "-fPIC",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        # ORACLE_LIB: a prebuilt copy of oracle.c (the sanitizer test builds
        # one with AddressSanitizer); default: build liboracle.so here
        path = os.environ.get("ORACLE_LIB")
        if not path:
            path = build()
        L = C.CDLL(path)
        L.orc_sweeps_in_stage.restype = _i64
        L.orc_sweeps_in_stage.argtypes = [_i64, _i64, _i64]
        L.orc_num_reflectors.restype = _i64
        L.orc_num_reflectors.argtypes = [_i64, _i64]
        L.orc_reflector_table.argtypes = [_i64, _i64, _i64p, _i64p, _i64p, _i64p]
        L.orc_larfg_d.argtypes = [_i64, _dp, _dp, _dp]
        L.orc_larfg_z.argtypes = [_i64, C.c_void_p, C.c_void_p, _dp]
        L.orc_band_to_tridi_d.argtypes = [_i64, _i64, _dp, _i64, _dp, _dp, _dp, _dp, _dp, _dp]
        L.orc_band_to_tridi_z.argtypes = [_i64, _i64, C.c_void_p, _i64, _dp, C.c_void_p,
                                          C.c_void_p, C.c_void_p, _dp, _dp]
        L.orc_back_transform_d.argtypes = [_i64, _i64, _i64, _i64, _dp, _dp, _dp, _i64]
        L.orc_back_transform_z.argtypes = [_i64, _i64, _i64, _i64, C.c_void_p, C.c_void_p,
                                           C.c_void_p, _i64]
        L.orc_apply_q_z.argtypes = [_i64, _i64, _i64, _i64, C.c_void_p, C.c_void_p,
                                    C.c_void_p, _i64]
        L.orc_adjoint_d.argtypes = [_i64, _i64, _i64, _dp, _dp, _dp, _i64, _dp, _i64, _dp, _dp]
        L.orc_adjoint_z.argtypes = [_i64, _i64, _i64, C.c_void_p, C.c_void_p, C.c_void_p, _i64,
                                    C.c_void_p, _i64, C.c_void_p, C.c_void_p]
        L.orc_tridi_ql.argtypes = [_i64, _dp, _dp, _dp, _i64]
        L.orc_jacobi_d.argtypes = [_i64, _dp, _dp, _dp]
        L.orc_num_threads.restype = C.c_int
        L.orc_full_reflectors.restype = _i64
        L.orc_full_reflectors.argtypes = [_i64, _i64]
        L.orc_full_to_band_d.argtypes = [_i64, _i64, _dp, _i64, _dp, _i64, _dp]
        L.orc_full_to_band_z.argtypes = [_i64, _i64, C.c_void_p, _i64, C.c_void_p, _i64,
                                         C.c_void_p]
        L.orc_back_transform_full_d.argtypes = [_i64, _i64, _i64, _i64, _dp, _i64, _dp, _dp,
                                                _i64]
        L.orc_back_transform_full_z.argtypes = [_i64, _i64, _i64, _i64, C.c_void_p, _i64,
                                                C.c_void_p, C.c_void_p, _i64]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _v(a: np.ndarray):
    return C.c_void_p(a.ctypes.data)


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")


def num_threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(lib().orc_num_threads())


# --------------------------------------------------------------------------
# Reflector geometry (Sec. 2.2.1)
# --------------------------------------------------------------------------
def sweeps_in_stage(n: int, nbw: int, s: int) -> int:
    """Sweeps of 0-based stage s (paper stage i = s+1): ceil((n-s-2)/nbw)."""
    return int(lib().orc_sweeps_in_stage(n, nbw, s))


def num_reflectors(n: int, nbw: int) -> int:
    return int(lib().orc_num_reflectors(n, nbw))


def reflector_table(n: int, nbw: int):
    """(stage, slot, row0, length) of every reflector in generation order."""
    K = num_reflectors(n, nbw)
    out = [np.zeros(K, np.int64) for _ in range(4)]
    _check(lib().orc_reflector_table(n, nbw, *[o.ctypes.data_as(_i64p) for o in out]),
           "reflector_table")
    return tuple(out)


# --------------------------------------------------------------------------
# Householder generation (Eq. householder, standard method)
# --------------------------------------------------------------------------
def larfg(x: np.ndarray):
    """Return (v, tau, beta) with (I - tau v v^H)^H x = beta e1, v[0] = 1."""
    x = np.array(x, copy=True)
    beta = C.c_double()
    if np.iscomplexobj(x):
        x = x.astype(np.complex128)
        tau = np.zeros(1, np.complex128)
        lib().orc_larfg_z(len(x), _v(x), _v(tau), C.byref(beta))
        return x, complex(tau[0]), beta.value
    x = x.astype(np.float64)
    tau = C.c_double()
    lib().orc_larfg_d(len(x), _p(x), C.byref(tau), C.byref(beta))
    return x, tau.value, beta.value


# --------------------------------------------------------------------------
# Banded -> tridiagonal bulge chasing (Sec. 2.2.1, Eq. 2stage_fwd2)
# --------------------------------------------------------------------------
def band_to_tridiagonal(ab: np.ndarray, nbw: int):
    """Reduce a Hermitian band matrix to tridiagonal form, storing reflectors.

    ab: LAPACK lower band layout, shape (nbw+1, n): ab[d, k] = B[k+d, k].
    Returns dict(d, e, hh_v (K x nbw), hh_tau (K,), offband, dropped).
    """
    n = ab.shape[1]
    K = num_reflectors(n, nbw)
    cplx = np.iscomplexobj(ab)
    dt = np.complex128 if cplx else np.float64
    abf = np.asfortranarray(ab.astype(dt))
    d = np.zeros(n)
    e = np.zeros(max(n - 1, 1), dt)
    hv = np.zeros((max(K, 1), nbw), dt)
    ht = np.zeros(max(K, 1), dt)
    off, drop = C.c_double(), C.c_double()
    if cplx:
        rc = lib().orc_band_to_tridi_z(n, nbw, _v(abf), abf.shape[0], _p(d), _v(e), _v(hv),
                                       _v(ht), C.byref(off), C.byref(drop))
    else:
        rc = lib().orc_band_to_tridi_d(n, nbw, _p(abf), abf.shape[0], _p(d), _p(e), _p(hv),
                                       _p(ht), C.byref(off), C.byref(drop))
    _check(rc, "band_to_tridi")
    return dict(d=d, e=e[: max(n - 1, 0)], hh_v=hv[:K], hh_tau=ht[:K],
                offband=off.value, dropped=drop.value)


# --------------------------------------------------------------------------
# Tridiagonal -> banded back-transformation (Sec. 2.2.2, Eq. 2stage_bkwd1)
# --------------------------------------------------------------------------
def back_transform(Z: np.ndarray, hh_v: np.ndarray, hh_tau: np.ndarray, nbw: int,
                   cols=None) -> np.ndarray:
    """Y = Q^* X: apply every reflector, in reverse generation order, one at a
    time, to the columns of Z (Eq. kernel).  Z is (n, nev); a Fortran-ordered
    copy is returned.  ``cols`` restricts the work to a subset of columns
    (columns are independent, Sec. 2.2.2); the result then has only those."""
    Z = np.asarray(Z)
    cplx = np.iscomplexobj(Z) or np.iscomplexobj(hh_v)
    dt = np.complex128 if cplx else np.float64
    if cols is not None:
        Z = Z[:, np.asarray(cols)]
    Y = np.array(Z, dtype=dt, order="F", copy=True)
    n, nev = Y.shape
    hv = np.ascontiguousarray(hh_v, dtype=dt)
    ht = np.ascontiguousarray(hh_tau, dtype=dt)
    if hv.size == 0:
        hv = np.zeros((1, nbw), dt)
        ht = np.zeros(1, dt)
    ld = max(n, 1)
    if cplx:
        rc = lib().orc_back_transform_z(n, nbw, 0, nev, _v(hv), _v(ht), _v(Y), ld)
    else:
        rc = lib().orc_back_transform_d(n, nbw, 0, nev, _p(hv), _p(ht), _p(Y), ld)
    _check(rc, "back_transform")
    return Y


def apply_q(Z: np.ndarray, hh_v, hh_tau, nbw: int) -> np.ndarray:
    """Z <- Q Z (the reflectors conjugate-transposed, in generation order)."""
    Y = np.array(Z, dtype=np.complex128, order="F", copy=True)
    n, nev = Y.shape
    hv = np.ascontiguousarray(hh_v, dtype=np.complex128)
    ht = np.ascontiguousarray(hh_tau, dtype=np.complex128)
    _check(lib().orc_apply_q_z(n, nbw, 0, nev, _v(hv), _v(ht), _v(Y), max(n, 1)), "apply_q")
    return Y if np.iscomplexobj(Z) else Y.real.copy(order="F")


def adjoint(Z_in: np.ndarray, G: np.ndarray, hh_v: np.ndarray, hh_tau: np.ndarray, nbw: int):
    """Reverse-mode derivative of the back-transformation
    Z_out = H_0 ... H_{K-1} Z_in (Eq. 2stage_bkwd1).
    G = dL/dZ_out (n, nev).  Returns (dL/dZ_in, dL/dv (K, nbw), dL/dtau (K,)).
    Complex inputs: conjugate-Wirtinger gradients (PyTorch's convention,
    dL = Re sum conj(grad) dx)."""
    if any(np.iscomplexobj(a) for a in (Z_in, G, hh_v, hh_tau)):
        return _adjoint_z(Z_in, G, hh_v, hh_tau, nbw)
    Zi = np.array(Z_in, dtype=np.float64, order="F", copy=True)
    Gi = np.array(G, dtype=np.float64, order="F", copy=True)
    n, nev = Zi.shape
    K = num_reflectors(n, nbw)
    hv = np.ascontiguousarray(hh_v, dtype=np.float64)
    ht = np.ascontiguousarray(hh_tau, dtype=np.float64)
    if hv.size == 0:
        hv = np.zeros((1, nbw))
        ht = np.zeros(1)
    dv = np.zeros((max(K, 1), nbw))
    dt = np.zeros(max(K, 1))
    ld = max(n, 1)
    _check(lib().orc_adjoint_d(n, nbw, nev, _p(hv), _p(ht), _p(Zi), ld, _p(Gi), ld, _p(dv),
                               _p(dt)), "adjoint")
    return Gi, dv[:K], dt[:K]


def _adjoint_z(Z_in, G, hh_v, hh_tau, nbw: int):
    Zi = np.array(Z_in, dtype=np.complex128, order="F", copy=True)
    Gi = np.array(G, dtype=np.complex128, order="F", copy=True)
    n, nev = Zi.shape
    K = num_reflectors(n, nbw)
    hv = np.ascontiguousarray(hh_v, dtype=np.complex128)
    ht = np.ascontiguousarray(hh_tau, dtype=np.complex128)
    if hv.size == 0:
        hv = np.zeros((1, nbw), np.complex128)
        ht = np.zeros(1, np.complex128)
    dv = np.zeros((max(K, 1), nbw), np.complex128)
    dt = np.zeros(max(K, 1), np.complex128)
    ld = max(n, 1)
    _check(lib().orc_adjoint_z(n, nbw, nev, _v(hv), _v(ht), _v(Zi), ld, _v(Gi), ld, _v(dv),
                               _v(dt)), "adjoint_z")
    return Gi, dv[:K], dt[:K]


# --------------------------------------------------------------------------
# Tridiagonal eigensolver (Eq. 2stage_solve) and brute force
# --------------------------------------------------------------------------
def tridiagonal_eigh(d: np.ndarray, e: np.ndarray):
    """Implicit QL with Wilkinson shift: eigenvalues ascending and
    orthonormal eigenvectors (columns) of the real symmetric tridiagonal T."""
    n = len(d)
    w = np.array(d, dtype=np.float64, copy=True)
    ee = np.zeros(max(n, 1))
    ee[: n - 1] = e
    X = np.zeros((n, n), order="F")
    _check(lib().orc_tridi_ql(n, _p(w), _p(ee), _p(X), n), "tridi_ql")
    return w, X


def jacobi_eigh(A: np.ndarray):
    """Cyclic Jacobi on a small real symmetric matrix (brute force)."""
    A = np.array(A, dtype=np.float64, order="F", copy=True)
    n = A.shape[0]
    w = np.zeros(n)
    V = np.zeros((n, n), order="F")
    _check(lib().orc_jacobi_d(n, _p(A), _p(w), _p(V)), "jacobi")
    return w, V


# --------------------------------------------------------------------------
# Stage-2 pipeline producing the back-transformation inputs
# --------------------------------------------------------------------------
def phase_fix(e: np.ndarray):
    """T from the complex chase is real except its last subdiagonal e[n-2]
    (every annihilated column gets a real beta).  With phi = arg e[n-2],
    T = D T_r D^H, D = diag(1, ..., 1, exp(i phi)), T_r real.  Returns
    (e_real, phase) so that the eigenvectors of T are D X_r."""
    e = np.asarray(e)
    if not np.iscomplexobj(e) or len(e) == 0:
        return np.asarray(e, dtype=np.float64).real.copy(), 1.0
    er = e.real.copy()
    last = e[-1]
    ph = last / abs(last) if abs(last) > 0 else 1.0 + 0j
    er[-1] = abs(last)
    # the other subdiagonals are real up to rounding of the similarity updates
    return er, ph


def stage2_pipeline(ab: np.ndarray, nbw: int, nev: int | None = None):
    """Band matrix -> (reflectors, tridiagonal eigenpairs, Z_in = X[:, :nev]).

    Follows Eq. 2stage_fwd2 (bulge chasing), Eq. 2stage_solve (tridiagonal
    eigensolver, lowest nev eigenpairs) and prepares X for Eq. 2stage_bkwd1.
    """
    n = ab.shape[1]
    nev = n if nev is None else nev
    r = band_to_tridiagonal(ab, nbw)
    er, ph = phase_fix(r["e"])
    w, X = tridiagonal_eigh(r["d"], er)
    Zin = X[:, :nev]
    if np.iscomplexobj(ab):
        Zin = Zin.astype(np.complex128)
        Zin[-1, :] *= ph
    r.update(w=w[:nev], Z_in=np.asfortranarray(Zin))
    return r


# --------------------------------------------------------------------------
# Stage 1: full -> band reduction (Eq. 2stage_fwd1) and its back-transformation
# (Eq. 2stage_bkwd2)
# --------------------------------------------------------------------------
def full_reflectors(n: int, nbw: int) -> int:
    """Number of stage-1 reflectors: one per column j = 0 .. n-nbw-2."""
    return int(lib().orc_full_reflectors(n, nbw))


def full_to_band(A: np.ndarray, nbw: int):
    """B = P A P^* for a dense Hermitian A (both triangles), one Householder
    reflector per column.  Returns dict(B (n, n), hh_v (n, J) with reflector
    j in rows [j+nbw, n) of column j, hh_tau (J,))."""
    cplx = np.iscomplexobj(A)
    dt = np.complex128 if cplx else np.float64
    B = np.array(A, dtype=dt, order="F", copy=True)
    n = B.shape[0]
    J = full_reflectors(n, nbw)
    V = np.zeros((max(n, 1), max(J, 1)), dt, order="F")
    tau = np.zeros(max(J, 1), dt)
    ld = max(n, 1)
    if cplx:
        rc = lib().orc_full_to_band_z(n, nbw, _v(B), ld, _v(V), ld, _v(tau))
    else:
        rc = lib().orc_full_to_band_d(n, nbw, _p(B), ld, _p(V), ld, _p(tau))
    _check(rc, "full_to_band")
    return dict(B=B, hh_v=V[:n, :J], hh_tau=tau[:J])


def back_transform_full(Z: np.ndarray, hh_v: np.ndarray, hh_tau: np.ndarray, nbw: int,
                        cols=None) -> np.ndarray:
    """C = P^* Y: every stage-1 reflector, in reverse generation order, one
    at a time, applied to the columns of Z (n, nev).  hh_v is (n, J) with
    reflector j in rows [j+nbw, n) of column j.  Returns a Fortran copy;
    ``cols`` restricts the work to those columns."""
    Z = np.asarray(Z)
    cplx = np.iscomplexobj(Z) or np.iscomplexobj(hh_v)
    dt = np.complex128 if cplx else np.float64
    if cols is not None:
        Z = Z[:, np.asarray(cols)]
    Y = np.array(Z, dtype=dt, order="F", copy=True)
    n, nev = Y.shape
    J = full_reflectors(n, nbw)
    V = np.asfortranarray(hh_v, dtype=dt)
    t = np.ascontiguousarray(hh_tau, dtype=dt)
    if J == 0:
        return Y
    if V.shape != (n, J) or t.shape != (J,):
        raise ValueError(f"hh_v must be ({n}, {J}) and hh_tau ({J},)")
    ld = max(n, 1)
    if cplx:
        rc = lib().orc_back_transform_full_z(n, nbw, 0, nev, _v(V), ld, _v(t), _v(Y), ld)
    else:
        rc = lib().orc_back_transform_full_d(n, nbw, 0, nev, _p(V), ld, _p(t), _p(Y), ld)
    _check(rc, "back_transform_full")
    return Y
