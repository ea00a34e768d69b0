"""Seeded synthetic inputs for the tridiagonal-to-banded back-transformation.

This module only draws random numbers in fixed, documented orders; it holds
none of the method's arithmetic.  Both the GPU tests/benchmark and the CPU
oracle take their inputs from here.  The reflector generator needs the
number of valid entries of every stored reflector; ``reflector_lengths``
states that input format (tests check it against the oracle and the
library).

Workloads (the paper's inputs are dense random Hermitian matrices and
materials Hamiltonians whose back-transformation sees only (v, tau, X); these
shapes stand in for them):

  C1  real, n=1024,  nbw=32, nev=1024  band N(0,1)               seed 1001
  C2  real, n=8192,  nbw=64, nev=4096  band N(0,1) + diag 4i/n   seed 1002
  C3  complex, n=32768, nbw=64, nev=8192  band N(0,1/2)+iN(0,1/2),
      real diagonal N(0,1)                                       seed 1003
  C4  64 real problems, n_p = 512*U{1..8}, nbw=32, nev=n_p/2      seed 1004
  C5  real adjoint, n=4096, nbw=64, nev=2048, G ~ N(0,1)          seed 1005
  FD  real, n=64, nbw=8, nev=16                                   seed 3005
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

CONFIGS = {
    "C1": dict(n=1024, nbw=32, nev=1024, dtype="d", seed=1001, diag_shift=False),
    "C2": dict(n=8192, nbw=64, nev=4096, dtype="d", seed=1002, diag_shift=True),
    "C3": dict(n=32768, nbw=64, nev=8192, dtype="z", seed=1003, diag_shift=False),
    "C5": dict(n=4096, nbw=64, nev=2048, dtype="d", seed=1005, diag_shift=False),
    "FD": dict(n=64, nbw=8, nev=16, dtype="d", seed=3005, diag_shift=False),
}

# Fixed chunk sizes: element (r, c) of a Gaussian matrix depends only on
# (seed, c // GAUSS_COLS_PER_CHUNK), and reflector k only on
# (seed, k // REFL_PER_CHUNK), so any column or reflector subset can be
# regenerated without drawing the rest.
GAUSS_COLS_PER_CHUNK = 64
REFL_PER_CHUNK = 4096


def _np_dtype(dtype: str):
    return np.complex128 if dtype == "z" else np.float64


def _workers() -> int:
    return max(1, min(16, len(os.sched_getaffinity(0))))


def _parallel(fn, items):
    """Run fn over independent chunks (each has its own seed, so the result
    does not depend on the number of threads)."""
    items = list(items)
    if len(items) <= 1:
        for it in items:
            fn(it)
        return
    with ThreadPoolExecutor(_workers()) as ex:
        list(ex.map(fn, items))


def reflector_lengths(n: int, nbw: int) -> np.ndarray:
    """Input-format bookkeeping: the number of valid entries of each stored
    reflector, in storage order.  Stage s = 0..n-3 owns rows s+1..n-1, cut
    into consecutive pieces of nbw rows; a trailing piece of a single row
    carries no reflector (and nbw = 1 gives none at all)."""
    if n < 3 or nbw < 2:
        return np.zeros(0, np.int64)
    out = []
    for s in range(n - 2):
        rows = n - s - 1
        full, rest = divmod(rows, nbw)
        piece = [nbw] * full + ([rest] if rest >= 2 else [])
        out.append(np.array(piece, np.int64))
    return np.concatenate(out)


def band_matrix(n: int, nbw: int, seed: int, dtype: str = "d", diag_shift: bool = False):
    """Hermitian band matrix in LAPACK lower band layout ab[d, k] = B[k+d, k].

    Draw order (numpy default_rng(seed)):
      real:    standard_normal((nbw+1, n))
      complex: diagonal standard_normal(n) (real); then the real parts and
               then the imaginary parts of standard_normal((nbw, n)), both
               scaled by sqrt(1/2), so E|b_ij|^2 = 1.
    Entries that would fall below row n are zeroed.  diag_shift adds 4*i/n
    (0-based i) to the diagonal.
    """
    rng = np.random.default_rng(seed)
    if dtype == "z":
        ab = np.zeros((nbw + 1, n), np.complex128)
        ab[0] = rng.standard_normal(n)
        re = rng.standard_normal((nbw, n))
        im = rng.standard_normal((nbw, n))
        ab[1:] = np.sqrt(0.5) * (re + 1j * im)
    else:
        ab = rng.standard_normal((nbw + 1, n))
    for d in range(1, nbw + 1):
        ab[d, max(n - d, 0):] = 0
    if diag_shift:
        ab[0] = ab[0] + 4.0 * np.arange(n) / n
    return ab


def dense_from_band(ab: np.ndarray) -> np.ndarray:
    """Full Hermitian matrix from lower band storage (test helper)."""
    nb1, n = ab.shape
    B = np.zeros((n, n), ab.dtype)
    for d in range(nb1):
        idx = np.arange(n - d)
        B[idx + d, idx] = ab[d, : n - d]
        if d:
            B[idx, idx + d] = np.conj(ab[d, : n - d])
    return B


def gaussian(n: int, ncols: int, seed: int, dtype: str = "d", cols=None) -> np.ndarray:
    """(n, ncols) Fortran-ordered matrix of N(0,1) entries (complex: each part
    N(0,1/2)).  Columns are drawn in chunks of GAUSS_COLS_PER_CHUNK from
    SeedSequence(seed).spawn; ``cols`` returns only those columns."""
    cols = np.arange(ncols) if cols is None else np.asarray(cols)
    out = np.empty((n, len(cols)), _np_dtype(dtype), order="F")
    nchunk = (ncols + GAUSS_COLS_PER_CHUNK - 1) // GAUSS_COLS_PER_CHUNK
    seqs = np.random.SeedSequence(seed).spawn(max(nchunk, 1))
    need = {}
    for i, c in enumerate(cols):
        need.setdefault(int(c) // GAUSS_COLS_PER_CHUNK, []).append((i, int(c)))

    def fill(item):
        ch, items = item
        rng = np.random.default_rng(seqs[ch])
        w = min(GAUSS_COLS_PER_CHUNK, ncols - ch * GAUSS_COLS_PER_CHUNK)
        if dtype == "z":
            blk = rng.standard_normal((w, n)) + 1j * rng.standard_normal((w, n))
            blk *= np.sqrt(0.5)
        else:
            blk = rng.standard_normal((w, n))
        for i, c in items:
            out[:, i] = blk[c - ch * GAUSS_COLS_PER_CHUNK]

    _parallel(fill, need.items())
    return out


def unitary_reflectors(lengths: np.ndarray, nbw: int, seed: int, dtype: str = "d"):
    """Random unitary Householder reflectors H = I - tau v v^H with the shape
    of bulge-chasing output: v[0] = 1, v[1:len] ~ N(0, 1/len) (complex: each
    part N(0, 1/(2 len))), zero beyond len; tau = (1 - exp(i theta))/||v||^2
    with theta ~ U(pi/2, 3pi/2) (complex) or theta = pi, i.e. 2/||v||^2
    (real).  Any such tau makes H unitary; the range of theta mirrors the
    real part of a Householder tau lying in [1, 2]/||v||^2.

    Used where running the CPU bulge chase would take too long (n = 32768);
    the back-transformation's cost and numerics depend only on (v, tau, X).
    Reflector k depends only on (seed, k // REFL_PER_CHUNK).
    """
    lengths = np.asarray(lengths, np.int64)
    K = len(lengths)
    dt = _np_dtype(dtype)
    V = np.zeros((K, nbw), dt)
    tau = np.zeros(K, dt)
    nchunk = (K + REFL_PER_CHUNK - 1) // REFL_PER_CHUNK
    seqs = np.random.SeedSequence(seed).spawn(max(nchunk, 1))
    col = np.arange(nbw)

    def fill(ch):
        a, b = ch * REFL_PER_CHUNK, min(K, (ch + 1) * REFL_PER_CHUNK)
        rng = np.random.default_rng(seqs[ch])
        L = lengths[a:b]
        scale = 1.0 / np.sqrt(L.astype(np.float64))[:, None]
        if dtype == "z":
            w = rng.standard_normal((b - a, nbw)) + 1j * rng.standard_normal((b - a, nbw))
            w *= np.sqrt(0.5) * scale
            theta = rng.uniform(0.5 * np.pi, 1.5 * np.pi, b - a)
        else:
            w = rng.standard_normal((b - a, nbw)) * scale
        w[col[None, :] >= L[:, None]] = 0
        w[:, 0] = 1.0
        nrm2 = np.sum(w.real ** 2 + w.imag ** 2, axis=1) if dtype == "z" else np.sum(w * w, axis=1)
        V[a:b] = w
        if dtype == "z":
            tau[a:b] = (1.0 - np.exp(1j * theta)) / nrm2
        else:
            tau[a:b] = 2.0 / nrm2

    _parallel(fill, range(nchunk))
    return V, tau


def batched_sizes(count: int = 64, seed: int = 1004):
    """C4 problem sizes: n_p = 512 * U{1..8} drawn by default_rng(seed)."""
    rng = np.random.default_rng(seed)
    return (512 * rng.integers(1, 9, count)).astype(np.int64)


def batched_seeds(count: int = 64, seed: int = 1004):
    """Per-problem band seeds for C4 from SeedSequence(seed).spawn(count)."""
    return [int(s.generate_state(1)[0]) for s in np.random.SeedSequence(seed).spawn(count)]


def hermitian_matrix(n: int, seed: int, dtype: str = "d") -> np.ndarray:
    """Dense Hermitian n x n matrix (Fortran order) with the entry law of the
    band workloads: real N(0,1) (symmetric); complex off-diagonal N(0,1/2) +
    i N(0,1/2), real diagonal N(0,1).  Draw order (default_rng(seed)): real
    standard_normal((n, n)), lower triangle mirrored; complex diagonal
    standard_normal(n), then real and imaginary parts standard_normal((n, n))
    each, lower triangles used."""
    rng = np.random.default_rng(seed)
    if dtype == "z":
        dg = rng.standard_normal(n)
        re = rng.standard_normal((n, n))
        im = rng.standard_normal((n, n))
        L = np.tril(np.sqrt(0.5) * (re + 1j * im), -1)
        A = L + L.conj().T + np.diag(dg).astype(np.complex128)
    else:
        L = np.tril(rng.standard_normal((n, n)))
        A = L + np.tril(L, -1).T
    return np.asfortranarray(A)


def full_reflector_count(n: int, nbw: int) -> int:
    """Input-format bookkeeping: the full-to-band reduction stores one
    reflector per column j = 0 .. n-nbw-2 (rows [j+nbw, n) of column j of an
    n x J array); a trailing length-1 piece carries none."""
    return max(n - nbw - 1, 0) if nbw >= 1 else 0


def full_unitary_reflectors(n: int, nbw: int, seed: int, dtype: str = "d", cols=None):
    """Random unitary Householder reflectors with the shape of full-to-band
    output: an (n, J) Fortran array whose column j holds v_j in rows
    [j+nbw, n) (v_j[0] = 1, the rest N(0, 1/len), complex each part
    N(0, 1/(2 len))) and zeros elsewhere, and tau as in unitary_reflectors
    (real 2/||v||^2; complex (1 - e^{i theta})/||v||^2, theta ~ U(pi/2,
    3pi/2)).  Column j depends only on (seed, j // 64), so ``cols`` returns
    just those columns of V (and their tau)."""
    J = full_reflector_count(n, nbw)
    cols = np.arange(J) if cols is None else np.asarray(cols)
    dt = _np_dtype(dtype)
    V = np.zeros((n, len(cols)), dt, order="F")
    tau = np.zeros(len(cols), dt)
    CH = 64
    nchunk = (J + CH - 1) // CH
    seqs = np.random.SeedSequence(seed).spawn(max(nchunk, 1))
    need = {}
    for i, c in enumerate(cols):
        need.setdefault(int(c) // CH, []).append((i, int(c)))

    def fill(item):
        ch, items = item
        rng = np.random.default_rng(seqs[ch])
        w = min(CH, J - ch * CH)
        if dtype == "z":
            blk = rng.standard_normal((w, n)) + 1j * rng.standard_normal((w, n))
            blk *= np.sqrt(0.5)
            theta = rng.uniform(0.5 * np.pi, 1.5 * np.pi, w)
        else:
            blk = rng.standard_normal((w, n))
        for i, c in items:
            q = c - ch * CH
            r = c + nbw
            m = n - r
            v = blk[q, r:] / np.sqrt(m)
            v[0] = 1.0
            V[r:, i] = v
            nrm2 = float(np.sum(np.abs(v) ** 2))
            tau[i] = (1.0 - np.exp(1j * theta[q])) / nrm2 if dtype == "z" else 2.0 / nrm2

    _parallel(fill, need.items())
    return V, tau
