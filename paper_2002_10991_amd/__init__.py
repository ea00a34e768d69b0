"""Python binding for libtrbt.so: the MI355X tridiagonal-to-banded eigenvector
back-transformation (Yu et al., CPC 2020, Sec. 2.2.2, Eq. 2stage_bkwd1).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``csrc/trbt.hip`` behind the C ABI declared in ``include/trbt.h``.
PyTorch supplies device memory and the stream.  There is no CPU fallback: if
the library is missing, every call raises.

The functions carry the C names.  Device buffers are passed as torch tensors
(their data_ptr is taken) or as raw integer addresses.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

__all__ = [
    "TrbtError", "lib", "trbt_num_reflectors", "trbt_stage_offsets", "trbt_workspace_bytes",
    "trans_ev_tridi_to_band_d", "trans_ev_tridi_to_band_z", "trbt_prepare_d", "trbt_prepare_z",
    "trbt_apply_d", "trbt_apply_z", "trbt_strerror", "back_transform", "alloc_workspace",
    "TRBT_WORK_ALIGN", "TRBT_NBW_MAX", "trbt_problem_d", "trbt_problem_z", "trbt_plan_config",
    "trbt_plan_create_batched_d", "trbt_plan_create_batched_z", "trbt_plan_exec",
    "trbt_plan_get_config", "trbt_plan_check", "trbt_plan_destroy", "BatchedPlan", "trbt_adjoint_workspace_bytes_d",
    "trans_ev_tridi_to_band_adjoint_d", "trans_ev_tridi_to_band_fwd_ckpt_d",
    "trans_ev_tridi_to_band_bwd_ckpt_d", "adjoint", "BackTransform", "back_transform_autograd",
    "trbt_band_to_tridi_workspace_bytes", "trbt_band_to_tridi_d", "trbt_band_to_tridi_z",
    "trbt_adjoint_workspace_bytes_z", "trans_ev_tridi_to_band_adjoint_z",
    "trans_ev_tridi_to_band_fwd_ckpt_z", "trans_ev_tridi_to_band_bwd_ckpt_z",
    "band_to_tridiagonal", "trbt_tridiag_eigh_workspace_bytes", "trbt_tridiag_eigh_d",
    "tridiagonal_eigh", "trbt_work_check", "trbt_band_to_full_workspace_bytes",
    "trans_ev_band_to_full_d", "trans_ev_band_to_full_z", "band_to_full",
    "trans_ev_band_to_full_z_noalloc", "TRBT_B2F_SCRATCH_BYTES",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
# TRBT_LIB selects another build of the same library (the host-sanitizer
# and wait-jitter debug builds); default: the in-tree release build.
LIB_PATH = os.environ.get("TRBT_LIB") or os.path.join(_HERE, "libtrbt.so")
TRBT_WORK_ALIGN = 256
TRBT_NBW_MAX = 256
TRBT_B2F_SCRATCH_BYTES = 32 << 20
_lib = None


class trbt_problem_d(C.Structure):
    """One problem of a batched plan (device pointers as integers)."""
    _fields_ = [("n", C.c_int64), ("nbw", C.c_int), ("nev", C.c_int64),
                ("hh_v", C.c_void_p), ("hh_tau", C.c_void_p), ("Z", C.c_void_p),
                ("ldz", C.c_int64)]


class trbt_problem_z(C.Structure):
    """One complex problem of a batched plan (device pointers as integers)."""
    _fields_ = [("n", C.c_int64), ("nbw", C.c_int), ("nev", C.c_int64),
                ("hh_v", C.c_void_p), ("hh_tau", C.c_void_p), ("Z", C.c_void_p),
                ("ldz", C.c_int64)]


class trbt_plan_config(C.Structure):
    _fields_ = [("strip_cols", C.c_int), ("waves", C.c_int), ("block_stages", C.c_int)]


class TrbtError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: status {status} ({trbt_strerror(status)})")


def lib():
    """Load libtrbt.so (built by ``python -m paper_2002_10991_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run python -m paper_2002_10991_amd.build")
        L = C.CDLL(LIB_PATH)
        i64, i32, vp, sz = C.c_int64, C.c_int, C.c_void_p, C.c_size_t
        L.trbt_num_reflectors.argtypes = [i64, i32, C.POINTER(i64)]
        L.trbt_stage_offsets.argtypes = [i64, i32, C.POINTER(i64)]
        L.trbt_workspace_bytes.argtypes = [i64, i32, i64, i32, C.POINTER(sz)]
        for f in (L.trans_ev_tridi_to_band_d, L.trans_ev_tridi_to_band_z, L.trbt_apply_d,
                  L.trbt_apply_z):
            f.argtypes = [i64, i32, i64, vp, vp, vp, i64, vp, sz, vp]
            f.restype = i32
        for f in (L.trbt_prepare_d, L.trbt_prepare_z):
            f.argtypes = [i64, i32, vp, vp, vp, sz, vp]
            f.restype = i32
        L.trbt_adjoint_workspace_bytes_d.argtypes = [i64, i32, i64, i32, C.POINTER(sz)]
        L.trbt_adjoint_workspace_bytes_d.restype = i32
        L.trans_ev_tridi_to_band_adjoint_d.argtypes = [i64, i32, i64, vp, vp, vp, i64, vp, i64,
                                                       vp, vp, i32, vp, sz, vp]
        L.trans_ev_tridi_to_band_adjoint_d.restype = i32
        L.trans_ev_tridi_to_band_fwd_ckpt_d.argtypes = [i64, i32, i64, vp, vp, vp, i64, i32, vp,
                                                        sz, vp]
        L.trans_ev_tridi_to_band_fwd_ckpt_d.restype = i32
        L.trans_ev_tridi_to_band_bwd_ckpt_d.argtypes = [i64, i32, i64, vp, vp, vp, i64, vp, vp,
                                                        i32, vp, sz, vp]
        L.trans_ev_tridi_to_band_bwd_ckpt_d.restype = i32
        L.trbt_adjoint_workspace_bytes_z.argtypes = [i64, i32, i64, i32, C.POINTER(sz)]
        L.trbt_adjoint_workspace_bytes_z.restype = i32
        L.trans_ev_tridi_to_band_adjoint_z.argtypes = \
            L.trans_ev_tridi_to_band_adjoint_d.argtypes
        L.trans_ev_tridi_to_band_adjoint_z.restype = i32
        L.trans_ev_tridi_to_band_fwd_ckpt_z.argtypes = \
            L.trans_ev_tridi_to_band_fwd_ckpt_d.argtypes
        L.trans_ev_tridi_to_band_fwd_ckpt_z.restype = i32
        L.trans_ev_tridi_to_band_bwd_ckpt_z.argtypes = \
            L.trans_ev_tridi_to_band_bwd_ckpt_d.argtypes
        L.trans_ev_tridi_to_band_bwd_ckpt_z.restype = i32
        L.trbt_tridiag_eigh_workspace_bytes.argtypes = [i64, i64, C.POINTER(sz)]
        L.trbt_tridiag_eigh_workspace_bytes.restype = i32
        L.trbt_tridiag_eigh_d.argtypes = [i64, i64, vp, vp, vp, vp, i64, vp, sz, vp]
        L.trbt_tridiag_eigh_d.restype = i32
        L.trbt_band_to_tridi_workspace_bytes.argtypes = [i64, i32, i32, C.POINTER(sz)]
        L.trbt_band_to_tridi_workspace_bytes.restype = i32
        for f in (L.trbt_band_to_tridi_d, L.trbt_band_to_tridi_z):
            f.argtypes = [i64, i32, vp, i64, vp, vp, vp, vp, vp, sz, vp]
            f.restype = i32
        L.trbt_plan_create_batched_d.argtypes = [C.POINTER(trbt_problem_d), i32,
                                                 C.POINTER(trbt_plan_config),
                                                 C.POINTER(vp), vp]
        L.trbt_plan_create_batched_d.restype = i32
        L.trbt_plan_create_batched_z.argtypes = [C.POINTER(trbt_problem_z), i32,
                                                 C.POINTER(trbt_plan_config),
                                                 C.POINTER(vp), vp]
        L.trbt_plan_create_batched_z.restype = i32
        L.trbt_plan_exec.argtypes = [vp, vp]
        L.trbt_plan_exec.restype = i32
        L.trbt_plan_get_config.argtypes = [vp, C.POINTER(trbt_plan_config),
                                           C.POINTER(C.c_double)]
        L.trbt_plan_get_config.restype = i32
        L.trbt_plan_check.argtypes = [vp, C.POINTER(i32)]
        L.trbt_plan_check.restype = i32
        L.trbt_plan_destroy.argtypes = [vp]
        L.trbt_plan_destroy.restype = i32
        L.trbt_band_to_full_workspace_bytes.argtypes = [i64, i32, i64, i32, C.POINTER(sz)]
        L.trbt_band_to_full_workspace_bytes.restype = i32
        for f in (L.trans_ev_band_to_full_d, L.trans_ev_band_to_full_z):
            f.argtypes = [i64, i32, i64, vp, i64, vp, vp, i64, vp, sz, vp]
            f.restype = i32
        L.trans_ev_band_to_full_z_noalloc.argtypes = [i64, i32, i64, vp, i64, vp, vp, i64, vp]
        L.trans_ev_band_to_full_z_noalloc.restype = i32
        L.trbt_work_check.argtypes = [vp, C.POINTER(i32), vp]
        L.trbt_work_check.restype = i32
        L.trbt_strerror.argtypes = [i32]
        L.trbt_strerror.restype = C.c_char_p
        _lib = L
    return _lib


def _ptr(x) -> int | None:
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return int(x.data_ptr())


def _stream(stream) -> int | None:
    if stream is None:
        import torch
        return int(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


def trbt_strerror(status: int) -> str:
    return lib().trbt_strerror(int(status)).decode()


def trbt_work_check(work, stream=None) -> int:
    """Synchronize `stream` and return the workspace's fault word (0 or 1):
    nonzero means a bounded wait between workgroups gave up and the outputs
    of the call that used `work` are invalid."""
    f = C.c_int()
    rc = lib().trbt_work_check(_ptr(work), C.byref(f), _stream(stream))
    if rc:
        raise TrbtError(rc, "trbt_work_check")
    return f.value


def trbt_num_reflectors(n: int, nbw: int) -> int:
    K = C.c_int64()
    rc = lib().trbt_num_reflectors(n, nbw, C.byref(K))
    if rc:
        raise TrbtError(rc, "trbt_num_reflectors")
    return K.value


def trbt_stage_offsets(n: int, nbw: int) -> np.ndarray:
    off = np.zeros(max(n - 1, 1), np.int64)
    rc = lib().trbt_stage_offsets(n, nbw, off.ctypes.data_as(C.POINTER(C.c_int64)))
    if rc:
        raise TrbtError(rc, "trbt_stage_offsets")
    return off


def trbt_workspace_bytes(n: int, nbw: int, nev: int, is_complex: bool) -> int:
    b = C.c_size_t()
    rc = lib().trbt_workspace_bytes(n, nbw, nev, int(bool(is_complex)), C.byref(b))
    if rc:
        raise TrbtError(rc, "trbt_workspace_bytes")
    return b.value


def trans_ev_tridi_to_band_d(n, nbw, nev, hh_v, hh_tau, Z, ldz, work, work_bytes, stream=None) -> int:
    """Status-returning call of the C entry point (real FP64)."""
    return lib().trans_ev_tridi_to_band_d(n, nbw, nev, _ptr(hh_v), _ptr(hh_tau), _ptr(Z), ldz,
                                          _ptr(work), work_bytes, _stream(stream))


def trans_ev_tridi_to_band_z(n, nbw, nev, hh_v, hh_tau, Z, ldz, work, work_bytes, stream=None) -> int:
    """Status-returning call of the C entry point (complex FP64)."""
    return lib().trans_ev_tridi_to_band_z(n, nbw, nev, _ptr(hh_v), _ptr(hh_tau), _ptr(Z), ldz,
                                          _ptr(work), work_bytes, _stream(stream))


def trbt_prepare_d(n, nbw, hh_v, hh_tau, work, work_bytes, stream=None) -> int:
    return lib().trbt_prepare_d(n, nbw, _ptr(hh_v), _ptr(hh_tau), _ptr(work), work_bytes,
                                _stream(stream))


def trbt_prepare_z(n, nbw, hh_v, hh_tau, work, work_bytes, stream=None) -> int:
    return lib().trbt_prepare_z(n, nbw, _ptr(hh_v), _ptr(hh_tau), _ptr(work), work_bytes,
                                _stream(stream))


def trbt_apply_d(n, nbw, nev, hh_v, hh_tau, Z, ldz, work, work_bytes, stream=None) -> int:
    return lib().trbt_apply_d(n, nbw, nev, _ptr(hh_v), _ptr(hh_tau), _ptr(Z), ldz, _ptr(work),
                              work_bytes, _stream(stream))


def trbt_apply_z(n, nbw, nev, hh_v, hh_tau, Z, ldz, work, work_bytes, stream=None) -> int:
    return lib().trbt_apply_z(n, nbw, nev, _ptr(hh_v), _ptr(hh_tau), _ptr(Z), ldz, _ptr(work),
                              work_bytes, _stream(stream))


def alloc_workspace(n: int, nbw: int, nev: int, is_complex: bool, device="cuda"):
    """A torch uint8 device buffer of the size the call needs (or None)."""
    import torch
    nb = trbt_workspace_bytes(n, nbw, nev, is_complex)
    if nb == 0:
        return None
    buf = torch.empty(nb + TRBT_WORK_ALIGN, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % TRBT_WORK_ALIGN
    return buf[off: off + nb]


def back_transform(Z, hh_v, hh_tau, nbw: int, work=None, stream=None):
    """In-place Y = Q^* X on a CUDA/HIP tensor.

    Z: (n, nev) float64 or complex128 tensor with unit row stride (a
    column-major view, e.g. ``buf.T[:n]`` of a (nev, ldz) buffer).
    hh_v: (K, nbw) contiguous, hh_tau: (K,) contiguous, same dtype family.
    Returns Z."""
    import torch
    n, nev = Z.shape
    if nev and n and Z.stride(0) != 1:
        raise ValueError("Z must be column-major (unit row stride)")
    ldz = Z.stride(1) if nev > 1 else max(n, 1)
    cplx = Z.dtype == torch.complex128
    if not cplx and Z.dtype != torch.float64:
        raise TypeError("Z must be float64 or complex128")
    for name, t in (("hh_v", hh_v), ("hh_tau", hh_tau)):
        if t.dtype != Z.dtype or not t.is_contiguous():
            raise TypeError(f"{name} must be contiguous and of Z's dtype")
    if work is None:
        work = alloc_workspace(n, nbw, nev, cplx, Z.device)
    wb = 0 if work is None else work.numel() * work.element_size()
    f = trans_ev_tridi_to_band_z if cplx else trans_ev_tridi_to_band_d
    rc = f(n, nbw, nev, hh_v, hh_tau, Z, max(ldz, 1), work, wb, stream)
    if rc:
        raise TrbtError(rc, f.__name__)
    return Z


# --------------------------------------------------------------------------
# Batched plans
# --------------------------------------------------------------------------
def _plan_create(fn, struct, probs, cfg, stream):
    arr = (struct * max(len(probs), 1))()
    for i, p in enumerate(probs):
        arr[i] = p if isinstance(p, struct) else struct(*p)
    c = None
    if cfg is not None:
        c = cfg if isinstance(cfg, trbt_plan_config) else trbt_plan_config(*cfg)
    h = C.c_void_p()
    rc = fn(arr if probs else None, len(probs), C.byref(c) if c is not None else None,
            C.byref(h), _stream(stream))
    return rc, (h.value if rc == 0 else None)


def trbt_plan_create_batched_d(probs, cfg=None, stream=None):
    """probs: sequence of trbt_problem_d (or of tuples in its field order).
    cfg: None (autotune) or trbt_plan_config / (strip_cols, waves, block_stages).
    Returns (status, plan handle or None)."""
    return _plan_create(lib().trbt_plan_create_batched_d, trbt_problem_d, probs, cfg, stream)


def trbt_plan_create_batched_z(probs, cfg=None, stream=None):
    """The same for complex problems (sequence of trbt_problem_z)."""
    return _plan_create(lib().trbt_plan_create_batched_z, trbt_problem_z, probs, cfg, stream)


def trbt_plan_exec(plan, stream=None) -> int:
    return lib().trbt_plan_exec(plan, _stream(stream))


def trbt_plan_get_config(plan):
    c = trbt_plan_config()
    ms = C.c_double()
    rc = lib().trbt_plan_get_config(plan, C.byref(c), C.byref(ms))
    if rc:
        raise TrbtError(rc, "trbt_plan_get_config")
    return (c.strip_cols, c.waves, c.block_stages), ms.value


def trbt_plan_check(plan) -> int:
    f = C.c_int()
    rc = lib().trbt_plan_check(plan, C.byref(f))
    if rc:
        raise TrbtError(rc, "trbt_plan_check")
    return f.value


def trbt_plan_destroy(plan) -> int:
    return lib().trbt_plan_destroy(plan)


class BatchedPlan:
    """A batched plan over torch tensors.

    problems: list of (Z, hh_v, hh_tau, nbw) with Z an (n, nev) column-major
    view (unit row stride) and hh_v (K, nbw), hh_tau (K,) contiguous, all
    float64 (a real plan) or all complex128 (a complex plan), on the current
    device.  The tensors must stay alive (same storage) for the plan's
    lifetime; their contents may change between runs."""

    def __init__(self, problems, cfg=None, stream=None):
        import torch
        descs = []
        self._keep = []
        dtypes = {t.dtype for Z, hv, ht, nbw in problems for t in (Z, hv, ht)}
        if not dtypes <= {torch.float64} and not dtypes <= {torch.complex128}:
            raise TypeError("batched plans are all float64 or all complex128")
        cplx = dtypes == {torch.complex128}
        struct = trbt_problem_z if cplx else trbt_problem_d
        for Z, hv, ht, nbw in problems:
            n, nev = Z.shape
            if nev and n and Z.stride(0) != 1:
                raise ValueError("Z must be column-major (unit row stride)")
            if not hv.is_contiguous() or not ht.is_contiguous():
                raise TypeError("hh_v and hh_tau must be contiguous")
            ldz = Z.stride(1) if nev > 1 else max(n, 1)
            descs.append(struct(n, nbw, nev, _ptr(hv) if hv.numel() else None,
                                _ptr(ht) if ht.numel() else None,
                                _ptr(Z) if Z.numel() else None, max(ldz, 1)))
            self._keep.append((Z, hv, ht))
        create = trbt_plan_create_batched_z if cplx else trbt_plan_create_batched_d
        rc, self.handle = create(descs, cfg, stream)
        if rc:
            raise TrbtError(rc, create.__name__)

    @property
    def config(self):
        return trbt_plan_get_config(self.handle)

    def run(self, stream=None):
        rc = trbt_plan_exec(self.handle, stream)
        if rc:
            raise TrbtError(rc, "trbt_plan_exec")

    def fault(self) -> int:
        return trbt_plan_check(self.handle)

    def close(self):
        if self.handle is not None:
            trbt_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --------------------------------------------------------------------------
# Adjoint
# --------------------------------------------------------------------------
def trbt_adjoint_workspace_bytes_d(n: int, nbw: int, nev: int, ckpt_every: int = 16) -> int:
    b = C.c_size_t()
    rc = lib().trbt_adjoint_workspace_bytes_d(n, nbw, nev, ckpt_every, C.byref(b))
    if rc:
        raise TrbtError(rc, "trbt_adjoint_workspace_bytes_d")
    return b.value


def trans_ev_tridi_to_band_adjoint_d(n, nbw, nev, hh_v, hh_tau, Z_in, ldz, G, ldg, dv, dtau,
                                     ckpt_every, work, work_bytes, stream=None) -> int:
    """Status-returning call of the C entry point."""
    return lib().trans_ev_tridi_to_band_adjoint_d(
        n, nbw, nev, _ptr(hh_v), _ptr(hh_tau), _ptr(Z_in), ldz, _ptr(G), ldg, _ptr(dv),
        _ptr(dtau), ckpt_every, _ptr(work), work_bytes, _stream(stream))


def trbt_adjoint_workspace_bytes_z(n: int, nbw: int, nev: int, ckpt_every: int = 16) -> int:
    b = C.c_size_t()
    rc = lib().trbt_adjoint_workspace_bytes_z(n, nbw, nev, ckpt_every, C.byref(b))
    if rc:
        raise TrbtError(rc, "trbt_adjoint_workspace_bytes_z")
    return b.value


def trans_ev_tridi_to_band_adjoint_z(n, nbw, nev, hh_v, hh_tau, Z_in, ldz, G, ldg, dv, dtau,
                                     ckpt_every, work, work_bytes, stream=None) -> int:
    """Status-returning call of the C entry point (complex)."""
    return lib().trans_ev_tridi_to_band_adjoint_z(
        n, nbw, nev, _ptr(hh_v), _ptr(hh_tau), _ptr(Z_in), ldz, _ptr(G), ldg, _ptr(dv),
        _ptr(dtau), ckpt_every, _ptr(work), work_bytes, _stream(stream))


def trans_ev_tridi_to_band_fwd_ckpt_d(n, nbw, nev, hh_v, hh_tau, Z, ldz, ckpt_every, work,
                                      work_bytes, stream=None) -> int:
    return lib().trans_ev_tridi_to_band_fwd_ckpt_d(
        n, nbw, nev, _ptr(hh_v), _ptr(hh_tau), _ptr(Z), ldz, ckpt_every, _ptr(work), work_bytes,
        _stream(stream))


def trans_ev_tridi_to_band_bwd_ckpt_d(n, nbw, nev, hh_v, hh_tau, G, ldg, dv, dtau, ckpt_every,
                                      work, work_bytes, stream=None) -> int:
    return lib().trans_ev_tridi_to_band_bwd_ckpt_d(
        n, nbw, nev, _ptr(hh_v), _ptr(hh_tau), _ptr(G), ldg, _ptr(dv), _ptr(dtau), ckpt_every,
        _ptr(work), work_bytes, _stream(stream))


def trans_ev_tridi_to_band_fwd_ckpt_z(n, nbw, nev, hh_v, hh_tau, Z, ldz, ckpt_every, work,
                                      work_bytes, stream=None) -> int:
    return lib().trans_ev_tridi_to_band_fwd_ckpt_z(
        n, nbw, nev, _ptr(hh_v), _ptr(hh_tau), _ptr(Z), ldz, ckpt_every, _ptr(work), work_bytes,
        _stream(stream))


def trans_ev_tridi_to_band_bwd_ckpt_z(n, nbw, nev, hh_v, hh_tau, G, ldg, dv, dtau, ckpt_every,
                                      work, work_bytes, stream=None) -> int:
    return lib().trans_ev_tridi_to_band_bwd_ckpt_z(
        n, nbw, nev, _ptr(hh_v), _ptr(hh_tau), _ptr(G), ldg, _ptr(dv), _ptr(dtau), ckpt_every,
        _ptr(work), work_bytes, _stream(stream))


def _adjoint_workspace(n, nbw, nev, device, cplx=False):
    import torch
    nb = (trbt_adjoint_workspace_bytes_z if cplx else trbt_adjoint_workspace_bytes_d)(n, nbw, nev)
    if not nb:
        return None, 0
    buf = torch.empty(nb + TRBT_WORK_ALIGN, dtype=torch.uint8, device=device)
    return buf[(-buf.data_ptr()) % TRBT_WORK_ALIGN:][:nb], nb


def _colmajor(t):
    """(n, nev) tensor -> (a new buffer (nev, n) contiguous holding a copy of
    it, and the buffer's column-major (n, nev) view).  Always a copy: the
    kernels work in place and must not write through an alias of t."""
    import torch
    buf = torch.empty((t.shape[1], t.shape[0]), dtype=t.dtype, device=t.device)
    buf.copy_(t.t())
    return buf, buf.t()


def adjoint(Z_in, G, hh_v, hh_tau, nbw: int, work=None, stream=None):
    """dL/dZ_in, dL/dv, dL/dtau of Z_out = H_0..H_{K-1} Z_in for G = dL/dZ_out.

    Z_in, G: (n, nev) float64 or complex128 tensors with unit row stride
    (column-major views); G is overwritten with dL/dZ_in.  Complex: the
    conjugate-Wirtinger gradients of a real L (PyTorch's convention).
    Returns (G, dv (K, nbw), dtau (K,))."""
    import torch
    n, nev = Z_in.shape
    cplx = Z_in.dtype == torch.complex128
    want = torch.complex128 if cplx else torch.float64
    for name, t in (("Z_in", Z_in), ("G", G), ("hh_v", hh_v), ("hh_tau", hh_tau)):
        if t.dtype != want:
            raise TypeError(f"{name} must be {want} like Z_in (float64 or complex128)")
    for name, t in (("Z_in", Z_in), ("G", G)):
        if nev and n and t.stride(0) != 1:
            raise ValueError(f"{name} must be column-major (unit row stride)")
    K = trbt_num_reflectors(n, nbw)
    dv = torch.empty(max(K, 1), nbw, dtype=want, device=G.device)[:K]
    dt = torch.empty(max(K, 1), dtype=want, device=G.device)[:K]
    if work is None:
        work, _ = _adjoint_workspace(n, nbw, nev, G.device, cplx)
    wb = 0 if work is None else work.numel() * work.element_size()
    ldz = Z_in.stride(1) if nev > 1 else max(n, 1)
    ldg = G.stride(1) if nev > 1 else max(n, 1)
    f = trans_ev_tridi_to_band_adjoint_z if cplx else trans_ev_tridi_to_band_adjoint_d
    rc = f(n, nbw, nev, hh_v, hh_tau, Z_in, max(ldz, 1), G, max(ldg, 1), dv if K else None,
           dt if K else None, 16, work, wb, stream)
    if rc:
        raise TrbtError(rc, f.__name__)
    return G, dv, dt


def _back_transform_function():
    import torch

    class BackTransform(torch.autograd.Function):
        """Z_out = H_0 ... H_{K-1} Z_in with the hand-written adjoint.

        The forward pass runs the checkpointing forward kernel and keeps its
        workspace (a checkpoint every 16 stages, not the states in between)
        for the backward pass, which recomputes the states inside each
        16-stage block from it; the backward pass only reads the
        checkpoints, so it may run more than once (retain_graph).  Complex (conjugate-Wirtinger gradients, as
        PyTorch's complex autograd expects) takes the same split pair for
        nbw in {16, 32, 48, 64}; for other band widths the forward pass is
        the plain transformation and the backward pass the one-call complex
        adjoint from the saved Z_in."""

        @staticmethod
        def forward(ctx, Z_in, hh_v, hh_tau, nbw):
            obuf, out = _colmajor(Z_in.detach())
            n, nev = out.shape
            v = hh_v.detach().contiguous()
            t = hh_tau.detach().contiguous()
            if out.dtype == torch.complex128 and v.dtype == out.dtype and t.dtype == out.dtype:
                ctx.cplx, ctx.nbw, ctx.shape = True, nbw, (n, nev)
                if nbw in (16, 32, 48, 64):
                    work, nb = _adjoint_workspace(n, nbw, nev, out.device, True)
                    rc = trans_ev_tridi_to_band_fwd_ckpt_z(n, nbw, nev, v, t, out, max(n, 1), 16,
                                                           work, nb)
                    if rc == 0:
                        ctx.split = True
                        ctx.save_for_backward(v, t)
                        ctx.work, ctx.nb = work, nb
                        return out
                    if rc != -1:   # -1 (n beyond the blocked kernels' range): nothing ran
                        raise TrbtError(rc, "trans_ev_tridi_to_band_fwd_ckpt_z")
                ctx.split = False
                back_transform(out, v, t, nbw)
                ctx.save_for_backward(v, t, Z_in.detach().clone())
                return out
            if v.dtype != torch.float64 or out.dtype != torch.float64 or t.dtype != torch.float64:
                raise TypeError("the differentiable back-transformation takes float64 or "
                                "complex128 (Z_in, hh_v, hh_tau of one dtype)")
            ctx.cplx = False
            work, nb = _adjoint_workspace(n, nbw, nev, out.device)
            rc = trans_ev_tridi_to_band_fwd_ckpt_d(n, nbw, nev, v, t, out, max(n, 1), 16, work,
                                                   nb)
            if rc:
                raise TrbtError(rc, "trans_ev_tridi_to_band_fwd_ckpt_d")
            ctx.save_for_backward(v, t)
            ctx.work, ctx.nb, ctx.nbw, ctx.shape = work, nb, nbw, (n, nev)
            return out

        @staticmethod
        def backward(ctx, grad_out):
            if ctx.cplx and ctx.split:
                v, t = ctx.saved_tensors
                n, nev = ctx.shape
                gbuf, g = _colmajor(grad_out.to(torch.complex128))
                K = v.shape[0]
                dv = torch.empty(max(K, 1), ctx.nbw, dtype=torch.complex128, device=v.device)[:K]
                dt = torch.empty(max(K, 1), dtype=torch.complex128, device=v.device)[:K]
                rc = trans_ev_tridi_to_band_bwd_ckpt_z(n, ctx.nbw, nev, v, t, g, max(n, 1),
                                                       dv if K else None, dt if K else None, 16,
                                                       ctx.work, ctx.nb)
                if rc:
                    raise TrbtError(rc, "trans_ev_tridi_to_band_bwd_ckpt_z")
                return g, dv, dt, None
            if ctx.cplx:
                v, t, zin = ctx.saved_tensors
                _, zc = _colmajor(zin)
                gbuf, g = _colmajor(grad_out.to(torch.complex128))
                g, dv, dt = adjoint(zc, g, v, t, ctx.nbw)
                return g, dv, dt, None
            v, t = ctx.saved_tensors
            n, nev = ctx.shape
            gbuf, g = _colmajor(grad_out)
            K = v.shape[0]
            dv = torch.empty(max(K, 1), ctx.nbw, dtype=torch.float64, device=v.device)[:K]
            dt = torch.empty(max(K, 1), dtype=torch.float64, device=v.device)[:K]
            rc = trans_ev_tridi_to_band_bwd_ckpt_d(n, ctx.nbw, nev, v, t, g, max(n, 1),
                                                   dv if K else None, dt if K else None, 16,
                                                   ctx.work, ctx.nb)
            if rc:
                raise TrbtError(rc, "trans_ev_tridi_to_band_bwd_ckpt_d")
            return g, dv, dt, None

    return BackTransform


class _Lazy:
    fn = None


def back_transform_autograd(Z_in, hh_v, hh_tau, nbw: int):
    """Differentiable back-transformation (torch.autograd), float64 or complex128
    (complex: conjugate-Wirtinger gradients, PyTorch's convention)."""
    if _Lazy.fn is None:
        _Lazy.fn = _back_transform_function()
    return _Lazy.fn.apply(Z_in, hh_v, hh_tau, nbw)


def __getattr__(name):
    if name == "BackTransform":
        if _Lazy.fn is None:
            _Lazy.fn = _back_transform_function()
        return _Lazy.fn
    raise AttributeError(name)


# --------------------------------------------------------------------------
# Banded -> tridiagonal bulge chasing (the producer of hh_v / hh_tau)
# --------------------------------------------------------------------------
def trbt_band_to_tridi_workspace_bytes(n: int, nbw: int, is_complex: bool) -> int:
    nb = C.c_size_t()
    rc = lib().trbt_band_to_tridi_workspace_bytes(n, nbw, int(bool(is_complex)), C.byref(nb))
    if rc:
        raise TrbtError(rc, "trbt_band_to_tridi_workspace_bytes")
    return nb.value


def trbt_band_to_tridi_d(n, nbw, ab, ldab, d, e, hh_v, hh_tau, work, work_bytes,
                         stream=None) -> int:
    return lib().trbt_band_to_tridi_d(n, nbw, _ptr(ab), ldab, _ptr(d), _ptr(e), _ptr(hh_v),
                                      _ptr(hh_tau), _ptr(work), work_bytes, _stream(stream))


def trbt_band_to_tridi_z(n, nbw, ab, ldab, d, e, hh_v, hh_tau, work, work_bytes,
                         stream=None) -> int:
    return lib().trbt_band_to_tridi_z(n, nbw, _ptr(ab), ldab, _ptr(d), _ptr(e), _ptr(hh_v),
                                      _ptr(hh_tau), _ptr(work), work_bytes, _stream(stream))


def band_to_tridiagonal(ab, nbw: int, work=None, stream=None):
    """Bulge-chase a Hermitian band matrix to tridiagonal form on the GPU.

    ab: (n, ldab) float64 or complex128 device tensor, C-contiguous, with
    ab[k, d] = B(k+d, k) for d = 0..nbw (LAPACK lower band storage read
    column by column).  Returns (d, e, hh_v, hh_tau): d (n,) float64, e
    (n-1,) of ab's dtype, hh_v (K, nbw) and hh_tau (K,) of ab's dtype, in
    the generation order trans_ev_tridi_to_band_{d,z} take."""
    import torch
    if ab.dim() != 2 or not ab.is_contiguous():
        raise ValueError("ab must be a contiguous (n, ldab) tensor")
    n, ldab = ab.shape
    cplx = ab.dtype == torch.complex128
    if not cplx and ab.dtype != torch.float64:
        raise TypeError("ab must be float64 or complex128")
    K = trbt_num_reflectors(n, nbw)
    dev = ab.device
    d = torch.empty(n, dtype=torch.float64, device=dev)
    e = torch.empty(max(n - 1, 0), dtype=ab.dtype, device=dev)
    hv = torch.empty((K, nbw), dtype=ab.dtype, device=dev)
    ht = torch.empty(K, dtype=ab.dtype, device=dev)
    if work is None:
        nb = trbt_band_to_tridi_workspace_bytes(n, nbw, cplx)
        if nb:
            buf = torch.empty(nb + TRBT_WORK_ALIGN, dtype=torch.uint8, device=dev)
            off = (-buf.data_ptr()) % TRBT_WORK_ALIGN
            work = buf[off: off + nb]
    wb = 0 if work is None else work.numel() * work.element_size()
    f = trbt_band_to_tridi_z if cplx else trbt_band_to_tridi_d
    rc = f(n, nbw, ab, ldab, d, e if n > 1 else None, hv if K else None, ht if K else None,
           work, wb, stream)
    if rc:
        raise TrbtError(rc, f.__name__)
    return d, e, hv, ht


# --------------------------------------------------------------------------
# Tridiagonal eigenpairs (bisection + inverse iteration)
# --------------------------------------------------------------------------
def trbt_tridiag_eigh_workspace_bytes(n: int, nev: int) -> int:
    nb = C.c_size_t()
    rc = lib().trbt_tridiag_eigh_workspace_bytes(n, nev, C.byref(nb))
    if rc:
        raise TrbtError(rc, "trbt_tridiag_eigh_workspace_bytes")
    return nb.value


def trbt_tridiag_eigh_d(n, nev, d, e, w, Z, ldz, work, work_bytes, stream=None) -> int:
    return lib().trbt_tridiag_eigh_d(n, nev, _ptr(d), _ptr(e), _ptr(w), _ptr(Z), ldz,
                                     _ptr(work), work_bytes, _stream(stream))


def tridiagonal_eigh(d, e, nev: int, stream=None):
    """The lowest nev eigenpairs of the real symmetric tridiagonal
    diag(d) + subdiag(e) on the GPU.  d (n,), e (n-1,) float64 device
    tensors.  Returns (w (nev,), Z (n, nev) column-major view)."""
    import torch
    n = d.shape[0]
    if d.dtype != torch.float64 or e.dtype != torch.float64:
        raise TypeError("d and e must be float64")
    w = torch.empty(nev, dtype=torch.float64, device=d.device)
    zb = torch.empty((max(nev, 1), max(n, 1)), dtype=torch.float64, device=d.device)
    nb = trbt_tridiag_eigh_workspace_bytes(n, nev)
    work = None
    if nb:
        buf = torch.empty(nb + TRBT_WORK_ALIGN, dtype=torch.uint8, device=d.device)
        work = buf[(-buf.data_ptr()) % TRBT_WORK_ALIGN:][:nb]
    rc = trbt_tridiag_eigh_d(n, nev, d.contiguous(), e.contiguous(), w, zb, max(n, 1), work,
                             nb, stream)
    if rc:
        raise TrbtError(rc, "trbt_tridiag_eigh_d")
    return w, zb[:nev].T[:n]


# --------------------------------------------------------------------------
# Band -> full back-transformation (Eq. 2stage_bkwd2)
# --------------------------------------------------------------------------
def trbt_band_to_full_workspace_bytes(n: int, nbw: int, nev: int, is_complex: bool) -> int:
    nb = C.c_size_t()
    rc = lib().trbt_band_to_full_workspace_bytes(n, nbw, nev, int(bool(is_complex)),
                                                 C.byref(nb))
    if rc:
        raise TrbtError(rc, "trbt_band_to_full_workspace_bytes")
    return nb.value


def trans_ev_band_to_full_d(n, nbw, nev, hh_v, ldv, hh_tau, Z, ldz, work, work_bytes,
                            stream=None) -> int:
    return lib().trans_ev_band_to_full_d(n, nbw, nev, _ptr(hh_v), ldv, _ptr(hh_tau), _ptr(Z), ldz,
                                         _ptr(work), work_bytes, _stream(stream))


def trans_ev_band_to_full_z(n, nbw, nev, hh_v, ldv, hh_tau, Z, ldz, work, work_bytes,
                            stream=None) -> int:
    return lib().trans_ev_band_to_full_z(n, nbw, nev, _ptr(hh_v), ldv, _ptr(hh_tau), _ptr(Z), ldz,
                                         _ptr(work), work_bytes, _stream(stream))


def trans_ev_band_to_full_z_noalloc(n, nbw, nev, hh_v, ldv, hh_tau, Z, ldz, stream=None) -> int:
    return lib().trans_ev_band_to_full_z_noalloc(n, nbw, nev, _ptr(hh_v), ldv, _ptr(hh_tau),
                                                 _ptr(Z), ldz, _stream(stream))


def band_to_full(Z, hh_v, hh_tau, nbw: int, work=None, stream=None):
    """In-place C = P^* Y (Eq. 2stage_bkwd2) on a CUDA/HIP tensor.

    Z: (n, nev) float64 or complex128 with unit row stride (column-major
    view).  hh_v: (n, J) column-major view (unit row stride, e.g. ``buf.T``
    of a (J, ldv) buffer), column j holding reflector j in rows
    [j+nbw, n); hh_tau: (J,) contiguous.  Returns Z."""
    import torch
    n, nev = Z.shape
    if nev and n and Z.stride(0) != 1:
        raise ValueError("Z must be column-major (unit row stride)")
    cplx = Z.dtype == torch.complex128
    if not cplx and Z.dtype != torch.float64:
        raise TypeError("Z must be float64 or complex128")
    J = max(n - nbw - 1, 0)
    if hh_v.dtype != Z.dtype or hh_tau.dtype != Z.dtype or not hh_tau.is_contiguous():
        raise TypeError("hh_v and hh_tau must have Z's dtype (hh_tau contiguous)")
    if J and (hh_v.shape[0] != n or hh_v.shape[1] < J or hh_v.stride(0) != 1):
        raise ValueError(f"hh_v must be an ({n}, {J}) column-major view")
    ldv = hh_v.stride(1) if J > 1 else max(n, 1)
    ldz = Z.stride(1) if nev > 1 else max(n, 1)
    if work is None:
        nb = trbt_band_to_full_workspace_bytes(n, nbw, nev, cplx)
        if nb:
            buf = torch.empty(nb + TRBT_WORK_ALIGN, dtype=torch.uint8, device=Z.device)
            work = buf[(-buf.data_ptr()) % TRBT_WORK_ALIGN:][:nb]
    wb = 0 if work is None else work.numel() * work.element_size()
    f = trans_ev_band_to_full_z if cplx else trans_ev_band_to_full_d
    rc = f(n, nbw, nev, hh_v if J else None, max(ldv, n, 1), hh_tau if J else None, Z,
           max(ldz, 1), work, wb, stream)
    if rc:
        raise TrbtError(rc, f.__name__)
    return Z
