#!/usr/bin/env python3
"""Benchmark: tridiagonal-to-banded eigenvector back-transformation on MI355X.

One step = one full back-transformation Y = Q^* X (Yu et al., CPC 2020,
Eq. 2stage_bkwd1) of the whole eigenvector matrix: the compact-WY prepare
kernel plus the blocked apply kernel, through the C ABI.  Inputs are
resident in HBM before the timed region; Z is transformed in place, so step
k+1 applies Q^* to the output of step k (same work, Q^* is unitary).

Default workload (the headline shape): complex Hermitian, n=32768, nbw=64,
nev=8192, synthetic unitary reflectors and a Gaussian Z (see synth/).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload C3]

Prints one JSON line.  FLOP/s use the algorithmic count of the operation:
c * nev * L, c = 16 (complex) or 4 (real), L = total reflector length.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6     # MI355X dense FP64 (vector and matrix)
PEAK_HBM_GBS = 8000.0

WORKLOADS = {
    "C1": dict(n=1024, nbw=32, nev=1024, dtype="d", seed=1001),
    "C2": dict(n=8192, nbw=64, nev=4096, dtype="d", seed=1002),
    "C3": dict(n=32768, nbw=64, nev=8192, dtype="z", seed=1003),
    "C5": dict(n=4096, nbw=64, nev=2048, dtype="d", seed=1005),
    # the headline size with the widest band of the blocked kernel, and one
    # GPU's column share of the headline shape when it is split over eight
    "C3w": dict(n=32768, nbw=128, nev=8192, dtype="z", seed=1013),
    "C3s": dict(n=32768, nbw=64, nev=1024, dtype="z", seed=1003),
}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def make_inputs(cfg):
    import synth
    n, nbw, nev, dt, seed = cfg["n"], cfg["nbw"], cfg["nev"], cfg["dtype"], cfg["seed"]
    lengths = synth.reflector_lengths(n, nbw)
    V, tau = synth.unitary_reflectors(lengths, nbw, seed, dt)
    Z = synth.gaussian(n, nev, seed + 1, dt)
    return lengths, V, tau, Z


def cpu_baseline(cfg, V, tau, Z, L_total, budget_s=20.0):
    """The oracle, as it stands, on a bounded column sample of the same
    workload; columns are independent so the rate scales to the full nev."""
    import oracle
    oracle.build()
    n, nbw, nev = cfg["n"], cfg["nbw"], cfg["nev"]
    c = 16 if cfg["dtype"] == "z" else 4
    cores = oracle.num_threads()
    # calibrate on one column per thread, then size the sample to the budget
    ncols = min(nev, cores)
    cols = np.linspace(0, nev - 1, ncols).astype(np.int64)
    t = time.perf_counter()
    oracle.back_transform(Z[:, cols], V, tau, nbw)
    t_cal = time.perf_counter() - t
    rounds = max(1, int(budget_s / max(t_cal, 1e-3)) - 1)
    ncols2 = min(nev, cores * rounds)
    cols2 = np.linspace(0, nev - 1, ncols2).astype(np.int64)
    t = time.perf_counter()
    oracle.back_transform(Z[:, cols2], V, tau, nbw)
    dt = time.perf_counter() - t
    flops = c * L_total * ncols2
    return {"value": round(flops / dt / 1e12, 6), "unit": "TFLOP/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{ncols2} of {nev} columns (evenly spaced), all {len(tau)} reflectors, "
                      f"{dt:.1f} s wall; rate scales to all columns (columns are independent)"}


def c4_inputs(dt: str = "d"):
    """The batched workload: 64 problems, n_p = 512*U{1..8} (seed 1004),
    nbw = 32, nev = n_p/2, per-problem seeds from SeedSequence(1004); real
    (dt "d", C4) or complex Hermitian (dt "z", C4z)."""
    import synth
    sizes, seeds = synth.batched_sizes(), synth.batched_seeds()
    out = []
    for n, sd in zip(sizes, seeds):
        n = int(n)
        lengths = synth.reflector_lengths(n, 32)
        V, tau = synth.unitary_reflectors(lengths, 32, sd, dt)
        Z = synth.gaussian(n, n // 2, sd + 1, dt)
        out.append((n, 32, n // 2, int(lengths.sum()), V, tau, Z))
    return out


def batched_leg(steps: int, warmup: int, dt: str = "d"):
    """Batched plan (one persistent graph-captured launch, autotuned) against
    64 looped single-problem calls on one stream, same inputs, same stream."""
    import torch
    import paper_2002_10991_amd as T
    dev = torch.device("cuda:0")
    cplx = dt == "z"
    name = "C4z" if cplx else "C4"
    t = time.perf_counter()
    probs = c4_inputs(dt)
    log(f"{name} inputs ready in {time.perf_counter() - t:.1f}s")
    flops = sum((16 if cplx else 4) * nev * L for n, nbw, nev, L, V, tau, Z in probs)
    tensors = []
    for n, nbw, nev, L, V, tau, Z in probs:
        tensors.append((torch.from_numpy(np.ascontiguousarray(Z.T)).to(dev),
                        torch.from_numpy(V).to(dev), torch.from_numpy(tau).to(dev), nbw))
    stream = torch.cuda.current_stream()
    wmax = max(T.trbt_workspace_bytes(n, nbw, nev, cplx) for n, nbw, nev, *_ in probs)
    work = torch.empty(wmax + T.TRBT_WORK_ALIGN, dtype=torch.uint8, device=dev)
    work = work[(-work.data_ptr()) % T.TRBT_WORK_ALIGN:][:wmax]
    single = T.trans_ev_tridi_to_band_z if cplx else T.trans_ev_tridi_to_band_d

    def looped():
        for Zb, Vd, td, nbw in tensors:
            n, nev = Zb.shape[1], Zb.shape[0]
            rc = single(n, nbw, nev, Vd, td, Zb, n, work, wmax, stream)
            if rc:
                raise T.TrbtError(rc, single.__name__)

    t = time.perf_counter()
    plan = T.BatchedPlan([(Zb.T, Vd, td, nbw) for Zb, Vd, td, nbw in tensors], None, stream)
    create_s = time.perf_counter() - t
    cfg, tuned_ms = plan.config
    log(f"{name} plan created in {create_s:.2f}s, tuned config {cfg} ({tuned_ms:.3f} ms)")

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    loop_ms = timed(looped)
    log(f"{name} looped: {loop_ms:.3f} ms per batch")
    batch_ms = timed(plan.run)
    log(f"{name} batched: {batch_ms:.3f} ms per batch")
    if plan.fault():
        raise RuntimeError("batched plan: device wait-timeout flag set")
    plan.close()
    return {
        "workload": (f"{name}: 64 {'complex Hermitian' if cplx else 'real'} problems, "
                     "n_p = 512*U{1..8} (seed 1004), nbw=32, nev=n_p/2"),
        "flops_per_batch": flops,
        "batched_ms": round(batch_ms, 4), "looped_ms": round(loop_ms, 4),
        "batched_tflops": round(flops / batch_ms / 1e9, 4),
        "looped_tflops": round(flops / loop_ms / 1e9, 4),
        "speedup": round(loop_ms / batch_ms, 3),
        "tuned_config": {"strip_cols": cfg[0], "waves": cfg[1], "block_stages": cfg[2]},
        "plan_create_s": round(create_s, 3),
    }


def plain_adjoint(Z, G, V, tau, nbw):
    """The plain form of the differentiation workload: eager PyTorch autograd
    through a per-stage implementation (one batched gather / bmm / update /
    index_copy per stage, all slots of the stage at once), with
    torch.utils.checkpoint over 16-stage segments so that memory stays
    bounded.  Returns (dL/dZ_in, dL/dv, dL/dtau) for L = <G, Z_out> (complex:
    L = Re sum conj(G) Z_out, conjugate-Wirtinger gradients)."""
    import torch
    from torch.utils.checkpoint import checkpoint
    dev = Z.device
    n, nev = Z.shape
    import paper_2002_10991_amd as T
    off = T.trbt_stage_offsets(n, nbw)
    # per stage: padded row indices (S_s, nbw); row n is a zero dummy row
    idx, lens = [], []
    for s in range(n - 2):
        S = int(off[s + 1] - off[s])
        r0 = s + 1 + nbw * np.arange(S)
        rows = r0[:, None] + np.arange(nbw)[None, :]
        rows[rows >= n] = n
        idx.append(torch.from_numpy(rows).to(dev))
    Zin = Z.detach().clone().requires_grad_(True)
    Vg = V.detach().clone().requires_grad_(True)
    tg = tau.detach().clone().requires_grad_(True)

    def stage(Zp, s):
        rows = idx[s]
        a, b = int(off[s]), int(off[s + 1])
        v = Vg[a:b]                                       # (S, nbw), zero beyond len
        W = Zp[rows.reshape(-1)].reshape(rows.shape[0], nbw, nev)
        vh = v.conj() if v.is_complex() else v
        d = torch.bmm(vh.unsqueeze(1), W)                 # (S, 1, nev): v^H W
        W2 = W - tg[a:b, None, None] * v.unsqueeze(2) * d
        return Zp.index_copy(0, rows.reshape(-1), W2.reshape(-1, nev))

    def segment(Zp, s_hi, s_lo):
        for s in range(s_hi, s_lo - 1, -1):
            Zp = stage(Zp, s)
        return Zp

    Zp = torch.cat([Zin, torch.zeros(1, nev, dtype=Z.dtype, device=dev)], 0)
    s = n - 3
    while s >= 0:
        lo = max(s - 15, 0)
        Zp = checkpoint(segment, Zp, s, lo, use_reentrant=False)
        s = lo - 1
    loss = torch.real((Zp[:n] * G.conj()).sum()) if Z.is_complex() else (Zp[:n] * G).sum()
    loss.backward()
    return Zin.grad, Vg.grad, tg.grad


def adjoint_leg(warmup: int, plain: bool = True):
    """Forward plus hand-written adjoint (checkpoints every 16 stages) against
    the plain form, on the differentiation workload: real, n=4096, nbw=64,
    nev=2048, G ~ N(0,1) (seed 2005)."""
    import torch
    import paper_2002_10991_amd as T
    import synth
    dev = torch.device("cuda:0")
    n, nbw, nev = 4096, 64, 2048
    lengths = synth.reflector_lengths(n, nbw)
    V, tau = synth.unitary_reflectors(lengths, nbw, 1005, "d")
    Zh = synth.gaussian(n, nev, 1006, "d")
    Gh = synth.gaussian(n, nev, 2005, "d")
    L = int(lengths.sum())
    Vd, td = torch.from_numpy(V).to(dev), torch.from_numpy(tau).to(dev)
    Zbuf = torch.from_numpy(np.ascontiguousarray(Zh.T)).to(dev)    # (nev, n): column-major Z
    Gsrc = torch.from_numpy(np.ascontiguousarray(Gh.T)).to(dev)
    Obuf, Gbuf = torch.empty_like(Zbuf), torch.empty_like(Gsrc)
    K = len(tau)
    dv = torch.empty(K, nbw, dtype=torch.float64, device=dev)
    dt = torch.empty(K, dtype=torch.float64, device=dev)
    fw = T.alloc_workspace(n, nbw, nev, False, dev)
    fwb = fw.numel()
    nb = T.trbt_adjoint_workspace_bytes_d(n, nbw, nev)
    abuf = torch.empty(nb + T.TRBT_WORK_ALIGN, dtype=torch.uint8, device=dev)
    aw = abuf[(-abuf.data_ptr()) % T.TRBT_WORK_ALIGN:][:nb]
    stream = torch.cuda.current_stream()

    def ours():
        # what the autograd wrapper runs: the checkpointing forward, then the
        # backward pass from its checkpoints
        Obuf.copy_(Zbuf)
        Gbuf.copy_(Gsrc)
        rc = T.trans_ev_tridi_to_band_fwd_ckpt_d(n, nbw, nev, Vd, td, Obuf, n, 16, aw, nb, stream)
        rc = rc or T.trans_ev_tridi_to_band_bwd_ckpt_d(n, nbw, nev, Vd, td, Gbuf, n, dv, dt, 16,
                                                       aw, nb, stream)
        if rc:
            raise T.TrbtError(rc, "adjoint leg")

    def one_call():
        # plain forward, then the one-call adjoint (which recomputes the forward)
        Obuf.copy_(Zbuf)
        Gbuf.copy_(Gsrc)
        rc = T.trans_ev_tridi_to_band_d(n, nbw, nev, Vd, td, Obuf, n, fw, fwb, stream)
        rc = rc or T.trans_ev_tridi_to_band_adjoint_d(n, nbw, nev, Vd, td, Zbuf, n, Gbuf, n, dv,
                                                      dt, 16, aw, nb, stream)
        if rc:
            raise T.TrbtError(rc, "adjoint leg")

    def timed(fn, reps=3):
        for _ in range(max(warmup, 1)):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        if T.trbt_work_check(aw):
            raise RuntimeError("adjoint: device wait-timeout flag set")
        return e0.elapsed_time(e1) / reps

    one_ms = timed(one_call)
    log(f"C5 forward + one-call adjoint: {one_ms:.2f} ms")
    ours_ms = timed(ours)
    log(f"C5 checkpointing forward + backward: {ours_ms:.2f} ms")
    flops = 18 * L * nev
    out = {
        "workload": "C5: real, n=4096, nbw=64, nev=2048, forward + adjoint, checkpoints every "
                    "16 stages, G ~ N(0,1) seed 2005",
        "flops_counted": flops,
        "ours_ms": round(ours_ms, 3),
        "ours_tflops": round(flops / ours_ms / 1e9, 4),
        "ours_form": "trans_ev_tridi_to_band_fwd_ckpt_d + trans_ev_tridi_to_band_bwd_ckpt_d",
        "forward_plus_one_call_adjoint_ms": round(one_ms, 3),
    }
    if not plain:
        return out
    t = time.perf_counter()
    pz, pv, pt = plain_adjoint(Zbuf.t(), Gsrc.t(), Vd, td, nbw)
    torch.cuda.synchronize()
    plain_ms = (time.perf_counter() - t) * 1e3
    log(f"C5 plain form: {plain_ms:.1f} ms")

    def rel(a, b):
        return float(torch.linalg.norm(a - b) / torch.linalg.norm(b))

    out.update({
        "plain_ms": round(plain_ms, 1),
        "speedup_vs_plain": round(plain_ms / ours_ms, 2),
        "plain_form": "eager PyTorch autograd, one batched op per stage, torch.utils.checkpoint "
                      "every 16 stages",
        "max_rel_diff_vs_plain": {"dZ_in": rel(Gbuf.t(), pz), "dv": rel(dv, pv),
                                  "dtau": rel(dt, pt)},
    })
    return out


def adjoint_complex_leg(warmup: int, plain: bool = True):
    """The complex variant of the differentiation workload (n=4096, nbw=64,
    nev=2048, complex Hermitian reflectors and Z, G seed 2005): the
    checkpointing forward + backward pair, and the forward plus the one-call
    complex adjoint, against the plain form."""
    import torch
    import paper_2002_10991_amd as T
    import synth
    dev = torch.device("cuda:0")
    n, nbw, nev = 4096, 64, 2048
    lengths = synth.reflector_lengths(n, nbw)
    V, tau = synth.unitary_reflectors(lengths, nbw, 1005, "z")
    Zh = synth.gaussian(n, nev, 1006, "z")
    Gh = synth.gaussian(n, nev, 2005, "z")
    L = int(lengths.sum())
    Vd, td = torch.from_numpy(V).to(dev), torch.from_numpy(tau).to(dev)
    Zbuf = torch.from_numpy(np.ascontiguousarray(Zh.T)).to(dev)
    Gsrc = torch.from_numpy(np.ascontiguousarray(Gh.T)).to(dev)
    Obuf, Gbuf = torch.empty_like(Zbuf), torch.empty_like(Gsrc)
    K = len(tau)
    dv = torch.empty(K, nbw, dtype=torch.complex128, device=dev)
    dt = torch.empty(K, dtype=torch.complex128, device=dev)
    fw = T.alloc_workspace(n, nbw, nev, True, dev)
    nb = T.trbt_adjoint_workspace_bytes_z(n, nbw, nev)
    abuf = torch.empty(nb + T.TRBT_WORK_ALIGN, dtype=torch.uint8, device=dev)
    aw = abuf[(-abuf.data_ptr()) % T.TRBT_WORK_ALIGN:][:nb]
    stream = torch.cuda.current_stream()

    def one_call():
        Obuf.copy_(Zbuf)
        Gbuf.copy_(Gsrc)
        rc = T.trans_ev_tridi_to_band_z(n, nbw, nev, Vd, td, Obuf, n, fw, fw.numel(), stream)
        rc = rc or T.trans_ev_tridi_to_band_adjoint_z(n, nbw, nev, Vd, td, Zbuf, n, Gbuf, n, dv,
                                                      dt, 16, aw, nb, stream)
        if rc:
            raise T.TrbtError(rc, "complex adjoint leg")

    def split():
        Obuf.copy_(Zbuf)
        Gbuf.copy_(Gsrc)
        rc = T.trans_ev_tridi_to_band_fwd_ckpt_z(n, nbw, nev, Vd, td, Obuf, n, 16, aw, nb, stream)
        rc = rc or T.trans_ev_tridi_to_band_bwd_ckpt_z(n, nbw, nev, Vd, td, Gbuf, n, dv, dt, 16,
                                                       aw, nb, stream)
        if rc:
            raise T.TrbtError(rc, "complex adjoint leg (split pair)")

    def timed(f):
        for _ in range(max(warmup, 1)):
            f()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        f()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    one_ms = timed(one_call)
    log(f"C5 complex forward + one-call adjoint: {one_ms:.1f} ms")
    ms = timed(split)   # last: its gradients are the ones compared below
    log(f"C5 complex checkpointing forward + backward: {ms:.1f} ms")
    flops = 4 * 18 * L * nev
    out = {
        "workload": "C5 complex: n=4096, nbw=64, nev=2048, forward + adjoint (blocked compact-WY form), "
                    "G seed 2005",
        "flops_counted": flops, "ours_ms": round(ms, 2),
        "ours_tflops": round(flops / ms / 1e9, 4),
        "ours_form": "trans_ev_tridi_to_band_fwd_ckpt_z + trans_ev_tridi_to_band_bwd_ckpt_z",
        "forward_plus_one_call_adjoint_ms": round(one_ms, 2),
    }
    if not plain:
        return out
    t = time.perf_counter()
    pz, pv, pt = plain_adjoint(Zbuf.t(), Gsrc.t(), Vd, td, nbw)
    torch.cuda.synchronize()
    plain_ms = (time.perf_counter() - t) * 1e3
    log(f"C5 complex plain form: {plain_ms:.1f} ms")

    def rel(a, b):
        return float(torch.linalg.norm(a - b) / torch.linalg.norm(b))

    out.update({"plain_ms": round(plain_ms, 1), "speedup_vs_plain": round(plain_ms / ms, 3),
                "max_rel_diff_vs_plain": {"dZ_in": rel(Gbuf.t(), pz), "dv": rel(dv, pv),
                                          "dtau": rel(dt, pt)}})
    return out


def chase_flops(n: int, b: int, cplx: bool) -> float:
    """Algorithmic FP64 flops of the bulge chase: per step, the reflector
    (~3 len), the left-block update (4 len per column), p = A v and the
    rank-2 update of the Hermitian diagonal block (4 len^2) and the right
    block's M v and rank-1 update (4 len nr); complex arithmetic x4."""
    tot = 0.0
    for s in range(n - 2):
        S = (n - s - 2 + b - 1) // b if b > 1 else 0
        r0 = s + 1 + b * np.arange(S, dtype=np.float64)
        ln = np.minimum(b, n - r0)
        nr = np.clip(n - r0 - ln, 0, b)
        nl = np.where(np.arange(S) == 0, 0, b - 1)
        tot += float(np.sum(3 * ln + 4 * ln * nl + 4 * ln * ln + 4 * ln * nr))
    return tot * (4 if cplx else 1)


def chase_leg(steps: int, warmup: int, cpu: bool = True):
    """Banded-to-tridiagonal bulge chasing on the GPU (the producer of the
    reflectors) on the bands of the n = 32768 complex and n = 8192 real
    workloads; the oracle's sequential chase timed on an n = 2048 sample of
    the same bandwidth and scaled by the flop count."""
    import torch
    import synth
    import paper_2002_10991_amd as T
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    res = {}
    for label, n, b, dt, seed, shift in (("C3 band", 32768, 64, "z", 1003, False),
                                         ("C2 band", 8192, 64, "d", 1002, True)):
        cplx = dt == "z"
        tdt = torch.complex128 if cplx else torch.float64
        ab = synth.band_matrix(n, b, seed, dt, diag_shift=shift)
        abd = torch.from_numpy(np.ascontiguousarray(ab.T)).to(dev)
        K = T.trbt_num_reflectors(n, b)
        d = torch.empty(n, dtype=torch.float64, device=dev)
        e = torch.empty(n - 1, dtype=tdt, device=dev)
        hv = torch.empty((K, b), dtype=tdt, device=dev)
        ht = torch.empty(K, dtype=tdt, device=dev)
        nb = T.trbt_band_to_tridi_workspace_bytes(n, b, cplx)
        buf = torch.empty(nb + T.TRBT_WORK_ALIGN, dtype=torch.uint8, device=dev)
        off = (-buf.data_ptr()) % T.TRBT_WORK_ALIGN
        work = buf[off: off + nb]
        f = T.trbt_band_to_tridi_z if cplx else T.trbt_band_to_tridi_d

        def run():
            rc = f(n, b, abd, b + 1, d, e, hv, ht, work, nb, stream)
            if rc:
                raise T.TrbtError(rc, f.__name__)

        for _ in range(warmup):
            run()
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(steps)]
        for e0, e1 in evs:
            e0.record(stream)
            run()
            e1.record(stream)
        torch.cuda.synchronize()
        if not bool(torch.isfinite(d).all()):
            raise RuntimeError("bulge chase: a pipeline wait timed out")
        ts = [a.elapsed_time(z) for a, z in evs]
        ms = float(np.mean(ts))
        fl = chase_flops(n, b, cplx)
        period = n - 2 + n - 2 + (n - 2 + b - 1) // b     # 2 steps per stage + the first stage
        r = {"n": n, "nbw": b, "dtype": "c128" if cplx else "f64", "reflectors": K,
             "ms": round(ms, 3), "ms_min": round(min(ts), 3),
             "pipeline_step_us": round(ms * 1e3 / period, 3),
             "achieved_tflops": round(fl / (ms / 1e3) / 1e12, 4),
             "peak_fp64_tflops": PEAK_FP64_TFLOPS}
        if cpu:
            import oracle
            ns = 2048
            abs_ = synth.band_matrix(ns, b, seed, dt, diag_shift=shift)
            t = time.perf_counter()
            oracle.band_to_tridiagonal(abs_, b)
            cs = time.perf_counter() - t
            est = cs * fl / chase_flops(ns, b, cplx)
            r["cpu_oracle"] = {"sample": f"n={ns}, nbw={b}, same dtype; scaled by the flop count",
                               "sample_s": round(cs, 3), "extrapolated_s": round(est, 1),
                               "cores": 1, "kind": "oracle"}
            r["speedup_vs_oracle"] = round(est / (ms / 1e3), 1)
        log(f"chase {label}: {ms:.1f} ms")
        res[label] = r
    return res


def tridiag_leg(steps: int, warmup: int, cpu: bool = True):
    """The lowest nev eigenpairs of the tridiagonal T that the GPU chase makes
    of the n = 8192 real and n = 32768 complex workloads' bands, by bisection and
    inverse iteration on the GPU (complex: Re e with the last entry |e[n-2]|);
    the oracle's implicit QL (all eigenpairs,
    O(n^3)) timed on an n = 1024 sample and scaled by n^3."""
    import torch
    import synth
    import paper_2002_10991_amd as T
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    res = {}
    for label, n, nev, dt, seed, shift in (("C2", 8192, 4096, "d", 1002, True),
                                           ("C3", 32768, 8192, "z", 1003, False)):
        ab = synth.band_matrix(n, 64, seed, dt, diag_shift=shift)
        d, e, _, _ = T.band_to_tridiagonal(torch.from_numpy(np.ascontiguousarray(ab.T)).to(dev),
                                           64)
        if dt == "z":   # real betas except the last subdiagonal: T = D T_r D^H
            er = e.real.clone()
            er[-1] = e[-1].abs()
            e = er
        e = e.to(torch.float64).contiguous()
        w = torch.empty(nev, dtype=torch.float64, device=dev)
        zb = torch.empty((nev, n), dtype=torch.float64, device=dev)
        nb = T.trbt_tridiag_eigh_workspace_bytes(n, nev)
        buf = torch.empty(nb + T.TRBT_WORK_ALIGN, dtype=torch.uint8, device=dev)
        work = buf[(-buf.data_ptr()) % T.TRBT_WORK_ALIGN:][:nb]

        def run():
            rc = T.trbt_tridiag_eigh_d(n, nev, d, e, w, zb, n, work, nb, stream)
            if rc:
                raise T.TrbtError(rc, "trbt_tridiag_eigh_d")

        for _ in range(max(warmup, 1)):
            run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            run()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        r = {"n": n, "nev": nev, "ms": round(ms, 3),
             "input": f"T from the GPU chase of the {label} band (nbw=64)"}
        if cpu:
            import oracle
            ns = 1024
            rng = np.random.default_rng(5)
            t = time.perf_counter()
            oracle.tridiagonal_eigh(rng.standard_normal(ns), rng.standard_normal(ns - 1))
            cs = time.perf_counter() - t
            est = cs * (n / ns) ** 3
            r["cpu_oracle"] = {"sample": f"implicit QL, all eigenpairs, n={ns}; scaled by n^3",
                               "sample_s": round(cs, 3), "extrapolated_s": round(est, 1),
                               "cores": oracle.num_threads(), "kind": "oracle"}
            r["speedup_vs_oracle"] = round(est / (ms / 1e3), 1)
        log(f"tridiagonal eigenpairs {label}: {ms:.1f} ms")
        res[label] = r
    return res


def b2f_leg(steps: int, warmup: int, cpu: bool = True):
    """The band-to-full back-transformation C = P^* Y (Eq. 2stage_bkwd2), the
    step after the headline one, on the same problem shapes: complex
    n = 32768, nbw = 64, nev = 8192 and real n = 8192, nbw = 64, nev = 4096,
    with seeded synthetic stage-1 reflectors (one per column, rows
    [j+nbw, n)) and a Gaussian Y; the oracle timed on a column sample."""
    import torch
    import synth
    import paper_2002_10991_amd as T
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    res = {}
    for label, n, nev, dt, seed in (("complex n=32768", 32768, 8192, "z", 5006),
                                    ("real n=8192", 8192, 4096, "d", 5005)):
        nbw = 64
        cplx = dt == "z"
        t = time.perf_counter()
        V, tau = synth.full_unitary_reflectors(n, nbw, seed, dt)
        Y = synth.gaussian(n, nev, 5007, dt)
        log(f"band_to_full {label}: inputs ready in {time.perf_counter() - t:.1f}s")
        vb = torch.from_numpy(np.ascontiguousarray(V.T)).to(dev)
        td = torch.from_numpy(tau).to(dev)
        zb = torch.from_numpy(np.ascontiguousarray(Y.T)).to(dev)
        nb = T.trbt_band_to_full_workspace_bytes(n, nbw, nev, cplx)
        buf = torch.empty(nb + T.TRBT_WORK_ALIGN, dtype=torch.uint8, device=dev)
        work = buf[(-buf.data_ptr()) % T.TRBT_WORK_ALIGN:][:nb]
        f = T.trans_ev_band_to_full_z if cplx else T.trans_ev_band_to_full_d

        def run():
            rc = f(n, nbw, nev, vb, n, td, zb, n, work, nb, stream)
            if rc:
                raise T.TrbtError(rc, f.__name__)

        for _ in range(max(warmup, 1)):
            run()
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(steps)]
        for e0, e1 in evs:
            e0.record(stream)
            run()
            e1.record(stream)
        torch.cuda.synchronize()
        ts = [a.elapsed_time(z) for a, z in evs]
        ms = float(np.mean(ts))
        m = n - nbw
        L1 = m * (m + 1) // 2 - 1            # sum of the reflector lengths, 2 .. n-nbw
        flops = (16 if cplx else 4) * nev * L1
        r = {"n": n, "nbw": nbw, "nev": nev, "dtype": "c128" if cplx else "f64",
             "reflectors": int(len(tau)), "ms": round(ms, 3), "ms_min": round(min(ts), 3),
             "flops": flops, "achieved_tflops": round(flops / (ms / 1e3) / 1e12, 4),
             "frac_fp64_peak": round(flops / (ms / 1e3) / 1e12 / PEAK_FP64_TFLOPS, 4),
             "kernels": "k_b2f_tfac (compact-WY factors) + k_b2f_apply, per call",
             "inputs": "synthetic unitary stage-1 reflectors + Gaussian Y, seeded"}
        if cpu:
            import oracle
            ncols = 2 * oracle.num_threads()
            cols = np.linspace(0, nev - 1, ncols).astype(np.int64)
            t = time.perf_counter()
            oracle.back_transform_full(Y, V, tau, nbw, cols=cols)
            cs = time.perf_counter() - t
            rate = (16 if cplx else 4) * L1 * ncols / cs
            r["cpu_baseline"] = {"value": round(rate / 1e12, 6), "unit": "TFLOP/s",
                                 "cores": oracle.num_threads(), "kind": "oracle",
                                 "sample": f"{ncols} of {nev} columns, all reflectors, "
                                           f"{cs:.1f} s wall"}
            r["speedup_vs_oracle"] = round(flops / (ms / 1e3) / rate, 1)
        log(f"band_to_full {label}: {ms:.2f} ms, {r['achieved_tflops']} TFLOP/s")
        res[label] = r
        del vb, zb, buf, work, V, Y
        torch.cuda.empty_cache()
    return res


def shapes_leg(steps: int, warmup: int, names=("C1", "C2", "C3s", "C3w")):
    """The other single-problem shapes, each timed like the headline step
    (prepare + apply through the C ABI, HIP events on the stream): the two
    real workloads (C1 n=1024 nbw=32 nev=1024, C2 n=8192 nbw=64 nev=4096),
    one GPU's column share of the headline shape split over eight (C3s,
    nev=1024) and the headline size with nbw=128 (C3w).  Roofline of the
    apply kernel against the FP64 peak; algorithmic flops c*nev*L."""
    import torch
    import paper_2002_10991_amd as T
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    res = {}
    for name in names:
        cfg = WORKLOADS[name]
        n, nbw, nev, dt = cfg["n"], cfg["nbw"], cfg["nev"], cfg["dtype"]
        cplx = dt == "z"
        t = time.perf_counter()
        lengths, V, tau, Z = make_inputs(cfg)
        L_total = int(lengths.sum())
        Vd = torch.from_numpy(V).to(dev)
        td = torch.from_numpy(tau).to(dev)
        Zbuf = torch.from_numpy(np.ascontiguousarray(Z.T)).to(dev)
        del V, Z
        work = T.alloc_workspace(n, nbw, nev, cplx, dev)
        wb = 0 if work is None else work.numel()
        prep = T.trbt_prepare_z if cplx else T.trbt_prepare_d
        appl = T.trbt_apply_z if cplx else T.trbt_apply_d
        log(f"shape {name}: inputs ready in {time.perf_counter() - t:.1f}s")

        def step(ev=None):
            if ev:
                ev[0].record(stream)
            if prep(n, nbw, Vd, td, work, wb, stream):
                raise RuntimeError(f"{name}: prepare failed")
            if ev:
                ev[1].record(stream)
            if appl(n, nbw, nev, Vd, td, Zbuf, n, work, wb, stream):
                raise RuntimeError(f"{name}: apply failed")
            if ev:
                ev[2].record(stream)

        for _ in range(max(warmup, 1)):
            step()
        torch.cuda.synchronize()
        k = max(steps, 3)
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(k)]
        t0 = time.perf_counter()
        for e in evs:
            step(e)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / k * 1e3
        if work is not None and T.trbt_work_check(work):
            raise RuntimeError(f"{name}: device wait-timeout flag set")
        apply_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
        flops = (16 if cplx else 4) * nev * L_total
        strips = -(-nev // 16)
        res[name] = {
            "n": n, "nbw": nbw, "nev": nev, "dtype": "c128" if cplx else "f64",
            "ms_per_step": round(ms, 3), "apply_ms": round(apply_ms, 3),
            "tflops_per_step": round(flops / (ms / 1e3) / 1e12, 4),
            "roofline": {"bound": "mfma",
                         "achieved": round(flops / (apply_ms / 1e3) / 1e12, 4),
                         "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(flops / (apply_ms / 1e3) / 1e12 / PEAK_FP64_TFLOPS, 4),
                         "kernel": "k_blocked (apply)"},
            "column_strips": strips,
        }
        log(f"shape {name}: {ms:.3f} ms per step, apply {apply_ms:.3f} ms, "
            f"{res[name]['roofline']['achieved']} TFLOP/s")
        del Vd, td, Zbuf, work
        torch.cuda.empty_cache()
    return res


def committed_traffic(workload: str):
    """HBM bytes per launch of the apply kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel source; else None."""
    import hashlib
    prof = os.path.join(ROOT, "profiles", f"k_blocked_{workload}.md")
    if not os.path.exists(prof):
        return None
    text = open(prof).read()
    h = hashlib.sha256()
    for f in ("trbt_device.h", "trbt.hip"):   # the apply kernel's sources
        h.update(open(os.path.join(ROOT, "paper_2002_10991_amd", "csrc", f), "rb").read())
    sha = h.hexdigest()
    if f"source_sha256: {sha}" not in text:
        return None
    for line in text.splitlines():
        if line.startswith("traffic_bytes_per_launch:"):
            return float(line.split(":", 1)[1])
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="C3", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-shapes", action="store_true",
                    help="skip the other single-problem shapes (C1, C2, C3s, C3w)")
    ap.add_argument("--shapes-only", action="store_true",
                    help="only the other single-problem shapes")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched-vs-looped comparison on the 64-problem workload")
    ap.add_argument("--batched-only", action="store_true",
                    help="run only the batched-vs-looped comparison and print its JSON")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the adjoint-vs-plain comparison on the differentiation workload")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="run only the adjoint-vs-plain comparison and print its JSON")
    ap.add_argument("--no-tridiag", action="store_true",
                    help="skip the tridiagonal eigenpairs leg")
    ap.add_argument("--tridiag-only", action="store_true",
                    help="run only the tridiagonal eigenpairs leg and print its JSON")
    ap.add_argument("--no-chase", action="store_true",
                    help="skip the banded-to-tridiagonal bulge chasing leg")
    ap.add_argument("--chase-only", action="store_true",
                    help="run only the bulge chasing leg and print its JSON")
    ap.add_argument("--no-b2f", action="store_true",
                    help="skip the band-to-full back-transformation leg")
    ap.add_argument("--b2f-only", action="store_true",
                    help="run only the band-to-full back-transformation leg and print its JSON")
    ap.add_argument("--no-plain", action="store_true",
                    help="in the adjoint comparison, time only the hand-written adjoint")
    ap.add_argument("--copy-kernel", type=int, default=0, metavar="BYTES",
                    help="only run one plain device-to-device copy of BYTES bytes (used to "
                         "calibrate the FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.copy_kernel:
        import torch
        src = torch.ones(args.copy_kernel // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.copy_kernel}))
        return
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the back-transformation shards by eigenvector columns with no communication)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2002_10991_amd as T

    if args.batched_only:
        print(json.dumps({"batched_vs_loop": batched_leg(args.steps, args.warmup),
                          "batched_complex_vs_loop": batched_leg(args.steps, args.warmup, "z")}),
              flush=True)
        return
    if args.tridiag_only:
        print(json.dumps({"tridiag": tridiag_leg(args.steps, args.warmup,
                                                 not args.no_cpu_baseline)}), flush=True)
        return
    if args.chase_only:
        print(json.dumps({"chase": chase_leg(args.steps, args.warmup,
                                             not args.no_cpu_baseline)}), flush=True)
        return
    if args.b2f_only:
        print(json.dumps({"band_to_full": b2f_leg(args.steps, args.warmup,
                                                  not args.no_cpu_baseline)}), flush=True)
        return
    if args.shapes_only:
        print(json.dumps({"shapes": shapes_leg(args.steps, args.warmup)}), flush=True)
        return
    if args.adjoint_only:
        print(json.dumps({"adjoint_vs_plain": adjoint_leg(args.warmup, not args.no_plain),
                          "adjoint_complex_vs_plain":
                              adjoint_complex_leg(args.warmup, not args.no_plain)}),
              flush=True)
        return

    cfg = WORKLOADS[args.workload]
    n, nbw, nev, dt = cfg["n"], cfg["nbw"], cfg["nev"], cfg["dtype"]
    cplx = dt == "z"
    log(f"workload {args.workload}: n={n} nbw={nbw} nev={nev} dtype={dt}; generating inputs")
    t = time.perf_counter()
    lengths, V, tau, Z = make_inputs(cfg)
    L_total = int(lengths.sum())
    K = len(lengths)
    log(f"inputs ready in {time.perf_counter() - t:.1f}s: K={K} L={L_total}")

    dev = torch.device("cuda:0")
    Vd = torch.from_numpy(V).to(dev)
    td = torch.from_numpy(tau).to(dev)
    Zbuf = torch.from_numpy(Z.T).to(dev)          # (nev, n) rows = columns of Z
    work = T.alloc_workspace(n, nbw, nev, cplx, dev)
    wb = 0 if work is None else work.numel()
    prep = T.trbt_prepare_z if cplx else T.trbt_prepare_d
    appl = T.trbt_apply_z if cplx else T.trbt_apply_d
    stream = torch.cuda.current_stream()

    def step(evs=None):
        if evs:
            evs[0].record(stream)
        rc = prep(n, nbw, Vd, td, work, wb, stream)
        if rc:
            raise T.TrbtError(rc, "prepare")
        if evs:
            evs[1].record(stream)
        rc = appl(n, nbw, nev, Vd, td, Zbuf, n, work, wb, stream)
        if rc:
            raise T.TrbtError(rc, "apply")
        if evs:
            evs[2].record(stream)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if work is not None:
        flag = T.trbt_work_check(work)
        if flag:
            raise RuntimeError("device wait-timeout flag set")
    prep_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    apply_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
    ms = (t1 - t0) / args.steps * 1e3
    c = 16 if cplx else 4
    flops = c * nev * L_total
    value = flops / (ms / 1e3) / 1e12
    achieved = flops / (apply_ms / 1e3) / 1e12
    log(f"step {ms:.2f} ms (prepare {prep_ms:.2f} ms, apply {apply_ms:.2f} ms)")

    out = {
        "metric": "back-transform FP64 TFLOP/s & %roofline, n=32768 nev=8192; batched vs loop",
        "value": round(value, 4),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128" if cplx else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: {'complex Hermitian' if cplx else 'real symmetric'} "
                        f"tridiagonal-to-banded back-transform, n={n}, nbw={nbw}, nev={nev}",
            "n": n, "nbw": nbw, "nev": nev, "reflectors": K, "reflector_rows": L_total,
            "inputs": "synthetic unitary Householder reflectors + Gaussian Z, seeded",
            "prepare_ms": round(prep_ms, 3), "apply_ms": round(apply_ms, 3),
        },
        "roofline": {
            "bound": "mfma", "achieved": round(achieved, 4), "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_TFLOPS, 4),
            "traffic": committed_traffic(args.workload),
            "kernel": "k_blocked (apply)",
        },
    }
    if not args.no_shapes:
        out["shapes"] = shapes_leg(min(args.steps, 10), args.warmup)
    if not args.no_batched:
        out["batched_vs_loop"] = batched_leg(args.steps, args.warmup)
        out["batched_complex_vs_loop"] = batched_leg(args.steps, args.warmup, "z")
    if not args.no_adjoint:
        out["adjoint_vs_plain"] = adjoint_leg(args.warmup, not args.no_plain)
        out["adjoint_complex_vs_plain"] = adjoint_complex_leg(args.warmup, not args.no_plain)
    if not args.no_chase:
        out["chase"] = chase_leg(min(args.steps, 3), args.warmup, not args.no_cpu_baseline)
    if not args.no_b2f:
        out["band_to_full"] = b2f_leg(min(args.steps, 3), args.warmup, not args.no_cpu_baseline)
    if not args.no_tridiag:
        out["tridiag"] = tridiag_leg(min(args.steps, 3), args.warmup, not args.no_cpu_baseline)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a column sample")
        out["cpu_baseline"] = cpu_baseline(cfg, V, tau, Z, L_total)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
