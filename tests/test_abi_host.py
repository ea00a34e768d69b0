"""Host-side checks of the C ABI (no GPU needed): the library loads and
exports every function include/trbt.h declares, argument validation returns
the documented codes before anything is launched, and the host helpers agree
with the oracle's reflector geometry."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "trbt.h")


@pytest.fixture(scope="module")
def T():
    import paper_2002_10991_amd as T
    if not os.path.exists(T.LIB_PATH):
        from paper_2002_10991_amd import build
        build.build()
    T.lib()
    return T


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b([a-z_][a-z0-9_]*)\s*\(", src, re.M)
    return sorted(set(n for n in names if not n.startswith("defined")))


def test_every_declared_symbol_is_exported(T):
    names = _declared_functions()
    assert {"trans_ev_tridi_to_band_d", "trans_ev_tridi_to_band_z", "trbt_prepare_d",
            "trbt_apply_z", "trbt_workspace_bytes", "trbt_strerror"} <= set(names)
    lib = T.lib()
    for n in names:
        assert hasattr(lib, n), n


# one invalid argument per case; every earlier argument valid, so the call
# returns from host validation before any HIP call
FAKE = 4096   # never dereferenced: validation fails first


@pytest.mark.parametrize("fn", ["trans_ev_tridi_to_band_d", "trans_ev_tridi_to_band_z",
                                "trbt_apply_d", "trbt_apply_z"])
def test_argument_validation_codes(T, fn):
    f = getattr(T, fn)
    ok = dict(n=100, nbw=32, nev=10, hh_v=FAKE, hh_tau=FAKE, Z=FAKE, ldz=100, work=None, work_bytes=0)

    def call(**kw):
        a = dict(ok, **kw)
        return f(a["n"], a["nbw"], a["nev"], a["hh_v"], a["hh_tau"], a["Z"], a["ldz"],
                 a["work"], a["work_bytes"], 0)

    assert call(n=-1) == -1
    assert call(nbw=0) == -2
    assert call(nbw=257) == -2
    assert call(nev=-1) == -3
    assert call(nev=101) == -3
    assert call(hh_v=None) == -4
    assert call(hh_tau=None) == -5
    assert call(Z=None) == -6
    assert call(ldz=99) == -7
    assert call(work=FAKE + 8) == -8          # misaligned
    assert call(work=None, work_bytes=64) == -8
    # quick returns touch nothing and need no device
    assert call(nev=0, hh_v=None, hh_tau=None, Z=None) == 0
    assert call(n=2, nev=2, ldz=2) == 0
    assert call(nbw=1, hh_v=None, hh_tau=None) == 0


@pytest.mark.parametrize("fn", ["trbt_prepare_d", "trbt_prepare_z"])
def test_prepare_validation_codes(T, fn):
    f = getattr(T, fn)
    assert f(-1, 32, FAKE, FAKE, None, 0, 0) == -1
    assert f(100, 0, FAKE, FAKE, None, 0, 0) == -2
    assert f(100, 32, None, FAKE, None, 0, 0) == -3
    assert f(100, 32, FAKE, None, None, 0, 0) == -4
    assert f(100, 32, FAKE, FAKE, FAKE + 8, 64, 0) == -5
    assert f(100, 32, FAKE, FAKE, None, 0, 0) == -101     # blocked shape needs workspace
    assert f(100, 7, FAKE, FAKE, None, 0, 0) == 0         # unblocked shape: nothing to do
    assert f(2, 32, None, None, None, 0, 0) == 0


@pytest.mark.parametrize("n,nbw", [(17, 4), (300, 7), (1000, 64), (3, 2), (5, 1), (64, 8)])
def test_geometry_helpers_match_oracle(T, oracle_mod, n, nbw):
    K = T.trbt_num_reflectors(n, nbw)
    assert K == oracle_mod.num_reflectors(n, nbw)
    off = T.trbt_stage_offsets(n, nbw)
    expect = np.zeros(n - 1, np.int64)
    for s in range(n - 2):
        expect[s + 1] = expect[s] + oracle_mod.sweeps_in_stage(n, nbw, s)
    assert np.array_equal(off, expect)
    assert off[-1] == K


def test_workspace_query(T):
    assert T.trbt_workspace_bytes(1000, 7, 100, False) == 0
    assert T.trbt_workspace_bytes(1000, 64, 0, True) == 0
    a = T.trbt_workspace_bytes(1000, 64, 100, False)
    b = T.trbt_workspace_bytes(1000, 64, 100, True)
    c = T.trbt_workspace_bytes(2000, 64, 100, True)
    assert 0 < a < b < c
    assert T.trbt_workspace_bytes(1000, 64, 5, True) == b     # independent of nev > 0
    with pytest.raises(T.TrbtError):
        T.trbt_workspace_bytes(10, 300, 1, False)


@pytest.mark.parametrize("n,nbw", [(1000, 64), (2000, 32), (777, 48), (300, 16), (66, 64),
                                   (1000, 128), (500, 80)])
@pytest.mark.parametrize("nev_frac", [0, 3])
def test_workspace_size_is_the_packed_layout(T, oracle_mod, n, nbw, nev_frac):
    """Blocked shapes: a 256-byte header plus, for every (slot j, 16-stage
    block t >= j*nbw/16), the two MFMA operand matrices of the block's
    compact-WY factor, (nbw+16) x 16 each, one plane real, two complex;
    then the slot-group progress counters, 8 ints for each 16-column strip
    and for 8 strips of padding, rounded up to 256 bytes."""
    nev = n // nev_frac if nev_frac else 10
    st = oracle_mod.reflector_table(n, nbw)[0]
    J = int(np.sum(st == 0))                   # slots of stage 0
    nblk = -(-(n - 2) // 16)
    nblocks = sum(nblk - j * (nbw // 16) for j in range(J))
    counters = -(-((-(-nev // 16) + 8) * 8 * 4) // 256) * 256
    for cplx, planes in ((False, 1), (True, 2)):
        expect = 256 + nblocks * 2 * (nbw + 16) * 16 * planes * 8 + counters
        assert T.trbt_workspace_bytes(n, nbw, nev, cplx) == expect, (n, nbw, cplx)


def test_strerror(T):
    assert T.trbt_strerror(0) == "success"
    assert "gfx950" in T.trbt_strerror(-100)
    assert "workspace" in T.trbt_strerror(-101)
    assert "argument" in T.trbt_strerror(-3)


def test_plan_validation_codes(T):
    """Batched plan creation rejects bad arguments on the host, before any
    HIP call: -1 probs, -2 count, -3 configuration, -4 plan, and
    TRBT_ERR_PROBLEM(i) = -(1000 + i) for the first bad descriptor."""
    import ctypes as C
    lib = T.lib()
    good = T.trbt_problem_d(100, 32, 10, FAKE, FAKE, FAKE, 100)
    arr = (T.trbt_problem_d * 3)(good, good, good)
    h = C.c_void_p()
    assert lib.trbt_plan_create_batched_d(None, 2, None, C.byref(h), None) == -1
    assert lib.trbt_plan_create_batched_d(arr, -1, None, C.byref(h), None) == -2
    for bad in [(8, 8, 16), (16, 6, 16), (16, 8, 4), (48, 8, 16)]:
        cfg = T.trbt_plan_config(*bad)
        assert lib.trbt_plan_create_batched_d(arr, 3, C.byref(cfg), C.byref(h), None) == -3
    assert lib.trbt_plan_create_batched_d(arr, 3, None, None, None) == -4
    for i, bad in [(0, dict(n=-1)), (1, dict(nev=101)), (2, dict(ldz=50)),
                   (1, dict(hh_v=None)), (2, dict(nbw=0)), (0, dict(Z=None))]:
        fields = dict(n=100, nbw=32, nev=10, hh_v=FAKE, hh_tau=FAKE, Z=FAKE, ldz=100)
        fields.update(bad)
        a = (T.trbt_problem_d * 3)(good, good, good)
        a[i] = T.trbt_problem_d(**fields)
        h = C.c_void_p(1234)
        assert lib.trbt_plan_create_batched_d(a, 3, None, C.byref(h), None) == -1000 - i
        assert h.value is None
    assert lib.trbt_plan_exec(None, None) == -1
    assert lib.trbt_plan_get_config(None, None, None) == -1
    assert lib.trbt_plan_destroy(None) == 0


def test_complex_plan_validation_codes(T):
    """Complex plans: the same host-side checks, and 32-column strips are
    not a complex configuration (-3)."""
    import ctypes as C
    lib = T.lib()
    good = T.trbt_problem_z(100, 32, 10, FAKE, FAKE, FAKE, 100)
    arr = (T.trbt_problem_z * 2)(good, good)
    h = C.c_void_p()
    assert lib.trbt_plan_create_batched_z(None, 2, None, C.byref(h), None) == -1
    assert lib.trbt_plan_create_batched_z(arr, -1, None, C.byref(h), None) == -2
    for bad in [(32, 8, 16), (32, 4, 1), (16, 6, 16)]:
        cfg = T.trbt_plan_config(*bad)
        assert lib.trbt_plan_create_batched_z(arr, 2, C.byref(cfg), C.byref(h), None) == -3
    assert lib.trbt_plan_create_batched_z(arr, 2, None, None, None) == -4
    bad = T.trbt_problem_z(100, 32, 10, FAKE, FAKE, FAKE, 50)   # ldz < n
    arr2 = (T.trbt_problem_z * 2)(good, bad)
    assert lib.trbt_plan_create_batched_z(arr2, 2, None, C.byref(h), None) == -1001
    assert h.value is None


@pytest.mark.parametrize("sfx", ["d", "z"])
def test_adjoint_validation_codes(T, sfx):
    """The adjoint entry points check their 15 arguments on the host, in
    order, before any HIP call."""
    f = getattr(T, "trans_ev_tridi_to_band_adjoint_" + sfx)
    wsb = getattr(T, "trbt_adjoint_workspace_bytes_" + sfx)
    ok = dict(n=100, nbw=32, nev=10, hh_v=FAKE, hh_tau=FAKE, Z_in=FAKE, ldz=100, G=FAKE, ldg=100,
              dv=FAKE, dtau=FAKE, ckpt=16, work=None, wb=0)

    def call(**kw):
        a = dict(ok, **kw)
        return f(a["n"], a["nbw"], a["nev"], a["hh_v"], a["hh_tau"], a["Z_in"], a["ldz"], a["G"],
                 a["ldg"], a["dv"], a["dtau"], a["ckpt"], a["work"], a["wb"], 0)

    assert call(n=-1) == -1
    assert call(nbw=0) == -2
    assert call(nev=101) == -3
    assert call(hh_v=None) == -4
    assert call(hh_tau=None) == -5
    assert call(Z_in=None) == -6
    assert call(ldz=99) == -7
    assert call(G=None) == -8
    assert call(ldg=50) == -9
    assert call(dv=None) == -10
    assert call(dtau=None) == -11
    assert call(ckpt=8) == -12
    assert call(work=FAKE + 8) == -13
    assert call(work=None, wb=64) == -13
    assert call(nbw=1, hh_v=None, hh_tau=None, dv=None, dtau=None) == 0   # K == 0: no-op
    assert wsb(100, 32, 10, 16) > 0
    assert wsb(100, 32, 0, 16) == 0
    assert wsb(100, 1, 10, 16) == 0
    for bad, code in [((-1, 32, 10, 16), -1), ((100, 0, 10, 16), -2), ((100, 32, 200, 16), -3),
                      ((100, 32, 10, 5), -4)]:
        with pytest.raises(T.TrbtError) as e:
            wsb(*bad)
        assert e.value.status == code


def test_split_adjoint_validation_codes(T):
    """The checkpointing forward and the backward-from-checkpoints entries
    validate on the host, in argument order, before any HIP call."""
    fw = T.trans_ev_tridi_to_band_fwd_ckpt_d
    okf = dict(n=100, nbw=32, nev=10, hv=FAKE, ht=FAKE, Z=FAKE, ldz=100, ck=16, work=None, wb=0)

    def callf(**kw):
        a = dict(okf, **kw)
        return fw(a["n"], a["nbw"], a["nev"], a["hv"], a["ht"], a["Z"], a["ldz"], a["ck"],
                  a["work"], a["wb"], 0)

    assert callf(n=-1) == -1
    assert callf(nbw=300) == -2
    assert callf(nev=-2) == -3
    assert callf(hv=None) == -4
    assert callf(ht=None) == -5
    assert callf(Z=None) == -6
    assert callf(ldz=10) == -7
    assert callf(ck=32) == -8
    assert callf(work=FAKE + 4) == -9
    assert callf(nev=0, hv=None, ht=None, Z=None) == 0
    bw = T.trans_ev_tridi_to_band_bwd_ckpt_d
    okb = dict(n=100, nbw=32, nev=10, hv=FAKE, ht=FAKE, G=FAKE, ldg=100, dv=FAKE, dt=FAKE, ck=16,
               work=None, wb=0)

    def callb(**kw):
        a = dict(okb, **kw)
        return bw(a["n"], a["nbw"], a["nev"], a["hv"], a["ht"], a["G"], a["ldg"], a["dv"],
                  a["dt"], a["ck"], a["work"], a["wb"], 0)

    assert callb(n=-1) == -1
    assert callb(nbw=0) == -2
    assert callb(nev=101) == -3
    assert callb(hv=None) == -4
    assert callb(ht=None) == -5
    assert callb(G=None) == -6
    assert callb(ldg=99) == -7
    assert callb(dv=None) == -8
    assert callb(dt=None) == -9
    assert callb(ck=1) == -10
    assert callb(work=None, wb=8) == -11
    assert callb(nbw=1, hv=None, ht=None, dv=None, dt=None) == 0


def test_complex_split_adjoint_validation_codes(T):
    """The complex pair validates like the real one, and rejects band widths
    without blocked kernels with -2, all before any HIP call."""
    fw = T.trans_ev_tridi_to_band_fwd_ckpt_z
    okf = dict(n=100, nbw=32, nev=10, hv=FAKE, ht=FAKE, Z=FAKE, ldz=100, ck=16, work=None, wb=0)

    def callf(**kw):
        a = dict(okf, **kw)
        return fw(a["n"], a["nbw"], a["nev"], a["hv"], a["ht"], a["Z"], a["ldz"], a["ck"],
                  a["work"], a["wb"], 0)

    assert callf(n=-1) == -1
    for nbw in (0, 8, 24, 80, 128, 300):
        assert callf(nbw=nbw) == -2
    assert callf(nev=-2) == -3
    assert callf(hv=None) == -4
    assert callf(ht=None) == -5
    assert callf(Z=None) == -6
    assert callf(ldz=10) == -7
    assert callf(ck=32) == -8
    assert callf(work=FAKE + 4) == -9
    assert callf(nev=0, hv=None, ht=None, Z=None) == 0
    bw = T.trans_ev_tridi_to_band_bwd_ckpt_z
    okb = dict(n=100, nbw=32, nev=10, hv=FAKE, ht=FAKE, G=FAKE, ldg=100, dv=FAKE, dt=FAKE, ck=16,
               work=None, wb=0)

    def callb(**kw):
        a = dict(okb, **kw)
        return bw(a["n"], a["nbw"], a["nev"], a["hv"], a["ht"], a["G"], a["ldg"], a["dv"],
                  a["dt"], a["ck"], a["work"], a["wb"], 0)

    assert callb(n=-1) == -1
    for nbw in (0, 1, 8, 96):
        assert callb(nbw=nbw) == -2
    assert callb(nev=101) == -3
    assert callb(hv=None) == -4
    assert callb(ht=None) == -5
    assert callb(G=None) == -6
    assert callb(ldg=99) == -7
    assert callb(dv=None) == -8
    assert callb(dt=None) == -9
    assert callb(ck=1) == -10
    assert callb(work=None, wb=8) == -11
    assert callb(n=2, hv=None, ht=None, dv=None, dt=None, G=None, ldg=2, nev=1) == 0


@pytest.mark.parametrize("fn", ["trbt_band_to_tridi_d", "trbt_band_to_tridi_z"])
def test_band_to_tridi_validation_codes(T, fn):
    f = getattr(T, fn)
    ok = dict(n=100, nbw=32, ab=FAKE, ldab=33, d=FAKE, e=FAKE, hh_v=FAKE, hh_tau=FAKE,
              work=None, work_bytes=0)

    def call(**kw):
        a = dict(ok, **kw)
        return f(a["n"], a["nbw"], a["ab"], a["ldab"], a["d"], a["e"], a["hh_v"], a["hh_tau"],
                 a["work"], a["work_bytes"], 0)

    assert call(n=-1) == -1
    assert call(nbw=0) == -2
    assert call(nbw=65) == -2          # the chase keeps one block column per lane
    assert call(ab=None) == -3
    assert call(ldab=32) == -4
    assert call(d=None) == -5
    assert call(e=None) == -6
    assert call(hh_v=None) == -7
    assert call(hh_tau=None) == -8
    assert call(work=FAKE + 8, work_bytes=1 << 20) == -9
    assert call() == -101                              # TRBT_ERR_WORKSPACE: none given
    assert call(work=FAKE, work_bytes=1024) == -101    # too small
    # nothing to annihilate: no reflector buffers needed; n = 0 returns at once
    assert call(n=0, ab=None, d=None, e=None, hh_v=None, hh_tau=None) == 0
    assert call(n=50, nbw=1, ldab=2, hh_v=None, hh_tau=None) == -101   # only the workspace missing


@pytest.mark.parametrize("n,nbw", [(1, 1), (17, 4), (1000, 64), (32768, 64)])
def test_band_to_tridi_workspace_formula(T, n, nbw):
    # header (ticket, error flag), one int progress counter per stage rounded
    # to 256 bytes, the band with 2*nbw stored diagonals
    for cplx, elem in ((False, 8), (True, 16)):
        want = 256 + (4 * n + 255) // 256 * 256 + n * 2 * nbw * elem
        assert T.trbt_band_to_tridi_workspace_bytes(n, nbw, cplx) == want
    assert T.trbt_band_to_tridi_workspace_bytes(0, 4, False) == 0
    with pytest.raises(T.TrbtError):
        T.trbt_band_to_tridi_workspace_bytes(10, 65, False)


def test_tridiag_eigh_validation_codes(T):
    f = T.trbt_tridiag_eigh_d
    ok = dict(n=100, nev=10, d=FAKE, e=FAKE, w=FAKE, Z=FAKE, ldz=100, work=None, wb=0)

    def call(**kw):
        a = dict(ok, **kw)
        return f(a["n"], a["nev"], a["d"], a["e"], a["w"], a["Z"], a["ldz"], a["work"], a["wb"], 0)

    assert call(n=-1) == -1
    assert call(nev=-1) == -2
    assert call(nev=101) == -2
    assert call(d=None) == -3
    assert call(e=None) == -4
    assert call(w=None) == -5
    assert call(Z=None) == -6
    assert call(ldz=99) == -7
    assert call(work=FAKE + 8, wb=1 << 20) == -8
    assert call() == -101                       # TRBT_ERR_WORKSPACE
    assert call(nev=0, d=None, e=None, w=None, Z=None) == 0
    assert call(n=1, nev=1, ldz=1, e=None) == -101   # n = 1 needs no e; only the workspace missing


@pytest.mark.parametrize("n,nev", [(1, 1), (100, 10), (8192, 4096)])
def test_tridiag_eigh_workspace_formula(T, n, nev):
    al = lambda x: (x + 255) // 256 * 256
    want = al(max(n - 1, 1) * 8) + al(32) + al(n * nev * 8) + al(n * nev * 32) + al(n * nev)
    assert T.trbt_tridiag_eigh_workspace_bytes(n, nev) == want
    assert T.trbt_tridiag_eigh_workspace_bytes(n, 0) == 0


def test_work_check_validation(T):
    """trbt_work_check rejects a null fault pointer and a misaligned
    workspace before it touches the device."""
    import ctypes as C
    f = C.c_int(7)
    assert T.lib().trbt_work_check(None, None, None) == -2
    assert T.lib().trbt_work_check(FAKE + 8, C.byref(f), None) == -1


@pytest.mark.parametrize("fn", ["trans_ev_band_to_full_d", "trans_ev_band_to_full_z"])
def test_band_to_full_validation_codes(T, fn):
    """Argument errors of the band-to-full back-transformation come back
    before any launch, one per argument position."""
    f = getattr(T, fn)
    ok = dict(n=100, nbw=16, nev=10, hh_v=FAKE, ldv=100, hh_tau=FAKE, Z=FAKE, ldz=100,
              work=None, work_bytes=0)

    def call(**kw):
        a = dict(ok, **kw)
        return f(a["n"], a["nbw"], a["nev"], a["hh_v"], a["ldv"], a["hh_tau"], a["Z"], a["ldz"],
                 a["work"], a["work_bytes"], 0)

    assert call(n=-1) == -1
    assert call(nbw=0) == -2
    assert call(nev=101) == -3
    assert call(hh_v=None) == -4
    assert call(ldv=99) == -5
    assert call(hh_tau=None) == -6
    assert call(Z=None) == -7
    assert call(ldz=50) == -8
    assert call(work=FAKE + 8) == -9
    assert call() == -101                      # J > 0 needs the T workspace
    # J == 0 (n <= nbw + 1) and nev == 0 are no-ops without a device
    assert call(n=17, nbw=16, nev=3, ldv=17, ldz=17, hh_v=None, hh_tau=None) == 0
    assert call(nev=0, hh_v=None, hh_tau=None, Z=None) == 0


def test_band_to_full_workspace_size(T):
    """A 256-byte header plus one 64 x 64 compact-WY factor per panel of 64
    consecutive reflectors (J = n - nbw - 1 reflectors)."""
    for n, nbw, cplx in ((100, 16, False), (1000, 64, True), (66, 64, False), (65, 64, False)):
        J = max(n - nbw - 1, 0)
        P = -(-J // 64)
        expect = 0 if J == 0 else 256 + P * 64 * 64 * (16 if cplx else 8)
        assert T.trbt_band_to_full_workspace_bytes(n, nbw, 5, cplx) == expect
    assert T.trbt_band_to_full_workspace_bytes(1000, 64, 0, True) == 0


def test_band_to_full_noalloc_validation_and_limit(T):
    """The allocation-free band-to-full call validates arguments 1-8 like
    trans_ev_band_to_full_z and rejects, before any launch, problems whose
    compact-WY factors exceed its fixed scratch (TRBT_B2F_SCRATCH_BYTES)."""
    f = T.trans_ev_band_to_full_z_noalloc
    ok = dict(n=300, nbw=16, nev=10, hh_v=FAKE, ldv=300, hh_tau=FAKE, Z=FAKE, ldz=300)

    def call(**kw):
        a = dict(ok, **kw)
        return f(a["n"], a["nbw"], a["nev"], a["hh_v"], a["ldv"], a["hh_tau"], a["Z"],
                 a["ldz"], 0)

    assert call(n=-1) == -1
    assert call(nbw=0) == -2
    assert call(nev=301) == -3
    assert call(hh_v=None) == -4
    assert call(ldv=299) == -5
    assert call(hh_tau=None) == -6
    assert call(Z=None) == -7
    assert call(ldz=10) == -8
    assert call(n=17, nbw=16, nev=3, ldv=17, ldz=17, hh_v=None, hh_tau=None) == 0
    assert call(nev=0, hh_v=None, hh_tau=None, Z=None) == 0
    # the largest J whose 64-reflector panels fit, and one panel more
    cap = T.TRBT_B2F_SCRATCH_BYTES
    pmax = (cap - 256) // (64 * 64 * 16)
    n_fit = 64 * pmax + 64 + 1
    assert T.trbt_band_to_full_workspace_bytes(n_fit, 64, 1, True) <= cap
    assert T.trbt_band_to_full_workspace_bytes(n_fit + 1, 64, 1, True) > cap
    big = n_fit + 1
    assert call(n=big, nbw=64, nev=1, ldv=big, ldz=big) == -104
    assert "scratch" in T.trbt_strerror(-104)
