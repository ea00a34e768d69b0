"""GPU parity of the batched plan (persistent graph-captured launch) against
the CPU oracle and against looped single-problem calls.

Every forced configuration and the autotuned one are run twice on the same
plan (graph replays), the second time with new Z and new reflectors in the
same buffers, and each replay is compared with the oracle.  Tolerance:
relative Frobenius error <= 1e-12 per problem (FP64 target accuracy).
"""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

TOL = 1e-12
CONFIGS = [(16, 8, 16), (16, 4, 16), (32, 8, 16), (32, 4, 16), (16, 8, 1), None]

# (n, nbw, nev): blocked groups for nbw 16/32/48/64 (ragged nev, several
# problems per group), streaming-only nbw, and problems with nothing to do
MIXED = [
    (300, 32, 150), (97, 32, 33), (512, 32, 256), (40, 32, 40),
    (200, 16, 17), (150, 48, 65), (301, 64, 63), (90, 64, 1),
    (129, 24, 31), (61, 3, 20),
    (2, 32, 2), (50, 1, 10), (64, 32, 0),
]


def _torch():
    import torch
    return torch


def _problem_inputs(n, nbw, nev, seed, oracle_mod, dt="d"):
    import synth
    lengths = oracle_mod.reflector_table(n, nbw)[3] if n >= 3 and nbw >= 2 else np.zeros(0, np.int64)
    V, tau = synth.unitary_reflectors(lengths, nbw, seed, dt)
    Z = synth.gaussian(n, nev, seed + 1, dt) if nev else np.zeros((n, 0), V.dtype)
    return Z, V, tau


class DeviceBatch:
    """Device buffers of a batch: Z (nev, ldz) per problem, hh_v, hh_tau."""

    def __init__(self, shapes, pad=0, cplx=False):
        torch = _torch()
        dtype = torch.complex128 if cplx else torch.float64
        self.shapes = shapes
        self.Z, self.V, self.tau = [], [], []
        for n, nbw, nev in shapes:
            K = max(int(_K(n, nbw)), 1)
            ldz = max(n, 1) + pad
            self.Z.append(torch.zeros(max(nev, 1), ldz, dtype=dtype, device="cuda"))
            self.V.append(torch.zeros(K, nbw, dtype=dtype, device="cuda"))
            self.tau.append(torch.zeros(K, dtype=dtype, device="cuda"))

    def load(self, inputs):
        torch = _torch()
        for i, (Z, V, tau) in enumerate(inputs):
            n = self.shapes[i][0]
            if Z.shape[1]:
                self.Z[i][:, :n].copy_(torch.from_numpy(np.ascontiguousarray(Z.T)))
            if V.size:
                self.V[i][: V.shape[0]].copy_(torch.from_numpy(V))
                self.tau[i][: tau.shape[0]].copy_(torch.from_numpy(tau))
        torch.cuda.synchronize()

    def problems(self):
        return [(self.Z[i].T[: n, : nev] if nev else self.Z[i].T[:n, :0], self.V[i], self.tau[i], nbw)
                for i, (n, nbw, nev) in enumerate(self.shapes)]

    def result(self, i):
        n, _, nev = self.shapes[i]
        return self.Z[i].cpu().numpy()[:nev, :n].T


def _K(n, nbw):
    import paper_2002_10991_amd as T
    return T.trbt_num_reflectors(n, nbw)


def _relerr(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _check_against_oracle(batch, inputs, oracle_mod):
    for i, (Z, V, tau) in enumerate(inputs):
        n, nbw, nev = batch.shapes[i]
        out = batch.result(i)
        if nev == 0:
            continue
        ref = oracle_mod.back_transform(Z, V, tau, nbw) if V.size else Z
        assert _relerr(out, ref) <= TOL, (i, n, nbw, nev, _relerr(out, ref))


@pytest.mark.parametrize("cfg", CONFIGS, ids=lambda c: "tuned" if c is None else "x".join(map(str, c)))
def test_batched_mixed_two_replays(oracle_mod, cfg):
    import paper_2002_10991_amd as T
    print(f"[gpu] batched mixed cfg={cfg}", flush=True)
    batch = DeviceBatch(MIXED, pad=3)
    inputs = [_problem_inputs(n, nbw, nev, 500 + 7 * i, oracle_mod) for i, (n, nbw, nev) in enumerate(MIXED)]
    batch.load(inputs)
    plan = T.BatchedPlan(batch.problems(), cfg)
    try:
        got_cfg, ms = plan.config
        if cfg is not None:
            assert got_cfg == tuple(cfg) and ms == 0.0
        else:
            assert ms > 0.0
        plan.run()
        _torch().cuda.synchronize()
        assert plan.fault() == 0
        _check_against_oracle(batch, inputs, oracle_mod)
        # second replay: new contents in the same buffers
        inputs2 = [_problem_inputs(n, nbw, nev, 900 + 5 * i, oracle_mod)
                   for i, (n, nbw, nev) in enumerate(MIXED)]
        batch.load(inputs2)
        plan.run()
        _torch().cuda.synchronize()
        assert plan.fault() == 0
        _check_against_oracle(batch, inputs2, oracle_mod)
    finally:
        plan.close()


def test_tuning_leaves_z_untouched(oracle_mod):
    import paper_2002_10991_amd as T
    torch = _torch()
    shapes = [(300, 32, 150), (129, 24, 31), (200, 16, 17)]
    batch = DeviceBatch(shapes)
    batch.load([_problem_inputs(n, nbw, nev, 40 + i, oracle_mod) for i, (n, nbw, nev) in enumerate(shapes)])
    before = [z.clone() for z in batch.Z]
    plan = T.BatchedPlan(batch.problems(), None)
    torch.cuda.synchronize()
    try:
        for a, b in zip(before, batch.Z):
            assert torch.equal(a, b)
    finally:
        plan.close()


def test_empty_and_degenerate_plans(oracle_mod):
    import paper_2002_10991_amd as T
    torch = _torch()
    plan = T.BatchedPlan([], None)
    plan.run()
    torch.cuda.synchronize()
    plan.close()
    shapes = [(2, 32, 2), (50, 1, 10), (64, 32, 0)]
    batch = DeviceBatch(shapes)
    for z in batch.Z:
        z.normal_()
    before = [z.clone() for z in batch.Z]
    plan = T.BatchedPlan(batch.problems(), (16, 8, 16))
    plan.run()
    torch.cuda.synchronize()
    plan.close()
    for a, b in zip(before, batch.Z):
        assert torch.equal(a, b)


@pytest.mark.parametrize("cfg", [(16, 8, 16), (32, 4, 16), (16, 8, 1)],
                         ids=lambda c: "x".join(map(str, c)))
def test_batched_equals_looped_bitwise(oracle_mod, cfg):
    """Batched plans against looped single calls: bitwise where both sides
    take the same form.  The blocked forms run the same window form (fixed
    for nbw <= 32, rotating for 48 and 64) with the same compact-WY blocks
    (the single call gives a wave two column tiles, the plan one or two:
    each tile's products are the same), and the streaming form has the same
    per-column arithmetic.  A plan with one-stage blocks streams every
    problem, so against a blocked single call it agrees to rounding."""
    import paper_2002_10991_amd as T
    torch = _torch()
    shapes = [(300, 32, 150), (97, 32, 33), (200, 16, 17), (150, 48, 65), (129, 24, 31)]
    inputs = [_problem_inputs(n, nbw, nev, 70 + i, oracle_mod) for i, (n, nbw, nev) in enumerate(shapes)]
    a, b = DeviceBatch(shapes), DeviceBatch(shapes)
    a.load(inputs)
    b.load(inputs)
    plan = T.BatchedPlan(a.problems(), cfg)
    plan.run()
    for Zv, V, tau, nbw in b.problems():
        T.back_transform(Zv, V, tau, nbw)
    torch.cuda.synchronize()
    plan.close()
    for i, (n, nbw, nev) in enumerate(shapes):
        same_form = cfg[2] == 16 or nbw not in (16, 32, 48, 64)
        if same_form:
            assert np.array_equal(a.result(i), b.result(i)), (i, shapes[i])
        else:
            assert _relerr(a.result(i), b.result(i)) <= 1e-14, (i, shapes[i])


def _c4_shapes():
    import synth
    return [(int(n), 32, int(n) // 2) for n in synth.batched_sizes()]


def test_c4_full_batch_sampled(oracle_mod):
    """The 64-problem batch (n_p = 512*U{1..8}, nbw=32, nev=n_p/2) with the
    autotuned plan, in the configuration the benchmark times: every problem
    checked on sampled columns against the oracle, and in full against looped
    single calls."""
    import paper_2002_10991_amd as T
    import synth
    torch = _torch()
    shapes = _c4_shapes()
    seeds = synth.batched_seeds()
    inputs = []
    for i, (n, nbw, nev) in enumerate(shapes):
        lengths = synth.reflector_lengths(n, nbw)
        V, tau = synth.unitary_reflectors(lengths, nbw, seeds[i], "d")
        Z = synth.gaussian(n, nev, seeds[i] + 1, "d")
        inputs.append((Z, V, tau))
    print(f"[gpu] C4 batch: {len(shapes)} problems, n in [{min(s[0] for s in shapes)}, "
          f"{max(s[0] for s in shapes)}]", flush=True)
    a, b = DeviceBatch(shapes), DeviceBatch(shapes)
    a.load(inputs)
    b.load(inputs)
    plan = T.BatchedPlan(a.problems(), None)
    print(f"[gpu] C4 tuned config {plan.config}", flush=True)
    plan.run()
    torch.cuda.synchronize()
    assert plan.fault() == 0
    plan.close()
    for Zv, V, tau, nbw in b.problems():
        T.back_transform(Zv, V, tau, nbw)
    torch.cuda.synchronize()
    rng = np.random.default_rng(4)
    for i, (n, nbw, nev) in enumerate(shapes):
        out = a.result(i)
        cols = np.unique(np.concatenate([[0, nev - 1], rng.integers(0, nev, 6)]))
        Z, V, tau = inputs[i]
        ref = oracle_mod.back_transform(Z, V, tau, nbw, cols=cols)
        assert _relerr(out[:, cols], ref) <= TOL, (i, n)
        assert _relerr(out, b.result(i)) <= TOL, (i, n)


def test_c4_pipeline_problems(oracle_mod):
    """A few C4-style problems end to end: band N(0,1) from the per-problem
    seeds, reflectors from the oracle's bulge chase, the lowest n/2
    eigenvectors from its QL solve; the batched result matches the oracle
    back-transform and is an eigenbasis of B."""
    import paper_2002_10991_amd as T
    import synth
    torch = _torch()
    seeds = synth.batched_seeds()
    shapes, inputs, pipes = [], [], []
    for i, n in enumerate([512, 1024, 512]):
        ab = synth.band_matrix(n, 32, seeds[i], "d")
        p = oracle_mod.stage2_pipeline(ab, 32, n // 2)
        shapes.append((n, 32, n // 2))
        inputs.append((p["Z_in"], p["hh_v"], p["hh_tau"]))
        pipes.append((ab, p))
    batch = DeviceBatch(shapes)
    batch.load(inputs)
    plan = T.BatchedPlan(batch.problems(), None)
    plan.run()
    torch.cuda.synchronize()
    plan.close()
    _check_against_oracle(batch, inputs, oracle_mod)
    for i, (ab, p) in enumerate(pipes):
        Y = batch.result(i)
        B = synth.dense_from_band(ab)
        n = B.shape[0]
        assert np.linalg.norm(B @ Y - Y * p["w"]) / np.linalg.norm(B) <= 1e-12 * n
        assert np.linalg.norm(Y.T @ Y - np.eye(Y.shape[1])) <= 1e-12 * n


# complex Hermitian problems: blocked groups for every nbw, the streaming form,
# ragged nev and problems with nothing to do
CMIXED = [
    (300, 32, 150), (97, 32, 33), (200, 16, 17), (150, 48, 65), (301, 64, 63),
    (90, 64, 1), (129, 24, 31), (61, 3, 20), (2, 32, 2), (64, 32, 0),
]


@pytest.mark.parametrize("cfg", [(16, 8, 16), (16, 4, 16), (16, 8, 1), None],
                         ids=lambda c: "tuned" if c is None else "x".join(map(str, c)))
def test_batched_complex_two_replays(oracle_mod, cfg):
    import paper_2002_10991_amd as T
    print(f"[gpu] batched complex cfg={cfg}", flush=True)
    batch = DeviceBatch(CMIXED, pad=2, cplx=True)
    inputs = [_problem_inputs(n, nbw, nev, 700 + 3 * i, oracle_mod, "z")
              for i, (n, nbw, nev) in enumerate(CMIXED)]
    batch.load(inputs)
    plan = T.BatchedPlan(batch.problems(), cfg)
    try:
        got_cfg, ms = plan.config
        if cfg is not None:
            assert got_cfg == tuple(cfg) and ms == 0.0
        else:
            assert got_cfg[0] == 16 and ms > 0.0
        for rep, seed0 in enumerate((700, 1100)):
            if rep:
                inputs = [_problem_inputs(n, nbw, nev, seed0 + 3 * i, oracle_mod, "z")
                          for i, (n, nbw, nev) in enumerate(CMIXED)]
                batch.load(inputs)
            plan.run()
            _torch().cuda.synchronize()
            assert plan.fault() == 0
            _check_against_oracle(batch, inputs, oracle_mod)
    finally:
        plan.close()


@pytest.mark.parametrize("cfg", [(16, 8, 16), (16, 4, 16)], ids=lambda c: "x".join(map(str, c)))
def test_batched_complex_equals_looped_bitwise(oracle_mod, cfg):
    """Complex plans run the single-call per-column arithmetic too: results
    agree bitwise with looped trans_ev_tridi_to_band_z calls."""
    import paper_2002_10991_amd as T
    torch = _torch()
    shapes = [(300, 32, 150), (97, 32, 33), (200, 16, 17), (150, 48, 65), (129, 24, 31),
              (260, 64, 40)]
    inputs = [_problem_inputs(n, nbw, nev, 80 + i, oracle_mod, "z")
              for i, (n, nbw, nev) in enumerate(shapes)]
    a, b = DeviceBatch(shapes, cplx=True), DeviceBatch(shapes, cplx=True)
    a.load(inputs)
    b.load(inputs)
    plan = T.BatchedPlan(a.problems(), cfg)
    plan.run()
    for Zv, V, tau, nbw in b.problems():
        T.back_transform(Zv, V, tau, nbw)
    torch.cuda.synchronize()
    plan.close()
    for i in range(len(shapes)):
        assert np.array_equal(a.result(i), b.result(i)), (i, shapes[i])


def test_batched_rejects_mixed_precision():
    import paper_2002_10991_amd as T
    torch = _torch()
    Zr = torch.zeros(4, 100, dtype=torch.float64, device="cuda")
    Zc = torch.zeros(4, 100, dtype=torch.complex128, device="cuda")
    Vr = torch.zeros(10, 8, dtype=torch.float64, device="cuda")
    Vc = torch.zeros(10, 8, dtype=torch.complex128, device="cuda")
    tr = torch.zeros(10, dtype=torch.float64, device="cuda")
    tc = torch.zeros(10, dtype=torch.complex128, device="cuda")
    with pytest.raises(TypeError):
        T.BatchedPlan([(Zr.T, Vr, tr, 8), (Zc.T, Vc, tc, 8)])


def test_c4z_full_batch_sampled(oracle_mod):
    """The complex batch the benchmark times (64 problems, n_p = 512*U{1..8},
    nbw=32, nev=n_p/2, same seeds as the real one) with the autotuned plan:
    every problem checked on sampled columns against the oracle, and in full
    (bitwise) against looped single complex calls."""
    import paper_2002_10991_amd as T
    import synth
    torch = _torch()
    shapes = _c4_shapes()
    seeds = synth.batched_seeds()
    inputs = []
    for i, (n, nbw, nev) in enumerate(shapes):
        lengths = synth.reflector_lengths(n, nbw)
        V, tau = synth.unitary_reflectors(lengths, nbw, seeds[i], "z")
        Z = synth.gaussian(n, nev, seeds[i] + 1, "z")
        inputs.append((Z, V, tau))
    print(f"[gpu] C4z batch: {len(shapes)} complex problems", flush=True)
    a, b = DeviceBatch(shapes, cplx=True), DeviceBatch(shapes, cplx=True)
    a.load(inputs)
    b.load(inputs)
    plan = T.BatchedPlan(a.problems(), None)
    print(f"[gpu] C4z tuned config {plan.config}", flush=True)
    plan.run()
    torch.cuda.synchronize()
    assert plan.fault() == 0
    plan.close()
    for Zv, V, tau, nbw in b.problems():
        T.back_transform(Zv, V, tau, nbw)
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    for i, (n, nbw, nev) in enumerate(shapes):
        out = a.result(i)
        cols = np.unique(np.concatenate([[0, nev - 1], rng.integers(0, nev, 4)]))
        Z, V, tau = inputs[i]
        ref = oracle_mod.back_transform(Z, V, tau, nbw, cols=cols)
        assert _relerr(out[:, cols], ref) <= TOL, (i, n)
        assert np.array_equal(out, b.result(i)), (i, n)


def test_tuning_cache_round_trip(oracle_mod, tmp_path, monkeypatch):
    """TRBT_TUNE_CACHE: the first tuned plan of a problem set times the
    candidates and appends one line; a second plan of the same shapes (other
    buffers) takes the cached choice without timing; another shape set is a
    miss.  Results are the same either way."""
    import time
    import paper_2002_10991_amd as T
    torch = _torch()
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("TRBT_TUNE_CACHE", str(cache))
    shapes = [(300, 32, 40), (520, 32, 100), (130, 16, 7)]
    inputs = [_problem_inputs(n, nbw, nev, 7100 + i, oracle_mod)
              for i, (n, nbw, nev) in enumerate(shapes)]
    plans = []
    for k in range(2):
        batch = DeviceBatch(shapes)
        batch.load(inputs)
        print(f"[gpu] tuned plan {k}", flush=True)
        t0 = time.perf_counter()
        plan = T.BatchedPlan(batch.problems())
        dt = time.perf_counter() - t0
        plans.append((plan, batch, dt))
        assert len(cache.read_text().splitlines()) == 1     # a hit appends nothing
    (p1, b1, t1), (p2, b2, t2) = plans
    cfg1, ms1 = p1.config
    cfg2, ms2 = p2.config
    assert cfg1 == cfg2 and ms2 == pytest.approx(ms1, rel=1e-5)
    assert cache.read_text().startswith("trbt-tune-v1 ")
    print(f"[gpu] tuned plan {t1:.3f} s, cached plan {t2:.3f} s, config {cfg1}", flush=True)
    for plan, batch, _ in plans:
        plan.run()
        torch.cuda.synchronize()
        assert plan.fault() == 0
        _check_against_oracle(batch, inputs, oracle_mod)
        plan.close()
    other = DeviceBatch(shapes[:2])
    other.load(inputs[:2])
    T.BatchedPlan(other.problems()).close()
    assert len(cache.read_text().splitlines()) == 2         # a new signature
