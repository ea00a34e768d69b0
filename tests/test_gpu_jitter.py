"""Race shake-out for the waits between waves of the blocked kernels.

The debug build libtrbt_jitter.so (TRBT_WAIT_JITTER) puts a pseudo-random
delay in front of every wait on an LDS progress / ring counter, so the slot
hand-offs of the forward, batched and adjoint kernels (real and complex) run
in orders the release timing never produces.  In a child process on that build:
* the blocked parity, batched and split-adjoint tests (against the oracle,
  and batched against looped calls bitwise);
* a digest of the outputs of a few blocked cases, which must equal the
  release build's bit for bit (the arithmetic order of every column is fixed;
  only the timing changes).
"""
import os
import subprocess
import sys

import pytest

from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DIGEST = """
import hashlib, numpy as np, torch, synth
import paper_2002_10991_amd as T
h = hashlib.sha256()
for dt, n, nbw, nev in (("z", 517, 64, 100), ("d", 700, 32, 90), ("d", 400, 48, 33),
                        ("z", 300, 16, 47)):
    V, tau = synth.unitary_reflectors(synth.reflector_lengths(n, nbw), nbw, n, dt)
    Z = synth.gaussian(n, nev, n + 1, dt)
    zb = torch.from_numpy(np.ascontiguousarray(Z.T)).to("cuda")
    work = T.alloc_workspace(n, nbw, nev, dt == "z")
    T.back_transform(zb.T, torch.from_numpy(V).to("cuda"), torch.from_numpy(tau).to("cuda"),
                     nbw, work=work)
    assert T.trbt_work_check(work) == 0
    h.update(zb.cpu().numpy().tobytes())
print("DIGEST", h.hexdigest())
"""


def _child(args, lib, timeout=900):
    env = dict(os.environ, TRBT_LIB=lib)
    env["PYTHONPATH"] = ROOT + os.pathsep + env.get("PYTHONPATH", "")
    return subprocess.run([sys.executable, *args], cwd=ROOT, env=env, capture_output=True,
                          text=True, timeout=timeout)


def _jitter_lib():
    from paper_2002_10991_amd import build
    if not os.path.exists(build.OUT_JITTER):
        pytest.skip("libtrbt_jitter.so is not built (python -m paper_2002_10991_amd.build "
                    "--jitter)")
    return build.OUT_JITTER


@pytest.mark.timeout(900)
def test_blocked_tests_pass_under_wait_jitter():
    lib = _jitter_lib()
    print("[gpu] parity / batched / adjoint tests on the wait-jitter build", flush=True)
    r = _child(["-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                "tests/test_gpu_parity.py::test_parity_shapes",
                "tests/test_gpu_parity.py::test_parity_slot_groups",
                "tests/test_gpu_batched.py::test_batched_mixed_two_replays",
                "tests/test_gpu_batched.py::test_batched_equals_looped_bitwise",
                "tests/test_gpu_adjoint.py::test_adjoint_vs_oracle",
                "tests/test_gpu_adjoint.py::test_split_adjoint",
                "tests/test_gpu_adjoint_z.py::test_complex_adjoint_vs_oracle"], lib)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]


@pytest.mark.timeout(600)
def test_jitter_build_is_bitwise_the_release_result():
    from paper_2002_10991_amd import build
    lib = _jitter_lib()
    digests = []
    for path in (build.OUT, lib):
        print(f"[gpu] output digest with {os.path.basename(path)}", flush=True)
        r = _child(["-c", DIGEST], path)
        assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
        digests.append([l for l in r.stdout.splitlines() if l.startswith("DIGEST")][-1])
    assert digests[0] == digests[1]
