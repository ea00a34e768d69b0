"""Host AddressSanitizer (and UndefinedBehaviorSanitizer for the oracle) runs
of the plain-C oracle and of the host side of the C ABI, on the CPU.

* oracle.c is rebuilt with gcc -fsanitize=address,undefined and exercised in
  a child process (LD_PRELOAD of gcc's ASan runtime, since the Python
  interpreter is not instrumented): geometry, Householder generation, bulge
  chasing, QL, Jacobi, both back-transformations and both adjoints, the
  full-to-band reduction, at small ragged sizes.
* libtrbt is rebuilt with the host pass instrumented (hipcc -Xarch_host
  -fsanitize=address; device code as usual) and the host-only ABI tests run
  against it in a child process (LD_PRELOAD of clang's ASan runtime).
Any sanitizer report makes the child fail.
"""
import glob
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ENV_BASE = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:exitcode=99",
            "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1:exitcode=98",
            "OMP_NUM_THREADS": "4"}

ORACLE_SCRIPT = textwrap.dedent("""
    import numpy as np, oracle, synth
    assert oracle.num_reflectors(17, 4) == 36
    oracle.reflector_table(50, 7)
    oracle.larfg(np.array([1.0, 2.0, -3.0])); oracle.larfg(np.array([1 + 2j, 0.5j]))
    for dt in ("d", "z"):
        n, b = 61, 6
        ab = synth.band_matrix(n, b, 3, dt)
        p = oracle.stage2_pipeline(ab, b, 13)
        Y = oracle.back_transform(p["Z_in"], p["hh_v"], p["hh_tau"], b)
        oracle.back_transform(p["Z_in"], p["hh_v"], p["hh_tau"], b, cols=[0, 5])
        G = synth.gaussian(n, 13, 4, dt)
        oracle.adjoint(p["Z_in"], G, p["hh_v"], p["hh_tau"], b)
        A = synth.hermitian_matrix(45, 5, dt)
        r = oracle.full_to_band(A, 5)
        oracle.back_transform_full(synth.gaussian(45, 3, 6, dt), r["hh_v"], r["hh_tau"], 5)
    oracle.apply_q(synth.gaussian(30, 2, 1, "z"), *synth.unitary_reflectors(
        synth.reflector_lengths(30, 4), 4, 2, "z"), 4)
    oracle.jacobi_eigh(np.eye(5) + 0.1)
    oracle.tridiagonal_eigh(np.arange(7.0), np.ones(6))
    print("oracle under sanitizers: ok")
""")


def _run(cmd, env, timeout=900):
    e = dict(os.environ, **ENV_BASE, **env)
    e["PYTHONPATH"] = ROOT + os.pathsep + e.get("PYTHONPATH", "")
    return subprocess.run(cmd, cwd=ROOT, env=e, capture_output=True, text=True, timeout=timeout)


def _report(r):
    return f"rc={r.returncode}\\n--- stdout\\n{r.stdout[-3000:]}\\n--- stderr\\n{r.stderr[-6000:]}"


def test_oracle_under_asan_ubsan(tmp_path):
    lib = str(tmp_path / "liboracle_asan.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-fopenmp", "-std=gnu11", "-shared", "-fPIC",
                           os.path.join(ROOT, "oracle", "oracle.c"), "-o", lib, "-lm"])
    asan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    ubsan = subprocess.check_output(["gcc", "-print-file-name=libubsan.so"], text=True).strip()
    r = _run([sys.executable, "-c", ORACLE_SCRIPT],
             {"LD_PRELOAD": f"{asan} {ubsan}", "ORACLE_LIB": lib})
    assert r.returncode == 0 and "oracle under sanitizers: ok" in r.stdout, _report(r)
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, _report(r)


def _clang_asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


@pytest.mark.skipif(_clang_asan_runtime() is None, reason="clang ASan runtime not found")
def test_abi_host_side_under_asan(tmp_path):
    from paper_2002_10991_amd import build as b
    lib = str(tmp_path / "libtrbt_asan.so")
    flags = [f for f in b.HIPCC_FLAGS if f != "-O3"] + ["-O1", "-Xarch_host", "-fsanitize=address",
                                                          "-Xarch_host", "-fno-omit-frame-pointer"]
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    subprocess.check_call([hipcc, *flags, "-I", os.path.join(ROOT, "include"), "-I", b.CSRC,
                           *b.SRCS, "-o", lib])
    r = _run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
              os.path.join(ROOT, "tests", "test_abi_host.py")],
             {"LD_PRELOAD": _clang_asan_runtime(), "TRBT_LIB": lib})
    assert r.returncode == 0, _report(r)
    assert "AddressSanitizer" not in r.stderr, _report(r)
