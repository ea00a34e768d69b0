"""On-disk cache of oracle results for the large parity cases (test
infrastructure).

At the workload sizes the CPU oracle is slow: about a minute on 16 cores for
512 columns of the n = 32768 back-transformation, longer for the full-width
adjoint at n = 4096, hours for a CPU bulge chase at n = 32768.  Its results
depend only on the seeded inputs, so a result is stored under a key made of
the case's parameters (config, seeds, dtype, sampled columns ...) and a hash
of the sources of the oracle and of the seeded input generators: a change
in either computes it afresh.  A run that stops part way (a killed session,
a failed GPU step after the oracle part) resumes from what was stored.

Storage: one .npz file per result (numpy arrays only, read back with
allow_pickle=False), written to a temporary name and renamed, in the folder
named by $TRBT_ORACLE_CACHE, else tests/.oracle_cache (kept out of version
control).  TRBT_ORACLE_CACHE=off computes every result and stores nothing.
A file that cannot be read (truncated, foreign) is computed again and
replaced.  Nothing here runs on the GPU or reads the GPU path's results.
"""
import hashlib
import json
import os
import tempfile

import numpy as np

_ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# the oracle and the seeded input generators: what a cached result depends on
_SOURCES = ("oracle/oracle.c", "oracle/__init__.py", "synth/__init__.py")


def cache_dir():
    d = os.environ.get("TRBT_ORACLE_CACHE", "")
    if d.lower() == "off":
        return None
    return d or os.path.join(_ROOT, "tests", ".oracle_cache")


def sources_hash() -> str:
    h = hashlib.sha256()
    for rel in _SOURCES:
        with open(os.path.join(_ROOT, rel), "rb") as f:
            h.update(rel.encode() + b"\0" + f.read() + b"\0")
    return h.hexdigest()


def _normalise(v):
    if isinstance(v, np.ndarray):
        return v.tolist()
    if isinstance(v, (np.integer,)):
        return int(v)
    if isinstance(v, (np.floating,)):
        return float(v)
    if isinstance(v, (list, tuple)):
        return [_normalise(x) for x in v]
    if isinstance(v, dict):
        return {str(k): _normalise(x) for k, x in sorted(v.items())}
    return v


def key_file(kind: str, key: dict) -> str:
    """File name of a result: the kind (a readable prefix) and the hash of
    the key, the sources hash included."""
    text = json.dumps({"kind": kind, "key": _normalise(key), "sources": sources_hash()},
                      sort_keys=True)
    return f"{kind}-{hashlib.sha256(text.encode()).hexdigest()[:32]}.npz"


def cached(kind: str, key: dict, compute):
    """The arrays compute() returns (a dict name -> ndarray), from the cache
    when a result for (kind, key, sources) is stored, else computed and
    stored."""
    d = cache_dir()
    if d is None:
        return compute()
    path = os.path.join(d, key_file(kind, key))
    if os.path.exists(path):
        try:
            with np.load(path, allow_pickle=False) as f:
                return {k: f[k] for k in f.files}
        except Exception:
            pass   # unreadable: compute it again and replace the file
    out = compute()
    os.makedirs(d, exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=d, suffix=".tmp")
    try:
        with os.fdopen(fd, "wb") as f:
            np.savez(f, **{k: np.asarray(v) for k, v in out.items()})
        os.replace(tmp, path)
    finally:
        if os.path.exists(tmp):
            os.remove(tmp)
    return out
