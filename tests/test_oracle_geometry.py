"""Pins for the oracle's reflector geometry (Sec. 2.2.1 / 2.2.2 / 3.2).

The only numbers the paper prints for this path are the N=17, b=4 worked
example (tests/golden/worked_example_n17_b4.json).  The counts K and L are
checked against an independent closed form.
"""
import json
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_example_n17_b4.json")


def _rows_1based(table, stage_1b, sweep_1b):
    st, sl, r0, ln = table
    k = np.nonzero((st == stage_1b - 1) & (sl == sweep_1b - 1))[0]
    assert len(k) == 1, (stage_1b, sweep_1b)
    k = k[0]
    return int(r0[k]) + 1, int(r0[k] + ln[k])


def test_worked_example_facts(oracle_mod):
    g = json.load(open(GOLDEN))
    n, b = g["n"], g["b"]
    tab = oracle_mod.reflector_table(n, b)
    facts = g["facts"]
    # fourth stage has 3 sweeps
    assert oracle_mod.sweeps_in_stage(n, b, facts[0]["stage_1based"] - 1) == facts[0]["sweeps"]
    # first sweep of the fourth stage: a length-4 reflector starting right
    # below the diagonal of column 4 eliminates 3 elements of that column
    lo, hi = _rows_1based(tab, 4, 1)
    assert lo == facts[1]["annihilated_column_1based"] + 1
    assert hi - lo == facts[1]["eliminated"]
    # v(1,4) alters only the last four rows
    assert list(range(*_rows_1based(tab, 1, 4))) + [_rows_1based(tab, 1, 4)[1]] == \
        facts[2]["rows_1based"]
    # kernel walk-through: X_local is the N_R rows ending with the last row of Q(8,1)
    f = facts[3]
    bottom = _rows_1based(tab, 8, 1)[1]
    first = bottom - f["N_R"] + 1
    for key, (a, z) in f["x_local_rows_modified"].items():
        i, j = map(int, key.split(","))
        lo, hi = _rows_1based(tab, i, j)
        assert (lo - first + 1, hi - first + 1) == (a, z)
    # consecutive applied reflectors move up exactly one row
    prev = None
    for i, j in f["applied_1based"]:
        lo, hi = _rows_1based(tab, i, j)
        if prev is not None:
            assert (lo, hi) == (prev[0] - 1, prev[1] - 1)
        prev = (lo, hi)
    # Q(4,1), Q(3,1), Q(2,1) touch the top three rows of X_local; Q(1,1) does not
    f = facts[4]
    top = set()
    for i, j in f["also_touch_top"]:
        lo, hi = _rows_1based(tab, i, j)
        rows = set(range(lo, hi + 1)) & set(range(first, bottom + 1))
        assert rows and min(rows) == first
        top |= rows
    assert len(top) == f["top_rows_exchanged"]
    lo, hi = _rows_1based(tab, 1, 1)
    assert hi < first


def _closed_form_counts(n, b):
    """K = sum_s ceil((n-s-2)/b); L = sum_s (n-s-1 - [(n-s-1) mod b == 1])."""
    if b < 2 or n < 3:
        return 0, 0
    m = np.arange(n - 2)              # m = n - s - 2 for s = n-3 .. 0
    m = m + 1
    K = int(np.sum((m + b - 1) // b))
    rows = m + 1                       # n - s - 1
    L = int(np.sum(rows - ((rows % b) == 1)))
    return K, L


@pytest.mark.parametrize("n,b", [(17, 4), (64, 8), (1024, 32), (4096, 64), (8192, 64),
                                 (32768, 64), (100, 3), (33, 31), (5, 2), (3, 1), (2, 4)])
def test_counts_closed_form(oracle_mod, n, b):
    K, L = _closed_form_counts(n, b)
    assert oracle_mod.num_reflectors(n, b) == K
    if K:
        st, sl, r0, ln = oracle_mod.reflector_table(n, b)
        assert int(ln.sum()) == L
        assert ln.min() >= 2 and ln.max() <= b
        assert np.all(r0 + ln <= n)


def test_counts_at_the_workload_shapes(oracle_mod):
    # values tabulated from the closed form for the workload shapes
    expect = {(17, 4): (36, 132), (64, 8): (272, 2008), (1024, 32): (16832, 523744),
              (4096, 64): (132992, 8386496), (8192, 64): (528128, 33550208),
              (32768, 64): (8403968, 536854016)}
    for (n, b), (K, L) in expect.items():
        assert _closed_form_counts(n, b) == (K, L)
        assert oracle_mod.num_reflectors(n, b) == K


def test_same_stage_reflectors_disjoint_and_chain_shift(oracle_mod):
    n, b = 300, 16
    st, sl, r0, ln = oracle_mod.reflector_table(n, b)
    for s in range(n - 2):
        k = np.nonzero(st == s)[0]
        lo, hi = r0[k], r0[k] + ln[k]
        assert np.all(lo[1:] >= hi[:-1])          # disjoint, ordered by slot
        assert lo[0] == s + 1
    # slot j of stage s-1 starts one row above slot j of stage s
    for s in range(1, n - 2):
        a = r0[st == s]
        c = r0[st == s - 1][: len(a)]
        assert np.all(c == a - 1)
