"""The residue meet-in-the-middle oracle pinned against the heap
Schroeppel-Shamir oracle at the sizes its golden values are built on.

Every golden value for n >= 70 comes from ``orc_mitm_residues`` (one residue
class of the left key at a time, Algorithm 1's set of solutions gathered per
class).  ``orc_ss_heap`` reaches the same set by a different route: Algorithm
1's two heaps merge the sorted sums, with no residue classes at all.  Here
the two agree on whole solves of the (6,50) pair (seed 0 and its planted
twin) with one to three key rows, on five key rows in the mixed radix, and on
(5,40) with two key rows, each under two moduli or a split class range.

The C oracle keeps its sort comparators' context in file-scope variables
(it is single-threaded), so independent solves run in a small pool of
processes, one solve at a time in each.
"""
import os
import json
import multiprocessing as mp
from concurrent.futures import ProcessPoolExecutor

import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_05045_amd.inputs import make_instance

pytestmark = pytest.mark.slow

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "oracle_configs.json")


def _same(a, b, what):
    assert a.H == b.H, f"{what}: H {a.H} != {b.H}"
    assert a.nsol == b.nsol, f"{what}: |S| {a.nsol} != {b.nsol}"
    assert np.array_equal(a.solutions, b.solutions), what


def _mitm_split(inst, r, lm, key_base=0):
    """The whole solve as two halves of the class range, added up."""
    half = 1 << (lm - 1)
    lo = O.mitm(inst.A, inst.d, r, lm, 0, half, key_base=key_base)
    hi = O.mitm(inst.A, inst.d, r, lm, half, 2 * half, key_base=key_base)
    sols = O.canonical(np.concatenate([lo.solutions, hi.solutions]))
    return O.OracleResult(lo.H + hi.H, lo.nsol + hi.nsol, sols)


# (planted, key rows, key_base, modulus bits of the single-range solve,
#  modulus bits of the split-range solve)
CASES = [(False, 1, 0, 9, None), (True, 1, 0, 12, None),
         (False, 2, 0, 9, None), (True, 2, 0, 10, None),
         (False, 3, 0, 9, None), (True, 3, 0, None, 11),
         (True, 5, 1, 9, None)]


def _run_6_50(case):
    planted, r, kb, lm, lm_split = case
    inst = make_instance(6, 50, 0, planted=planted)
    heap = O.ss_heap(inst.A, inst.d, r, key_base=kb)
    if lm is not None:
        mitm = O.mitm(inst.A, inst.d, r, lm, key_base=kb)
    else:
        mitm = _mitm_split(inst, r, lm_split, key_base=kb)
    return case, heap, mitm


def test_mitm_equals_heap_on_the_6_50_pair():
    insts = {p: make_instance(6, 50, 0, planted=p) for p in (False, True)}
    with ProcessPoolExecutor(max_workers=4, mp_context=mp.get_context("fork")) as ex:
        results = list(ex.map(_run_6_50, CASES))
    for (planted, r, kb, lm, lms), heap, mitm in results:
        what = f"(6,50) planted={planted} r={r} key_base={kb} 2^{lm or lms}"
        _same(mitm, heap, what)
        if planted:
            inst = insts[True]
            assert any(np.array_equal(s, inst.planted) for s in mitm.solutions), what
    # The solve with one key row also matches the stored heap results (and
    # the textbook counting DP on row 1).
    golden = {(g["name"], g["key_rows"], g["key_base"]): g for g in json.load(open(GOLDEN))
              if g["routine"] == "ss_heap"}
    for (planted, r, kb, lm, lms), heap, mitm in results:
        g = golden.get((insts[planted].name, r, kb))
        if g is not None:
            assert int(g["H"]) == mitm.H and g["nsol"] == mitm.nsol
        if r == 1:
            inst = insts[planted]
            assert mitm.H == O.dp_count(inst.A[0], int(inst.d[0]))


def test_mitm_equals_heap_on_5_40_two_key_rows():
    for planted in (False, True):
        inst = make_instance(5, 40, 0, planted=planted)
        heap = O.ss_heap(inst.A, inst.d, 2)
        for lm in (8, 13):
            _same(O.mitm(inst.A, inst.d, 2, lm), heap, f"(5,40) planted={planted} 2^{lm}")
        _same(_mitm_split(inst, 2, 10), heap, f"(5,40) planted={planted} split")
        assert heap.H == O.dp_count2(inst.A[0], inst.A[1], int(inst.d[0]), int(inst.d[1]))
