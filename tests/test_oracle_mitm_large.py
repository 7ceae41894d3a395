"""The residue meet-in-the-middle oracle pinned at the sizes its golden values
are built on (n = 70, 80, 90), with two key rows, by counting.

With key rows 1-2 (radix B = n*D, Section 1 eq. surrogate) and a modulus M
above every left key, a residue class of the left key holds one pair of left
row sums (s1, s2) = (k_L mod B, k_L div B).  Its 1-D hits are then every left
vector with those sums against every right vector with the complementary
ones:

    H(class) = N_L(s1, s2) * N_R(d1 - s1, d2 - s2),

where N_L and N_R count the subsets of each half's columns by their two row
sums.  The counts come from a dynamic programme over the columns written
here in numpy, which shares nothing with the oracle's quarter lists, residue
sort and equal-key counting.  The classes are the planted solution's (whose
H runs to 7e12 at (9,80); the planted vector must be among the class's
solutions) and, at (10,90), the largest class with at most a million
vectors per side.
"""
import itertools

import numpy as np
import pytest

from half_counts import half_counts
from oracle import oracle as O
from paper_2507_05045_amd.inputs import make_instance

pytestmark = pytest.mark.slow


def test_half_counts_is_the_subset_count():
    rng = np.random.default_rng(3)
    a1, a2 = rng.integers(0, 9, 12), rng.integers(0, 9, 12)
    N = half_counts(a1, a2)
    ref = np.zeros_like(N)
    for bits in itertools.product((0, 1), repeat=12):
        x = np.array(bits)
        ref[int(a1 @ x), int(a2 @ x)] += 1
    assert np.array_equal(N, ref)
    assert N.sum() == 2 ** 12


def test_half_counts_equals_the_oracle_two_row_dp():
    """The test's DP and the oracle's 2-row counting DP, written apart,
    agree on the (6,50) matrix's first two rows over all 50 columns."""
    inst = make_instance(6, 50, 0)
    a1, a2 = inst.A[0].astype(np.int64), inst.A[1].astype(np.int64)
    N = half_counts(a1, a2)
    rng = np.random.default_rng(5)
    targets = [(int(a1.sum()) // 2, int(a2.sum()) // 2), (0, 0), (int(a1.sum()), int(a2.sum()))]
    targets += [(int(rng.integers(0, N.shape[0])), int(rng.integers(0, N.shape[1])))
                for _ in range(6)]
    for t1, t2 in targets:
        assert int(N[t1, t2]) == O.dp_count2(a1, a2, t1, t2), (t1, t2)


def _class_counts(inst):
    A, d = inst.A.astype(np.int64), inst.d.astype(np.int64)
    hl = (A.shape[1] + 1) // 2
    NL = half_counts(A[0, :hl], A[1, :hl])
    NR = half_counts(A[0, hl:], A[1, hl:])
    assert NL.sum() == 2 ** hl and NR.sum() == 2 ** (A.shape[1] - hl)
    base, _, _, _ = O.key_setup(inst.A, inst.d, 2)
    # Every left key s1 + s2 * B lies below 2^lm: one (s1, s2) per class.
    lm = int(NL.shape[0] - 1 + (NL.shape[1] - 1) * base).bit_length()
    assert NL.shape[0] <= base

    def right(s1, s2):
        r1, r2 = int(d[0]) - s1, int(d[1]) - s2
        if 0 <= r1 < NR.shape[0] and 0 <= r2 < NR.shape[1]:
            return int(NR[r1, r2])
        return 0
    return NL, right, base, lm


def _check_solutions(inst, res, rho, lm):
    for x in res.solutions:
        assert np.array_equal(inst.A.astype(np.int64) @ x, inst.d.astype(np.int64))
        assert O.left_key(inst.A, inst.d, x, 2) % (1 << lm) == rho


@pytest.mark.parametrize("m,n", [(8, 70), (9, 80)])
def test_planted_class_hits_equal_the_half_counts(m, n):
    inst = make_instance(m, n, 0, planted=True)
    NL, right, base, lm = _class_counts(inst)
    x = inst.planted
    hl = (n + 1) // 2
    s1 = int(inst.A[0, :hl].astype(np.int64) @ x[:hl])
    s2 = int(inst.A[1, :hl].astype(np.int64) @ x[:hl])
    rho = O.left_key(inst.A, inst.d, x, 2)
    assert rho == s1 + s2 * base
    res = O.mitm(inst.A, inst.d, 2, lm, rho, rho + 1)
    assert res.H == int(NL[s1, s2]) * right(s1, s2)
    assert res.H > 10 ** 9
    assert any(np.array_equal(s, x) for s in res.solutions)
    _check_solutions(inst, res, rho, lm)


def test_10_90_class_hits_equal_the_half_counts():
    inst = make_instance(10, 90, 0)
    NL, right, base, lm = _class_counts(inst)
    best, cls = 0, None
    for s1 in range(NL.shape[0]):
        for s2 in np.nonzero((NL[s1] > 0) & (NL[s1] <= 10 ** 6))[0]:
            nr = right(s1, int(s2))
            if 0 < nr <= 10 ** 6 and int(NL[s1, s2]) * nr > best:
                best, cls = int(NL[s1, s2]) * nr, (s1, int(s2))
    assert cls is not None and best > 10 ** 11
    rho = cls[0] + cls[1] * base
    res = O.mitm(inst.A, inst.d, 2, lm, rho, rho + 1)
    assert res.H == best
    _check_solutions(inst, res, rho, lm)
