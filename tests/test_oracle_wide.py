"""The oracle with keys past int64 (six or more key rows in radix n*D).

Such a key is known to the oracle modulo 2^64 only, which is exact for its
residues modulo 2^k; two keys are then compared through what they encode
(k_L + k_R = K_d exactly when rows 1..r hold, eq. surrogate).  Pinned here
by brute force, whose H is the definition (x with rows 1..r holding, no key
at all), by the mixed radix (where the same r rows fit int64 and keys are
compared directly), and by slices that partition the solve.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_05045_amd.inputs import random_small


def _same(a, b, what):
    assert a.H == b.H, f"{what}: H {a.H} != {b.H}"
    assert a.nsol == b.nsol, f"{what}: |S| {a.nsol} != {b.nsol}"
    assert np.array_equal(a.solutions, b.solutions), what


def test_key_past_int64_is_flagged_and_wrapped():
    inst = random_small(7, 22, 3, planted=True)
    _, kd, w, _, wide = O.key_setup_wide(inst.A, inst.d, 6)
    assert wide
    with pytest.raises(O.OracleError):
        O.key_setup(inst.A, inst.d, 6)
    # Exact place values (Python integers): the oracle's values are the
    # same numbers modulo 2^64.
    B = 22 * 100
    exact_w = [sum(int(inst.A[i, j]) * B ** i for i in range(6)) for j in range(22)]
    exact_kd = sum(int(inst.d[i]) * B ** i for i in range(6))
    assert exact_kd >= 2 ** 63
    assert [int(x) % 2 ** 64 for x in w] == [x % 2 ** 64 for x in exact_w]
    assert int(kd) % 2 ** 64 == exact_kd % 2 ** 64
    # r = 5 in radix n*D and r = 6 in the mixed radix still fit int64.
    assert not O.key_setup_wide(inst.A, inst.d, 5)[4]
    assert not O.key_setup_wide(inst.A, inst.d, 6, key_base=1)[4]


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_wide_mitm_equals_brute_force(seed):
    inst = random_small(7, 22, seed, K=100 if seed % 2 else 6, planted=bool(seed % 2))
    for r in (6, 7):
        ref = O.brute(inst.A, inst.d, r)
        assert ref.H == int(ref.hr[r - 1])
        for lm in (6, 11):
            _same(O.mitm(inst.A, inst.d, r, lm), ref, f"seed {seed} r={r} 2^{lm}")
        half = 1 << 9
        lo = O.mitm(inst.A, inst.d, r, 10, 0, half)
        hi = O.mitm(inst.A, inst.d, r, 10, half, 2 * half)
        assert lo.H + hi.H == ref.H and lo.nsol + hi.nsol == ref.nsol
        if inst.planted is not None:
            assert any(np.array_equal(s, inst.planted) for s in ref.solutions)


def test_wide_equals_mixed_radix_and_slices_partition():
    inst = random_small(7, 22, 11, K=2, planted=True)     # 0/1 rows: many 1-D hits
    r = 6
    wide = O.mitm(inst.A, inst.d, r, 9)
    mixed = O.mitm(inst.A, inst.d, r, 9, key_base=1)      # fits int64: keys compared
    _same(wide, mixed, "radix n*D (wide) vs mixed radix (int64)")
    assert wide.H > 100
    tot, sols = 0, []
    for res in range(8):
        b = O.brute(inst.A, inst.d, r, slice_mod=8, slice_res=res)
        m = O.mitm(inst.A, inst.d, r, 9, slice_mod=8, slice_res=res)
        _same(m, b, f"slice {res} of 8")
        tot += m.H
        sols += [bytes(s) for s in m.solutions]
    assert tot == wide.H
    assert sorted(sols) == sorted(bytes(s) for s in wide.solutions)
    # The class of x* modulo 2^20 holds it.
    rho = O.left_key(inst.A, inst.d, inst.planted, r) % (1 << 20)
    c = O.mitm(inst.A, inst.d, r, 20, rho, rho + 1)
    assert any(np.array_equal(s, inst.planted) for s in c.solutions)
