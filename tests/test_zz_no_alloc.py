"""msp_solve_noalloc (the entry point for callers that cannot allocate)
against msp_solve: identical H, |S| and solution vectors on two calls in a
row, the second with a smaller instance, and a clear error for an instance
whose plan does not fit the fixed scratch array."""
import sys

import numpy as np
import pytest

from paper_2507_05045_amd.inputs import make_instance, random_small

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _res(ctx):
    return ctx.hits(), ctx.num_solutions(), ctx.solutions(), ctx.stats()


def _same(a, b, what):
    assert a[0] == b[0], f"{what}: H {a[0]} != {b[0]}"
    assert a[1] == b[1], f"{what}: |S| {a[1]} != {b[1]}"
    assert np.array_equal(a[2], b[2]), what


def test_noalloc_matches_solve_two_calls_in_a_row():
    from paper_2507_05045_amd import msp
    cases = [(make_instance(6, 50, 0, planted=True), dict(key_rows=1, verify_join=2)),
             (make_instance(5, 40, 3, planted=True), dict(key_rows=2)),
             (random_small(4, 22, 901, K=8, planted=True), dict(key_rows=2))]
    for inst, kw in cases:                       # larger first, then smaller
        say("noalloc", inst.name, kw)
        ref = msp.Context(inst.A, inst.d)
        ref.solve(**kw)
        r = _res(ref)
        ref.close()
        c = msp.Context(inst.A, inst.d)
        c.solve_noalloc(**kw)
        g = _res(c)
        _same(g, r, f"noalloc {inst.name}")
        assert g[3]["windows"] >= 1 and g[3]["complete"] == 1
        c.close()


def test_noalloc_plan_beyond_the_scratch_is_rejected():
    from paper_2507_05045_amd import msp
    inst = make_instance(9, 80, 0)
    c = msp.Context(inst.A, inst.d)
    with pytest.raises(msp.MspError) as e:
        c.solve_noalloc(key_rows=4)
    assert e.value.code == -5                    # MSP_E_NOMEM: does not fit the scratch
    with pytest.raises(msp.MspError) as e:
        c.solve_noalloc(key_rows=4, workspace_bytes=1 << 20)
    assert e.value.code == -1
    c.close()
