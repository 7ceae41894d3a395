"""CPU checks of the C ABI: the library loads, exports every function that
include/msp.h declares, and validates instances before touching a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "msp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(msp_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ("msp_create", "msp_solve", "msp_hits", "msp_get_solutions", "msp_destroy"):
        assert want in names


def test_library_exports_every_declared_symbol():
    from paper_2507_05045_amd import msp
    for name in declared_functions():
        assert hasattr(msp.lib, name), name
    assert set(declared_functions()) == set(msp.EXPORTS)


def test_create_validates():
    from paper_2507_05045_amd import msp
    with pytest.raises(msp.MspError) as e:
        msp.Context(-np.ones((2, 3)), [1, 1])
    assert e.value.code == -1
    with pytest.raises(msp.MspError) as e:
        msp.Context(np.full((1, 3), 30000), [1])
    assert e.value.code == -2
    with pytest.raises(msp.MspError) as e:
        msp.Context(np.ones((2, 101)), [1, 1])
    assert e.value.code == -4
    ctx = msp.Context(np.ones((2, 5)), [2, 2])
    with pytest.raises(msp.MspError) as e:
        ctx.hits()                                   # nothing solved yet
    assert e.value.code == -9
    ctx.close()


def test_workspace_query_and_key_overflow():
    from paper_2507_05045_amd import msp
    ctx = msp.Context(np.full((9, 90), 99), [4455] * 9)
    assert ctx.workspace_bytes(msp.msp_default_opts(key_rows=4)) > 0
    # Five rows in radix 9000: a 66-bit key, past int64: two key words only.
    assert ctx.workspace_bytes(msp.msp_default_opts(key_rows=5, key_words=1)) == 0
    assert ctx.workspace_bytes(msp.msp_default_opts(key_rows=5)) > 0
    # Eight rows: 105 bits, past the 96 the records can hold.
    assert ctx.workspace_bytes(msp.msp_default_opts(key_rows=8)) == 0
    # A budget too small to hold even the quarter lists cannot be met.
    assert ctx.workspace_bytes(msp.msp_default_opts(key_rows=4, workspace_bytes=1 << 20)) == 0
    ctx.close()


def test_strerror_names_codes():
    from paper_2507_05045_amd import msp
    assert "row sum" in msp.strerror(-2)
    assert msp.strerror(0) == "ok"


@pytest.mark.skipif(os.path.exists("/dev/kfd"), reason="a GPU is present")
def test_solve_without_gpu_fails_loudly():
    from paper_2507_05045_amd import msp
    ctx = msp.Context(np.ones((1, 4)), [2])
    with pytest.raises(msp.MspError) as e:
        ctx.solve(use_torch=False)
    assert e.value.code == -10
    ctx.close()


def _c_layout(tmp_path, struct, fields):
    """sizeof and offsetof of a header struct, from a C program built by gcc."""
    import subprocess
    src = tmp_path / "layout.c"
    body = "".join(f'    printf("%zu\\n", offsetof({struct}, {f}));\n' for f in fields)
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "msp.h"\n'
                   f'int main(void) {{\n    printf("%zu\\n", sizeof({struct}));\n{body}'
                   '    return 0;\n}\n')
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src),
                           "-o", str(exe)])
    out = subprocess.check_output([str(exe)], text=True).split()
    return int(out[0]), [int(v) for v in out[1:]]


@pytest.mark.parametrize("struct", ["msp_opts", "msp_stats_t", "msp_batch_opts"])
def test_binding_structs_match_the_header(tmp_path, struct):
    from paper_2507_05045_amd import msp
    cls = getattr(msp, struct)
    names = [f for f, _ in cls._fields_]
    size, offs = _c_layout(tmp_path, struct, names)
    assert C.sizeof(cls) == size, struct
    assert [getattr(cls, f).offset for f in names] == offs, struct


def test_mixed_radix_key_fits_a_fifth_row():
    """key_base = 1 (radix rowsum_i + 1) holds five key rows at (9,80) in
    int64 where the radix n*D needs more (then two key words, 128-bit sums);
    an unknown key_base is rejected."""
    from paper_2507_05045_amd import msp
    from paper_2507_05045_amd.inputs import make_instance
    inst = make_instance(9, 80, 0)
    ctx = msp.Context(inst.A, inst.d)
    assert ctx.workspace_bytes(msp.msp_default_opts(key_rows=5, key_words=1)) == 0
    p = ctx.plan(key_rows=5)
    assert p["key_words"] == 2 and p["record_bytes"] == 16     # sums reach past 2^63
    p = ctx.plan(key_rows=5, key_base=1)
    assert p["key_bits"] <= 63
    # 60 bits: one word would need M = 2^36 (24 key bits per header)...
    p1 = ctx.plan(key_rows=5, key_base=1, key_words=1)
    assert (p1["key_words"], p1["log2_m"], p1["record_bytes"]) == (1, 36, 12)
    # ... the planner takes a second word instead and keeps M = 2^30.
    assert (p["key_words"], p["log2_m"], p["record_bytes"]) == (2, 30, 16)
    assert ctx.workspace_bytes(msp.msp_default_opts(key_rows=4, key_base=2)) == 0
    with pytest.raises(msp.MspError) as e:
        ctx.plan(key_rows=5, key_words=2, row_fingerprint=2)
    assert e.value.code == -4
    with pytest.raises(msp.MspError) as e:
        ctx.plan(key_rows=4, key_words=3)
    assert e.value.code == -1
    ctx.close()


def test_target_far_above_a_key_row_sum_is_planned_as_empty():
    """d_i > rowsum_i on a key row: no x can hit, the plan needs no key
    arithmetic on d (a d_i near 2^31 would overflow it)."""
    from paper_2507_05045_amd import msp
    A = np.full((5, 40), 99)
    ctx = msp.Context(A, [2 ** 31 - 1] * 5)
    for kb in (0, 1):
        assert ctx.workspace_bytes(msp.msp_default_opts(key_rows=4, key_base=kb)) > 0
    ctx.close()


def test_plan_struct_matches_the_header(tmp_path):
    from paper_2507_05045_amd import msp
    names = [f for f, _ in msp.msp_plan_t._fields_]
    size, offs = _c_layout(tmp_path, "msp_plan_t", names)
    assert C.sizeof(msp.msp_plan_t) == size
    assert [getattr(msp.msp_plan_t, f).offset for f in names] == offs


# The largest plans the solver runs: every launch whose size the plan fixes
# stays below 2^32 work-items, and the windows cover every cell.
LARGE_PLANS = [
    ((8, 70), dict(key_rows=5, key_base=1)),
    ((9, 80), dict(key_rows=5, key_base=1)),
    ((9, 80), dict(key_rows=4)),
    ((9, 80), dict(key_rows=4, slice_mod=64)),
    ((10, 90), dict(key_rows=4, slice_mod=64)),
    ((10, 90), dict(key_rows=4)),
    ((10, 90), dict(key_rows=4, slice_mod=64, verify_join=1)),
    ((6, 50), dict(key_rows=1)),
    ((6, 50), dict(key_rows=1, verify_join=2)),
    ((11, 100), dict(key_rows=4, slice_mod=4096)),
    ((11, 100), dict(key_rows=4)),
    ((10, 90), dict(key_rows=5, key_base=1, slice_mod=64)),
]


@pytest.mark.parametrize("shape,kw", LARGE_PLANS, ids=lambda v: str(v))
def test_largest_plans_fit_the_launch_limits(shape, kw):
    from paper_2507_05045_amd import autotune, msp
    from paper_2507_05045_amd.inputs import make_instance
    inst = make_instance(*shape, 0)
    ctx = msp.Context(inst.A, inst.d)
    tuned = autotune.lookup(inst.A, kw["key_rows"], kw.get("key_base", 0)) or {}
    budget = 64 << 30
    for opts in ({**kw}, {**kw, **tuned}):
        pl = ctx.plan(budget=budget, **opts)
        assert 0 < pl["max_grid_items"] < 2 ** 32, (opts, pl)
        assert pl["windows"] * pl["cells_per_window"] >= pl["cells"]
        assert pl["workspace_bytes"] <= budget
        assert pl["log2_m"] - pl["log2_cells"] == pl["log2_fine"] <= 12
    ctx.close()


def test_plan_picks_the_vector_join_for_large_equal_key_groups():
    """The (6,50) row-1 key has runs of ~10^5 records per side: the planner
    decides them by the vector join unless pairwise checks are asked for;
    (8,70) with four key rows has groups of about one record: pairwise."""
    from paper_2507_05045_amd import msp
    from paper_2507_05045_amd.inputs import make_instance
    big = msp.Context(make_instance(6, 50, 0).A, make_instance(6, 50, 0).d)
    assert big.plan(key_rows=1)["vector_join"] == 1
    assert big.plan(key_rows=1, verify_join=2)["vector_join"] == 0
    every = make_instance(4, 30, 0)
    ctx4 = msp.Context(every.A, every.d)
    assert ctx4.plan(key_rows=4, verify_join=1)["vector_join"] == 0   # every row a key row
    ctx4.close()
    small = msp.Context(make_instance(8, 70, 0).A, make_instance(8, 70, 0).d)
    assert small.plan(key_rows=4)["vector_join"] == 0
    assert small.plan(key_rows=4, verify_join=1)["vector_join"] == 1
    # (9,80): groups of ~23 records, still walked pair by pair; (10,90):
    # hundreds, decided by the vector join.
    mid = msp.Context(make_instance(9, 80, 0).A, make_instance(9, 80, 0).d)
    assert mid.plan(key_rows=4)["vector_join"] == 0
    wide = msp.Context(make_instance(10, 90, 0).A, make_instance(10, 90, 0).d)
    assert wide.plan(key_rows=4)["vector_join"] == 1
    big.close()
    small.close()
    mid.close()
    wide.close()


def test_set_allocator_rejects_half_a_pair():
    from paper_2507_05045_amd import msp
    a = msp.ALLOC_FN(lambda n, u: None)
    assert msp.lib.msp_set_allocator(a, msp.RELEASE_FN(), None) == -1
    assert msp.lib.msp_set_allocator(msp.ALLOC_FN(), msp.RELEASE_FN(), None) == 0


def test_quarter_split_plans():
    """log2_outer moves variables from each half's outer quarter to its
    inner one; the planner does so itself when the key room forces more
    residue cells than the equal quarters have inner elements."""
    from paper_2507_05045_amd import msp
    from paper_2507_05045_amd.inputs import make_instance
    i = make_instance(9, 80, 0)
    ctx = msp.Context(i.A, i.d)
    p = ctx.plan(key_rows=4)
    assert (p["log2_outer"], p["log2_inner"]) == (20, 20)
    p = ctx.plan(key_rows=4, log2_outer=18, log2_m=30, log2_cells=21)
    assert (p["log2_outer"], p["log2_inner"], p["log2_fine"]) == (18, 22, 9)
    for bad in (21, -1):
        with pytest.raises(msp.MspError) as e:
            ctx.plan(key_rows=4, log2_outer=bad)
        assert e.value.code == -1
    with pytest.raises(msp.MspError) as e:
        ctx.plan(key_rows=4, log2_cells=30)
    assert e.value.code == -1
    ctx.close()
    # (11,100), four key rows: 50 position bits leave 14 key bits in a
    # record header, so M = 2^40, 2^28 cells and q_B = 28.
    i = make_instance(11, 100, 0)
    ctx = msp.Context(i.A, i.d)
    p = ctx.plan(key_rows=4, slice_mod=4096)
    assert (p["log2_m"], p["log2_cells"], p["log2_outer"], p["log2_inner"]) == (40, 28, 22, 28)
    ctx.close()
    # (10,90), five key rows in the mixed radix: a 60-bit key.  With one key
    # word (19 key bits per header) M = 2^41, 2^29 cells; the planner's
    # choice keeps M = 2^35 with a second key word.
    i = make_instance(10, 90, 0)
    ctx = msp.Context(i.A, i.d)
    p = ctx.plan(key_rows=5, key_base=1, key_words=1)
    assert (p["log2_m"], p["log2_cells"], p["log2_outer"], p["log2_inner"]) == (41, 29, 17, 28)
    p = ctx.plan(key_rows=5, key_base=1)
    assert (p["log2_m"], p["log2_cells"], p["key_words"]) == (35, 23, 2)
    ctx.close()


@pytest.mark.parametrize("n", [1, 2, 3, 5])
def test_tiny_instances_plan(n):
    """Halves of one variable leave an empty right quarter (one subset)."""
    from paper_2507_05045_amd import msp
    ctx = msp.Context(np.ones((2, n)), [1, 1])
    p = ctx.plan(key_rows=1)
    assert p["log2_outer"] + p["log2_inner"] == (n + 1) // 2 and p["workspace_bytes"] > 0
    ctx.close()


def test_window_records_is_a_floor_on_the_record_buffers():
    """A one-cell window (a slice finer than the cells) is sized for the
    average cell; window_records raises its buffers for a denser class."""
    from paper_2507_05045_amd import msp
    from paper_2507_05045_amd.inputs import make_instance
    inst = make_instance(9, 80, 0, planted=True)
    ctx = msp.Context(inst.A, inst.d)
    kw = dict(key_rows=2, slice_mod=1 << 24, slice_res=12345)
    base = ctx.plan(**kw)
    assert base["windows"] == 1 and base["cells_per_window"] == 1
    assert base["window_records"] < 1 << 20
    big = ctx.plan(**kw, window_records=1 << 22)
    assert big["windows"] == 1 and big["window_records"] == 1 << 22
    assert big["workspace_bytes"] > base["workspace_bytes"] + 2 * 12 * ((1 << 22) - (1 << 20))
    ctx.close()
