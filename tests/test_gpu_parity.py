"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Everything is exact integer, so the bar is bit-exact: the 1-D hit count H,
|S| and the canonical list of solution vectors must be identical.
"""
import json
import os
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_05045_amd.inputs import make_instance, random_small

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "oracle_configs.json")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def gsolve(A, d, **kw):
    from paper_2507_05045_amd import msp
    return msp.solve(A, d, **kw)


def same(g, o, what=""):
    assert g.H == o.H, f"{what}: H {g.H} != {o.H}"
    assert g.nsol == o.nsol, f"{what}: |S| {g.nsol} != {o.nsol}"
    assert g.solutions.shape == o.solutions.shape, what
    assert np.array_equal(g.solutions, o.solutions), what


def satisfies(A, d, sols):
    return all(np.array_equal(np.asarray(A, np.int64) @ s.astype(np.int64), d) for s in sols)


SMALL = [
    dict(m=3, n=20, K=100, zero=0, r=1),
    dict(m=4, n=21, K=100, zero=0, r=2),
    dict(m=4, n=22, K=6, zero=0, r=1),      # heavy key ties
    dict(m=4, n=22, K=6, zero=0, r=3),
    dict(m=4, n=24, K=4, zero=0, r=2),      # large equal-key groups (tiled verify by index)
    dict(m=3, n=19, K=100, zero=3, r=1),    # zero columns
    dict(m=5, n=17, K=3, zero=2, r=2),
    dict(m=2, n=5, K=4, zero=0, r=1),
    dict(m=6, n=24, K=100, zero=0, r=2),
    dict(m=4, n=20, K=10, zero=0, r=4),     # r = m: every 1-D hit is a solution
]


@pytest.mark.parametrize("case", SMALL, ids=lambda c: "m{m}n{n}K{K}z{zero}r{r}".format(**c))
def test_small_random_vs_brute_force(case):
    for seed in range(3):
        inst = random_small(case["m"], case["n"], 500 + seed, K=case["K"],
                            zero_cols=case["zero"], planted=bool(seed % 2 == 0))
        say("case", case, "seed", seed)
        ref = O.brute(inst.A, inst.d, key_rows=case["r"])
        same(gsolve(inst.A, inst.d, key_rows=case["r"]), ref, f"default {case} {seed}")
        # every run pair checked pair by pair, and decided by the vector join
        same(gsolve(inst.A, inst.d, key_rows=case["r"], verify_join=2), ref,
             f"pairwise {case} {seed}")
        same(gsolve(inst.A, inst.d, key_rows=case["r"], verify_join=1), ref,
             f"vector join {case} {seed}")
        # half records with the packed rows themselves, and with a fingerprint
        # even when the rows take one word
        for rf in (1, 2):
            for vj in (1, 2):
                same(gsolve(inst.A, inst.d, key_rows=case["r"], verify_join=vj,
                            row_fingerprint=rf), ref,
                     f"row_fingerprint={rf} verify_join={vj} {case} {seed}")
        # force hash buckets (modulus below K_d) and a few cell layouts
        # parts 8 and 16 take the XCD-aware work-group mapping
        for lm, lc, parts, jv in [(3, 1, 1, 1), (5, 2, 3, 2), (6, 6, 2, 0), (6, 3, 2, 2),
                                  (5, 2, 8, 1), (6, 3, 16, 2), (3, 1, 2, 3), (8, 3, 8, 3)]:
            for rf in (0, 2):
                g = gsolve(inst.A, inst.d, key_rows=case["r"], log2_m=lm, log2_cells=lc,
                           parts=parts, join_variant=jv, verify_join=2, row_fingerprint=rf)
                same(g, ref, f"M=2^{lm} T=2^{lc} P={parts} join={jv} rows={rf} {case} {seed}")
            # hash buckets decided by the vector join inside the grouped kernel
            for rf in (0, 2):
                g = gsolve(inst.A, inst.d, key_rows=case["r"], log2_m=lm, log2_cells=lc,
                           parts=parts, verify_join=1, row_fingerprint=rf)
                same(g, ref, f"M=2^{lm} T=2^{lc} P={parts} vector join rows={rf} {case} {seed}")


WIDE = [
    dict(m=4, n=18, K=3, zero=3, r=4),      # full digits (s_i = rowsum_i) are common
    dict(m=5, n=22, K=8, zero=0, r=3),
    dict(m=6, n=24, K=100, zero=0, r=5),
]


@pytest.mark.parametrize("case", WIDE, ids=lambda c: "m{m}n{n}K{K}z{zero}r{r}".format(**c))
def test_mixed_radix_key_vs_brute_force(case):
    """key_base = 1: radix rowsum_i + 1 per key row.  Slices select on the
    mixed-radix left key, so the oracle takes the same key_base."""
    r = case["r"]
    for seed in range(2):
        inst = random_small(case["m"], case["n"], 760 + seed, K=case["K"],
                            zero_cols=case["zero"], planted=True)
        say("mixed radix", case, "seed", seed)
        ref = O.brute(inst.A, inst.d, key_rows=r, key_base=1)
        assert ref.H == O.brute(inst.A, inst.d, key_rows=r).H      # same hits, other key
        same(gsolve(inst.A, inst.d, key_rows=r, key_base=1), ref, f"default {case} {seed}")
        same(gsolve(inst.A, inst.d, key_rows=r, key_base=1, verify_join=1), ref,
             f"vector join {case} {seed}")
        same(gsolve(inst.A, inst.d, key_rows=r, key_base=1, verify_join=2), ref,
             f"pairwise {case} {seed}")
        for lm, lc, parts, jv in [(5, 2, 3, 2), (6, 3, 16, 1), (7, 3, 8, 3)]:
            g = gsolve(inst.A, inst.d, key_rows=r, key_base=1, log2_m=lm, log2_cells=lc,
                       parts=parts, join_variant=jv, verify_join=2)
            same(g, ref, f"M=2^{lm} T=2^{lc} P={parts} join={jv} {case} {seed}")
        for s in (0, 5):
            o = O.brute(inst.A, inst.d, key_rows=r, slice_mod=8, slice_res=s, key_base=1)
            g = gsolve(inst.A, inst.d, key_rows=r, key_base=1, slice_mod=8, slice_res=s)
            same(g, o, f"slice 8/{s} {case} {seed}")


def test_mixed_radix_carry_instance_and_bad_radix():
    from paper_2507_05045_amd import msp
    # Row 1 = x1 + x2, row 2 = x3 + .. + x6, d = (0, 2): C(4, 2) = 6 hits; a
    # radix one too small would add 4 carries from s1 = 2.
    A = np.array([[1, 1, 0, 0, 0, 0], [0, 0, 1, 1, 1, 1]], dtype=np.int32)
    d = np.array([0, 2], dtype=np.int32)
    ref = O.brute(A, d, key_rows=2, key_base=1)
    assert ref.H == 6 and ref.nsol == 6
    same(gsolve(A, d, key_rows=2, key_base=1), ref, "carry instance")
    same(gsolve(A, d, key_rows=2, key_base=1, log2_m=2, log2_cells=1, verify_join=2), ref,
         "carry, hash")
    with pytest.raises(msp.MspError):
        gsolve(A, d, key_rows=2, key_base=2)
    ctx = msp.Context(A, d)
    for jv in (1, 2, 3):
        ctx.solve(key_rows=2, key_base=1, log2_m=2, log2_cells=1, join_variant=jv, verify_join=2)
        st = ctx.stats()
        assert (st["key_base"], st["join_grouped"], st["exact_buckets"]) == (1, jv - 1, 0)
        assert ctx.hits() == 6
    ctx.close()


def test_many_buckets_per_window_every_join():
    """Five mixed-radix key rows at (8,70) force M = 2^30: windows would hold
    2^24+ buckets, beyond one work-group per bucket in a HIP grid.  Every join
    variant and the vector join must run and agree on a 1/64 slice."""
    inst = make_instance(8, 70, 0, planted=True)
    kw = dict(key_rows=5, key_base=1, slice_mod=64, slice_res=0)
    ref = gsolve(inst.A, inst.d, **kw)
    assert ref.H > 0
    for extra in (dict(join_variant=1, verify_join=2), dict(join_variant=2, verify_join=2),
                  dict(join_variant=3, verify_join=2), dict(verify_join=1),
                  dict(log2_cells=19, join_variant=2, verify_join=2)):
        say("many buckets", extra)
        same(gsolve(inst.A, inst.d, **kw, **extra), ref, f"{extra}")


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 7])
def test_tiny_and_empty_quarters(n):
    A = np.array([[2] * n, [1] * n, [3] * n], dtype=np.int32)
    d = np.array([2, 1, 3], dtype=np.int32)
    for r in (1, 2, 3):
        for vj in (0, 1, 2):
            same(gsolve(A, d, key_rows=r, verify_join=vj), O.brute(A, d, key_rows=r),
                 f"n={n} r={r} verify_join={vj}")


def test_degenerate_instances():
    rng = np.random.default_rng(3)
    A = rng.integers(0, 50, size=(4, 20)).astype(np.int32)
    rs = A.sum(axis=1)
    cases = {
        "key row infeasible": (1, np.array([rs[0] + 1, 3, 3, 3])),
        "other row infeasible": (1, np.array([rs[0] // 2, rs[1] + 7, 3, 3])),
        "zero target": (2, np.zeros(4, dtype=np.int64)),
        "full target": (2, rs),
    }
    for what, (r, d) in cases.items():
        d = d.astype(np.int32)
        same(gsolve(A, d, key_rows=r), O.brute(A, d, key_rows=r), what)
    Z = np.zeros((2, 16), dtype=np.int32)
    same(gsolve(Z, np.zeros(2, np.int32)), O.brute(Z, np.zeros(2, np.int32)), "all-zero")


def test_slices_partition_the_solve():
    inst = random_small(4, 22, 41, K=20, planted=True)
    full = gsolve(inst.A, inst.d, key_rows=2)
    same(full, O.brute(inst.A, inst.d, key_rows=2), "full")
    tot, sols = 0, []
    for s in range(8):
        g = gsolve(inst.A, inst.d, key_rows=2, slice_mod=8, slice_res=s)
        same(g, O.brute(inst.A, inst.d, key_rows=2, slice_mod=8, slice_res=s), f"slice {s}")
        tot += g.H
        sols += [bytes(x) for x in g.solutions]
    assert tot == full.H
    assert sorted(sols) == sorted(bytes(x) for x in full.solutions)


def test_window_splitting_is_invisible():
    inst = make_instance(4, 30, 0, planted=True)
    ref = gsolve(inst.A, inst.d)
    for wr in (1 << 12, 1 << 14):
        same(gsolve(inst.A, inst.d, window_records=wr), ref, f"window {wr}")
    same(gsolve(inst.A, inst.d, use_torch=False), ref, "library-owned workspace")


def test_solution_capacity():
    # r = m: every 1-D hit is a solution; only max_solutions are stored but
    # |S| stays exact.
    inst = random_small(2, 20, 7, K=5, planted=True)
    ref = O.brute(inst.A, inst.d, key_rows=2, capacity=1 << 20)
    from paper_2507_05045_amd import msp
    ctx = msp.Context(inst.A, inst.d)
    ctx.solve(key_rows=2, max_solutions=5)
    assert ctx.num_solutions() == ref.nsol and ctx.hits() == ref.H
    assert ctx.solutions().shape[0] == min(5, ref.nsol)
    assert satisfies(inst.A, inst.d, ctx.solutions())
    ctx.close()


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


def _golden_instance(e):
    acc = None
    if e["planted"] and (e["m"], e["n"]) == (10, 90):
        probe = make_instance(10, 90, 0)
        acc = lambda x: O.left_key(probe.A, probe.d, x, 4) % 64 == 0  # noqa: E731
    return make_instance(e["m"], e["n"], e["seed"], planted=e["planted"], accept=acc,
                         K=e.get("K", 100))


def _golden_result(e, n):
    sols = np.array([[int(c) for c in s] for s in e["solutions"]], dtype=np.uint8).reshape(-1, n)
    return O.OracleResult(int(e["H"]), e["nsol"], sols)


@pytest.mark.parametrize("cfg", ["4_30", "6_50", "6_50_K50", "6_50_K200"])
def test_full_configs_vs_oracle(cfg):
    m, n = map(int, cfg.split("_")[:2])
    K = int(cfg.split("_K")[1]) if "_K" in cfg else 100
    for e in _golden():
        if (e["m"], e["n"], e.get("K", 100)) != (m, n, K):
            continue
        inst = _golden_instance(e)
        say("config", e["name"])
        kb = e.get("key_base", 0)
        for vj, what in ((0, "planner's choice"), (1, "vector join"), (2, "pairwise")):
            for rf in (0, 2):
                g = gsolve(inst.A, inst.d, key_rows=e["key_rows"], key_base=kb, verify_join=vj,
                           row_fingerprint=rf)
                same(g, _golden_result(e, n), f"{e['name']} {what} rows={rf}")
                if inst.planted is not None:
                    assert any(np.array_equal(s, inst.planted) for s in g.solutions)
        if e["key_rows"] >= 4:
            # ~256 records per bucket and side: the wavefront-per-bucket join
            # in several 64-record chunks, and the heavy join past 256.
            for jv in (1, 3):
                g = gsolve(inst.A, inst.d, key_rows=e["key_rows"], key_base=kb, join_variant=jv,
                           verify_join=2)
                same(g, _golden_result(e, n), e["name"] + f" join variant {jv}")


@pytest.mark.parametrize("cfg", ["8_70", "9_80", "10_90", "8_70_K50", "8_70_K200"])
def test_large_configs_sampled_residue_classes(cfg):
    m, n = map(int, cfg.split("_")[:2])
    K = int(cfg.split("_K")[1]) if "_K" in cfg else 100
    for e in _golden():
        if (e["m"], e["n"], e.get("K", 100)) != (m, n, K):
            continue
        if e["slice_mod"] < (1 << 20):
            continue                     # multi-cell slices: test_multi_cell_slice_shipped_plan
        inst = _golden_instance(e)
        r, kb = e["key_rows"], e.get("key_base", 0)
        say("sampled", e["name"], "r", r, "key_base", kb, e["slice_mod"], e["slice_res"])
        for vj, rf, what in ((0, 0, "planner's choice"), (1, 0, "vector join"),
                             (2, 0, "pairwise"), (2, 2, "pairwise, packed rows")):
            g = gsolve(inst.A, inst.d, key_rows=r, key_base=kb, slice_mod=e["slice_mod"],
                       slice_res=e["slice_res"], verify_join=vj, row_fingerprint=rf)
            same(g, _golden_result(e, n), f"{e['name']} rho={e['slice_res']} {what}")
            if inst.planted is not None:
                assert any(np.array_equal(s, inst.planted) for s in g.solutions)


def test_8_70_slices_partition_the_full_solve():
    """The (8,70) planted twin solved whole and as its 64 residue slices
    k_L mod 64: the slices' H add up to the whole H and their solution sets
    to the whole set.  Five key rows in the mixed radix, and the vector join,
    reach the same solution set by other routes."""
    inst = make_instance(8, 70, 0, planted=True)
    say("full (8,70) planted")
    g = gsolve(inst.A, inst.d, key_rows=4, verify_join=2)
    assert satisfies(inst.A, inst.d, g.solutions)
    assert any(np.array_equal(s, inst.planted) for s in g.solutions)
    assert g.nsol == g.solutions.shape[0]
    tot, sols = 0, []
    for s in range(64):
        p = gsolve(inst.A, inst.d, key_rows=4, slice_mod=64, slice_res=s, verify_join=2)
        tot += p.H
        sols += [bytes(x) for x in p.solutions]
    say("slices", tot, g.H, len(sols), g.nsol)
    assert tot == g.H
    assert sorted(sols) == sorted(bytes(x) for x in g.solutions)
    sset = {bytes(x) for x in g.solutions}
    r5 = gsolve(inst.A, inst.d, key_rows=5, key_base=1)
    assert {bytes(x) for x in r5.solutions} == sset and r5.nsol == g.nsol
    assert r5.H <= g.H
    vj = gsolve(inst.A, inst.d, key_rows=4, verify_join=1)
    assert vj.H == g.H and {bytes(x) for x in vj.solutions} == sset


def test_multi_cell_slice_shipped_plan():
    """A (8,70) slice k_L mod 256 that spans many residue cells, against the
    MITM oracle: with the shipped autotuned plan as it is, and split into
    several windows."""
    from paper_2507_05045_amd import autotune, msp
    for e in _golden():
        if (e["m"], e["n"], e["slice_mod"]) != (8, 70, 256):
            continue
        inst = _golden_instance(e)
        ref = _golden_result(e, 70)
        plan = autotune.lookup(inst.A, 4) or {}
        assert plan, "no shipped plan for (8,70)"
        kw = dict(key_rows=4, slice_mod=256, slice_res=e["slice_res"], **plan)
        for extra in (dict(), dict(window_records=1 << 24), dict(verify_join=2),
                      dict(verify_join=2, window_records=1 << 24),
                      dict(verify_join=2, row_fingerprint=2)):
            ctx = msp.Context(inst.A, inst.d)
            ctx.solve(**kw, **extra)
            st = ctx.stats()
            say("multi-cell slice", e["name"], extra, st["windows"], st["parts"], st["log2_cells"])
            same(ctx.result(), ref, f"{e['name']} {extra}")
            assert st["parts"] == plan.get("parts", st["parts"])
            if "window_records" in extra:
                assert st["windows"] >= 4
            ctx.close()


@pytest.mark.parametrize("lm", [6, 8])
def test_oversized_buckets_vs_oracle(lm):
    # A modulus far below the key range makes buckets of thousands of records
    # per side: the join walks them in chunk pairs and exports big groups.
    for planted in (False, True):
        inst = make_instance(5, 40, 5, planted=planted)
        ref = O.ss_heap(inst.A, inst.d, key_rows=2)
        say("oversized", inst.name, lm)
        for jv in (1, 2):
            same(gsolve(inst.A, inst.d, key_rows=2, log2_m=lm, log2_cells=min(lm, 4),
                        join_variant=jv, verify_join=2), ref, f"{inst.name} M=2^{lm} join={jv}")
        # the vector join takes these buckets in left chunks (heavy kernel)
        same(gsolve(inst.A, inst.d, key_rows=2, log2_m=lm, log2_cells=min(lm, 4), verify_join=1),
             ref, f"{inst.name} M=2^{lm} vector join")


@pytest.mark.parametrize("lm", [9, 10])
def test_grouped_join_mid_buckets_vs_oracle(lm):
    # Buckets of several hundred to over a thousand records per side, with
    # groups of many equal keys: the grouped join walks its group-ordered
    # left rows eight at a time (larger left sides go to the heavy kernel).
    for planted in (False, True):
        inst = make_instance(5, 40, 6, planted=planted)
        ref = O.ss_heap(inst.A, inst.d, key_rows=2)
        say("grouped mid buckets", inst.name, lm)
        for lc in (4, 6):
            same(gsolve(inst.A, inst.d, key_rows=2, log2_m=lm, log2_cells=lc, join_variant=2,
                        verify_join=2), ref, f"{inst.name} M=2^{lm} T=2^{lc} grouped")
            same(gsolve(inst.A, inst.d, key_rows=2, log2_m=lm, log2_cells=lc, verify_join=1),
                 ref, f"{inst.name} M=2^{lm} T=2^{lc} vector join")


def test_vector_join_ties_and_windows():
    # Few distinct values: many left records per run share one packed vector,
    # so a probe walks several equal entries; split windows reuse the table.
    from paper_2507_05045_amd import msp
    for seed in range(3):
        inst = random_small(5, 22, 700 + seed, K=4, planted=True)
        ref = O.brute(inst.A, inst.d, key_rows=1)
        say("vector join ties", seed, ref.H, ref.nsol)
        for wr in (0, 1 << 12):
            ctx = msp.Context(inst.A, inst.d)
            ctx.solve(key_rows=1, verify_join=1, window_records=wr)
            st = ctx.stats()
            assert st["exact_buckets"] == 1 and st["vector_join"] == 1
            same(O.OracleResult(ctx.hits(), ctx.num_solutions(), ctx.solutions()), ref,
                 f"seed {seed} window_records={wr}")
            ctx.close()


def _first_only_vs_oracle(inst, r, **kw):
    """First-solution mode against the oracle: the solve stops after the
    first residue window with a solution; its H and solutions are exactly the
    oracle's over the cells it processed (classes k_L mod T below cells_done)."""
    from paper_2507_05045_amd import msp
    ctx = msp.Context(inst.A, inst.d)
    ctx.solve(key_rows=r, first_only=1, first_order=1, **kw)
    first = ctx.result()
    st = first.stats
    ctx.close()
    assert st["window_order"] == 0
    assert first.nsol >= 1
    assert st["windows"] <= st["windows_total"] and st["cells_done"] >= 1
    ref = O.mitm(inst.A, inst.d, r, st["log2_cells"], 0, st["cells_done"])
    same(first, ref, f"{inst.name} first solution over {st['cells_done']} cells")
    assert satisfies(inst.A, inst.d, first.solutions)
    return first, st


def test_first_solution_mode():
    # Algorithm 2 returns the first x: the solve stops after the first residue
    # window that yields a solution.
    for m, n, r in ((5, 40, 2), (6, 50, 2)):
        inst = make_instance(m, n, 0, planted=True)
        first, st = _first_only_vs_oracle(inst, r, window_records=1 << 16, verify_join=2)
        say("first solution", inst.name, st["windows"], "/", st["windows_total"])
        _first_only_vs_oracle(inst, r, window_records=1 << 16, verify_join=1)
    # (8,70): the returned solutions satisfy Ax = d and lie in the full set.
    inst = make_instance(8, 70, 0, planted=True)
    full = gsolve(inst.A, inst.d, key_rows=4)
    for order in (0, 1):
        g = gsolve(inst.A, inst.d, key_rows=4, first_only=1, first_order=order,
                   window_records=1 << 28)
        assert 1 <= g.nsol <= full.nsol and g.H <= full.H
        assert satisfies(inst.A, inst.d, g.solutions)
        assert {bytes(x) for x in g.solutions} <= {bytes(x) for x in full.solutions}
        assert g.stats["window_order"] == (1 - order)


def test_first_solution_density_order():
    """First-solution mode takes the windows with the most candidate pairs
    first.  With one key row every bucket is one key value, so a window's
    score is its number of 1-D hits: the first window processed must be the
    one the oracle finds with the most hits, and what it returns must be the
    oracle's result over that window when it holds a solution."""
    from paper_2507_05045_amd import msp
    for m, n, seed in ((5, 40, 0), (5, 40, 3)):
        inst = make_instance(m, n, seed, planted=True)
        kw = dict(key_rows=1, verify_join=2, window_records=1 << 14)
        ctx = msp.Context(inst.A, inst.d)
        plan = ctx.plan(**kw)
        assert plan["exact_buckets"] == 1 and plan["windows"] > 4, plan
        ctx.solve(first_only=1, **kw)
        g = ctx.result()
        st = g.stats
        ctx.close()
        kwin, cells, lc = plan["cells_per_window"], plan["cells"], plan["log2_cells"]
        hw = [O.mitm(inst.A, inst.d, 1, lc, w * kwin, min((w + 1) * kwin, cells)).H
              for w in range((cells + kwin - 1) // kwin)]
        best = max(range(len(hw)), key=lambda w: (hw[w], -w))
        say("density order", inst.name, "windows", len(hw), "first", st["first_cell"] // kwin,
            "best", best, "done", st["windows"])
        assert st["window_order"] == 1 and st["first_cell"] == best * kwin
        assert satisfies(inst.A, inst.d, g.solutions) and g.nsol >= 1
        full = O.ss_heap(inst.A, inst.d, key_rows=1)
        assert {bytes(x) for x in g.solutions} <= full.solution_set()
        if st["cells_done"] == min(kwin, cells - best * kwin):      # stopped after one window
            ref = O.mitm(inst.A, inst.d, 1, lc, best * kwin, min((best + 1) * kwin, cells))
            same(g, ref, f"{inst.name} densest window")


WIDE_GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                           "oracle_wide.json")


def test_quarter_split_vs_oracle():
    """Unequal quarters (log2_outer below the balanced q_A) give the oracle's
    result: the (6,50) pair solved whole with one and five key rows, and the
    multi-cell (8,70) slice with the shipped plan's modulus and more cells."""
    from paper_2507_05045_amd import autotune
    for e in _golden():
        if (e["m"], e["n"], e.get("K", 100)) == (6, 50, 100):
            inst = _golden_instance(e)
            r, kb = e["key_rows"], e.get("key_base", 0)
            for lo in (12, 10, 8):
                for vj in (0, 2):
                    g = gsolve(inst.A, inst.d, key_rows=r, key_base=kb, log2_outer=lo,
                               verify_join=vj)
                    say("split", e["name"], r, lo, vj, g.stats["log2_cells"])
                    assert g.stats["log2_outer"] == lo
                    same(g, _golden_result(e, 50), f"{e['name']} r={r} q_A={lo} vj={vj}")
        elif (e["m"], e["n"], e["slice_mod"]) == (8, 70, 256):
            inst = _golden_instance(e)
            plan = dict(autotune.lookup(inst.A, 4) or {})
            plan.pop("log2_outer", None)
            for lo, dc in ((17, 1), (16, 2), (15, 2)):
                kw = dict(plan, log2_cells=plan.get("log2_cells", 15) + dc)
                kw["log2_m"] = max(kw.get("log2_m", 0), kw["log2_cells"])
                g = gsolve(inst.A, inst.d, key_rows=4, slice_mod=256, slice_res=e["slice_res"],
                           log2_outer=lo, **kw)
                say("split", e["name"], lo, kw, g.stats["windows"])
                same(g, _golden_result(e, 70), f"{e['name']} q_A={lo} {kw}")


def test_more_cells_than_2_24_vs_oracle():
    """2^25 - 2^27 residue cells (cell indices past 2^24) on (6,50) with two
    key rows, inner quarters of 2^19 - 2^21 subsets: a residue slice against
    the MITM oracle."""
    for planted in (False, True):
        inst = make_instance(6, 50, 0, planted=planted)
        rho = O.left_key(inst.A, inst.d, inst.planted, 2) % 4096 if planted else 77
        ref = O.mitm(inst.A, inst.d, 2, 12, rho, rho + 1)
        for lc, lo in ((25, 6), (27, 4)):
            g = gsolve(inst.A, inst.d, key_rows=2, log2_m=lc + 10, log2_cells=lc, log2_outer=lo,
                       slice_mod=4096, slice_res=rho)
            say("cells", inst.name, lc, lo, g.H, ref.H, g.stats["windows"])
            assert g.stats["log2_cells"] == lc and g.stats["log2_outer"] == lo
            same(g, ref, f"{inst.name} 2^{lc} cells q_A={lo}")
            if planted:
                assert any(np.array_equal(s, inst.planted) for s in g.solutions)


def test_forced_modulus_plans_sampled_classes():
    """(11,100) with four key rows and (10,90) with five (mixed radix): the
    key room forces a modulus of 2^40 - 2^41, hence 2^28 - 2^29 cells and
    unequal quarters.  Sampled residue classes against the MITM oracle
    (tests/golden/oracle_wide.json), with the planner's plan."""
    from paper_2507_05045_amd import msp
    with open(WIDE_GOLDEN) as f:
        gold = [e for e in json.load(f) if e["key_rows"] in (4, 5)]
    assert len(gold) == 5
    for e in gold:
        inst = make_instance(e["m"], e["n"], e["seed"], planted=e["planted"], K=e["K"])
        assert inst.name == e["name"]
        r, kb = e["key_rows"], e["key_base"]
        ctx = msp.Context(inst.A, inst.d)
        plan = ctx.plan(key_rows=r, key_base=kb, key_words=1)
        assert plan["log2_cells"] >= 28 and plan["log2_outer"] < plan["log2_inner"], plan
        # One key word (the forced modulus), and for five rows also the
        # planner's plan (a second key word, M = 2^35).
        for vj, kwd in (((0, 1), (2, 1)) if r == 4 else ((0, 1), (0, 0))):
            ctx.solve(key_rows=r, key_base=kb, slice_mod=e["slice_mod"],
                      slice_res=e["slice_res"], verify_join=vj, key_words=kwd)
            st = ctx.stats()
            say("forced", e["name"], r, e["slice_res"], vj, kwd, ctx.hits(), e["H"],
                st["log2_m"], st["log2_cells"], st["log2_outer"], st["key_words"], st["ms_total"])
            same(ctx.result(), _golden_result(e, e["n"]), f"{e['name']} r={r} vj={vj} words={kwd}")
            if inst.planted is not None:
                assert any(np.array_equal(s, inst.planted) for s in ctx.solutions())
        ctx.close()


WIDE_SMALL = [
    dict(m=7, n=22, K=100, r=6),
    dict(m=7, n=22, K=100, r=7),            # r = m: every 1-D hit is a solution
    dict(m=8, n=22, K=2, r=7),              # 0/1 rows: large equal-key groups
    dict(m=8, n=24, K=3, r=7),
]


@pytest.mark.parametrize("case", WIDE_SMALL, ids=lambda c: "m{m}n{n}K{K}r{r}".format(**c))
def test_keys_past_int64_vs_brute_force(case):
    """Six or seven key rows in radix n*D (65-80-bit keys): 128-bit sums in
    the count and scatter passes, a second key word per record, every join
    variant and run check, and slices, against brute force."""
    m, n, r = case["m"], case["n"], case["r"]
    for seed in range(2):
        inst = random_small(m, n, 700 + seed, K=case["K"], planted=seed == 0)
        ref = O.brute(inst.A, inst.d, r)
        plans = [dict(), dict(verify_join=1), dict(verify_join=2),
                 dict(log2_m=16, log2_cells=6, join_variant=1, verify_join=2),
                 dict(log2_m=16, log2_cells=8, join_variant=2),
                 dict(log2_m=18, log2_cells=7, join_variant=3, verify_join=2),
                 dict(log2_m=16, log2_cells=5, parts=3, window_records=1 << 12)]
        for kw in plans:
            g = gsolve(inst.A, inst.d, key_rows=r, **kw)
            assert g.stats["key_words"] == 2 and g.stats["key_bits"] > 63
            same(g, ref, f"{inst.name} r={r} {kw}")
        if seed == 0:
            assert any(np.array_equal(s_, inst.planted) for s_ in ref.solutions)
        tot = 0
        for res in range(4):
            b = O.brute(inst.A, inst.d, r, slice_mod=4, slice_res=res)
            g = gsolve(inst.A, inst.d, key_rows=r, slice_mod=4, slice_res=res)
            same(g, b, f"{inst.name} r={r} slice {res}")
            tot += g.H
        assert tot == ref.H


def test_second_key_word_for_header_room_vs_one_word():
    """Keys that fit int64 but not one header (five mixed-radix rows at
    (6,50)): two key words at the default modulus and one word with the
    modulus forced up give the oracle's result."""
    for e in _golden():
        if (e["m"], e["n"], e["key_rows"], e.get("K", 100)) != (6, 50, 5, 100):
            continue
        inst = _golden_instance(e)
        for kwd in (1, 2, 0):
            g = gsolve(inst.A, inst.d, key_rows=5, key_base=1, key_words=kwd)
            assert g.stats["key_words"] == (kwd or 2)
            same(g, _golden_result(e, 50), f"{e['name']} key words {kwd}")


def test_keys_past_int64_vs_oracle():
    """Six key rows: the (6,50) pair in radix n*D (72 bits) solved whole, and
    (10,90) in the mixed radix (73 bits) on sampled classes, against the
    residue MITM oracle (tests/golden/oracle_wide.json)."""
    from paper_2507_05045_amd import msp
    with open(WIDE_GOLDEN) as f:
        gold = [e for e in json.load(f) if e["key_rows"] == 6]
    assert len(gold) == 4
    for e in gold:
        inst = make_instance(e["m"], e["n"], e["seed"], planted=e["planted"], K=e["K"])
        assert inst.name == e["name"]
        kb = e["key_base"]
        ctx = msp.Context(inst.A, inst.d)
        for kw in (dict(), dict(verify_join=2), dict(verify_join=1)):
            ctx.solve(key_rows=6, key_base=kb, slice_mod=e["slice_mod"], slice_res=e["slice_res"],
                      **kw)
            st = ctx.stats()
            say("past int64", e["name"], e["slice_res"], kw, ctx.hits(), e["H"], st["log2_m"],
                st["key_bits"], st["ms_total"])
            assert st["key_words"] == 2 and st["key_bits"] > 63
            same(ctx.result(), _golden_result(e, e["n"]), f"{e['name']} {kw}")
            if inst.planted is not None:
                assert any(np.array_equal(s_, inst.planted) for s_ in ctx.solutions())
        ctx.close()


def test_bucket_of_2_32_records_is_refused():
    """A residue bucket whose parts add up to 2^32 or more records (one key
    value shared by C(43,11) = 5.75e9 left halves: 43 columns of weight 1,
    42 of weight 64, d = 51) cannot be addressed by 32-bit offsets: the
    solve returns MSP_E_NOMEM from the offset pass, before any scatter, and
    the context stays usable.  Every right key is 51 mod 64, so the right
    side of cell 11 enumerates nothing and each part's left count (C(43,11)
    / 64 parts) stays below 2^32: only the bucket's sum over parts wraps."""
    from paper_2507_05045_amd import msp
    A = np.zeros((1, 85), np.int32)
    A[0, :43] = 1
    A[0, 43:] = 64
    ctx = msp.Context(A, [51])
    p = ctx.plan(key_rows=1, verify_join=2, slice_mod=64, slice_res=11)
    assert p["parts"] > 1 and p["cells"] == 1          # each part's counts stay below 2^32
    say("bucket of 5.75e9 records")
    with pytest.raises(msp.MspError) as e:
        ctx.solve(key_rows=1, verify_join=2, slice_mod=64, slice_res=11)
    assert e.value.code == msp.MSP_E_NOMEM
    # Not a device error: the context is not poisoned (the same answer
    # again), and the GPU goes on solving.
    with pytest.raises(msp.MspError) as e:
        ctx.solve(key_rows=1, verify_join=2, slice_mod=64, slice_res=11)
    assert e.value.code == msp.MSP_E_NOMEM
    ctx.close()
    inst = make_instance(4, 30, 0, planted=True)
    g = gsolve(inst.A, inst.d, key_rows=1)
    assert any(np.array_equal(s_, inst.planted) for s_ in g.solutions)


def test_9_80_two_row_class_against_half_counts():
    """x*'s residue class of the (9,80) planted twin with key rows 1-2 and a
    slice modulus above every left key: the class is one pair of left row
    sums (s1, s2), so its H is N_L(s1, s2) * N_R(d1 - s1, d2 - s2), the
    halves' subset counts by row sums from a numpy DP (no oracle): about
    7e12 1-D hits in one equal-key run pair of millions of records per
    side, a class far denser than the average cell (the record buffers are
    sized by window_records).  S is compared with the oracle's, with every
    hit checked pair by pair and with the vector join."""
    from half_counts import half_counts
    inst = make_instance(9, 80, 0, planted=True)
    A64, d = inst.A.astype(np.int64), inst.d.astype(np.int64)
    hl = 40
    NL = half_counts(A64[0, :hl], A64[1, :hl])
    NR = half_counts(A64[0, hl:], A64[1, hl:])
    base = O.key_setup(inst.A, inst.d, 2)[0]
    lm = int(NL.shape[0] - 1 + (NL.shape[1] - 1) * base).bit_length()
    x = inst.planted
    s1, s2 = int(A64[0, :hl] @ x[:hl]), int(A64[1, :hl] @ x[:hl])
    rho = s1 + s2 * base
    nl, nr = int(NL[s1, s2]), int(NR[d[0] - s1, d[1] - s2])
    ref = O.mitm(inst.A, inst.d, 2, lm, rho, rho + 1)
    assert ref.H == nl * nr and ref.H > 10 ** 12
    wr = 1 << max(nl, nr).bit_length()
    for vj in (2, 1):
        say("(9,80) key rows 1-2, class", rho, "mod 2^%d" % lm, "sides", nl, nr,
            "verify_join", vj)
        g = gsolve(inst.A, inst.d, key_rows=2, slice_mod=1 << lm, slice_res=rho,
                   verify_join=vj, window_records=wr)
        same(g, ref, f"(9,80) key rows 1-2, x*'s class, verify_join={vj}")


def test_10_90_two_row_class_against_half_counts():
    """The largest class of (10,90) seed 0 under key rows 1-2 with at most a
    million vectors per side (a modulus above every left key): H against the
    per-half counting DP, S against the oracle, both run checks."""
    from half_counts import half_counts
    inst = make_instance(10, 90, 0)
    A64, d = inst.A.astype(np.int64), inst.d.astype(np.int64)
    hl = 45
    NL = half_counts(A64[0, :hl], A64[1, :hl])
    NR = half_counts(A64[0, hl:], A64[1, hl:])
    base = O.key_setup(inst.A, inst.d, 2)[0]
    lm = int(NL.shape[0] - 1 + (NL.shape[1] - 1) * base).bit_length()
    # NRd[s1, s2] = N_R(d1 - s1, d2 - s2) where defined
    NRd = np.zeros_like(NL)
    r1 = int(d[0]) - np.arange(NL.shape[0])
    r2 = int(d[1]) - np.arange(NL.shape[1])
    ok1, ok2 = (r1 >= 0) & (r1 < NR.shape[0]), (r2 >= 0) & (r2 < NR.shape[1])
    NRd[np.ix_(ok1, ok2)] = NR[np.ix_(r1[ok1], r2[ok2])]
    prod = np.where((NL <= 10 ** 6) & (NRd <= 10 ** 6), NL * NRd, 0)
    s1, s2 = (int(v) for v in np.unravel_index(np.argmax(prod), prod.shape))
    nl, nr = int(NL[s1, s2]), int(NRd[s1, s2])
    assert nl * nr > 10 ** 11
    rho = s1 + s2 * base
    ref = O.mitm(inst.A, inst.d, 2, lm, rho, rho + 1)
    assert ref.H == nl * nr
    wr = 1 << max(nl, nr).bit_length()
    for vj in (2, 1):
        say("(10,90) key rows 1-2, class", rho, "mod 2^%d" % lm, "sides", nl, nr,
            "verify_join", vj)
        g = gsolve(inst.A, inst.d, key_rows=2, slice_mod=1 << lm, slice_res=rho,
                   verify_join=vj, window_records=wr)
        same(g, ref, f"(10,90) key rows 1-2, class {rho}, verify_join={vj}")
