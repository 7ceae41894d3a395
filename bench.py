"""Benchmark: 1-D hits verified per second of the exact market-split solve.

One step = one pass of the whole hot path (quarter lists, residue-cell
sort, bucket count/scatter, join, verify) over one batch of synthetic
instances.  The default workload is the (m, n) = (9, 80) instance of the
hard family (a_ij uniform in [0, 99], d_i = floor(row sum / 2), seed 0) with
rows 1-4 folded into the int64 key: each timed step solves the residue slice
k_L mod 64 = 0 of it (warm-up steps solve other slices), and after the timed
steps the whole (9,80) solve is timed once and reported in the same line.

Prints ONE JSON line (rank 0).  Everything runs on one GPU; --gpus above 1
is refused.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks used for the roofline fraction.
PEAK_HBM_GBS = 8000.0
# Vector ALU: 256 CUs x 64 lanes x 2.4 GHz = 39.3 T 32-bit integer ops/s.
PEAK_ALU_TOPS = 256 * 64 * 2.4e9 / 1e12
# HBM bytes per launch of the dominant kernel, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE runs scaled by a plain-copy calibration; valid only while the
# kernel sources hash to the recorded value.
TRAFFIC = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SOURCES = ("paper_2507_05045_amd/csrc/msp_kernels.hip",
                  "paper_2507_05045_amd/csrc/msp_internal.h")


def kernel_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` on `workload`, or None when no
    counters were taken or the kernels changed since they were."""
    try:
        with open(TRAFFIC) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    e = t.get("workloads", {}).get(workload)
    if not e or t.get("kernel_sources_sha256") != kernel_sources_sha256():
        return None
    e = e.get("kernels", {}).get(kernel)
    if not e:
        return None
    cal = t["calibration"]
    return (e["fetch_kib_per_launch"] * cal["FETCH_SIZE"]
            + e["write_kib_per_launch"] * cal["WRITE_SIZE"]) * 1024.0


WORKLOADS = {
    "6_50": dict(m=6, n=50, key_rows=1, seeds=[0], planted=True, slice_mod=0,
                 desc="(6,50) seed 0 + planted twin, a_ij U[0,99], d = floor(rowsum/2), key row 1"),
    "4_30": dict(m=4, n=30, key_rows=1, seeds=[0], planted=True, slice_mod=0,
                 desc="(4,30) seed 0 + planted twin, key row 1"),
    "8_70": dict(m=8, n=70, key_rows=4, seeds=[0, 1, 2, 3, 4], planted=False, slice_mod=0,
                 desc="(8,70) seeds 0-4, int64 key of rows 1-4 (base 7000)"),
    "9_80": dict(m=9, n=80, key_rows=4, seeds=[0], planted=False, slice_mod=64, whole=True,
                 desc="(9,80) seed 0, key rows 1-4 (base 8000): steps solve the residue slice "
                      "k_L mod 64 = 0, then one whole solve"),
    "9_80_whole": dict(m=9, n=80, key_rows=4, seeds=[0], planted=False, slice_mod=0,
                       desc="(9,80) seed 0 whole solve per step, key rows 1-4 (base 8000)"),
    "10_90s": dict(m=10, n=90, key_rows=4, seeds=[0], planted=False, slice_mod=64,
                   desc="(10,90) seed 0, residue slice k_L mod 64 = 0, key rows 1-4 (base 9000)"),
    # The largest class of Section 4, (11,100): 2^50 pairs per half.  Four
    # key rows (base 10000) need a modulus of 2^40 in the record header, so
    # 2^28 residue cells and unequal quarters (q_A = 22, q_B = 28).
    "11_100s": dict(m=11, n=100, key_rows=4, seeds=[0], planted=False, slice_mod=65536,
                    desc="(11,100) seed 0, residue slice k_L mod 65536 = 0, key rows 1-4 "
                         "(base 10000)"),
    # Five key rows at (10,90) in the mixed radix (a 60-bit key): with two
    # key words per record the modulus stays 2^35 (one word would force
    # 2^41: 2^29 residue cells, unequal quarters q_A = 17, q_B = 28).
    "10_90_r5s": dict(m=10, n=90, key_rows=5, key_base=1, seeds=[0], planted=False,
                      slice_mod=512, desc="(10,90) seed 0, residue slice k_L mod 512 = 0, key "
                                          "rows 1-5 in mixed radix rowsum+1"),
    # Six key rows at (10,90) in the mixed radix: a 73-bit key (128-bit sums,
    # two key words per record).
    "10_90_r6s": dict(m=10, n=90, key_rows=6, key_base=1, seeds=[0], planted=False,
                      slice_mod=64, desc="(10,90) seed 0, residue slice k_L mod 64 = 0, key "
                                         "rows 1-6 in mixed radix rowsum+1 (73-bit key)"),
    # Coefficient range K (Section 4's classes K = 50, 100, 200): a_ij in [0, K).
    "6_50_K50": dict(m=6, n=50, key_rows=1, seeds=[0], planted=True, slice_mod=0, K=50,
                     desc="(6,50) K=50 seed 0 + planted twin, key row 1"),
    "6_50_K200": dict(m=6, n=50, key_rows=1, seeds=[0], planted=True, slice_mod=0, K=200,
                      desc="(6,50) K=200 seed 0 + planted twin, key row 1"),
    "8_70_K50": dict(m=8, n=70, key_rows=4, seeds=[0, 1, 2, 3, 4], planted=False, slice_mod=0,
                     K=50, desc="(8,70) K=50 seeds 0-4, key rows 1-4 (base 7000)"),
    "8_70_K200": dict(m=8, n=70, key_rows=4, seeds=[0, 1, 2, 3, 4], planted=False, slice_mod=0,
                      K=200, desc="(8,70) K=200 seeds 0-4, key rows 1-4 (base 14000)"),
    # Planted twins only (feasible, like the paper's benchmark set); with
    # --first-solution the solve stops at the first verified x (Algorithm 2).
    "8_70p": dict(m=8, n=70, key_rows=4, seeds=[0, 1, 2, 3, 4], planted=True, planted_only=True,
                  slice_mod=0, desc="(8,70) planted twins of seeds 0-4, key rows 1-4"),
    "9_80p": dict(m=9, n=80, key_rows=4, seeds=[0], planted=True, planted_only=True,
                  slice_mod=0, desc="(9,80) planted twin of seed 0, key rows 1-4"),
    # Five key rows in the mixed radix rowsum_i + 1 per row: H shrinks by
    # about the spread of row 5, the residue tables grow (more cells).
    "8_70_r5": dict(m=8, n=70, key_rows=5, key_base=1, seeds=[0, 1, 2, 3, 4], planted=False,
                    slice_mod=0, desc="(8,70) seeds 0-4, key rows 1-5 in mixed radix rowsum+1"),
    "6_50_r5": dict(m=6, n=50, key_rows=5, key_base=1, seeds=[0], planted=True, slice_mod=0,
                    desc="(6,50) seed 0 + planted twin, key rows 1-5 in mixed radix rowsum+1"),
}


def build_instances(w):
    from paper_2507_05045_amd.inputs import make_instance
    out = []
    for s in w["seeds"]:
        K = w.get("K", 100)
        if not w.get("planted_only"):
            out.append(make_instance(w["m"], w["n"], s, key_rows=w["key_rows"], K=K))
        if w["planted"]:
            out.append(make_instance(w["m"], w["n"], s, planted=True, key_rows=w["key_rows"], K=K))
    return out


def host_cpu():
    """CPU model and the cores this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "host_cores": len(os.sched_getaffinity(0))}


def cpu_baseline(w, insts, budget_s=30.0):
    """The oracle as it stands, single-threaded on the host, on a bounded
    sample: the smallest instance of the workload solved whole (n <= 50), or
    residue classes of the larger ones until about budget_s seconds."""
    from oracle import oracle as O
    if w["n"] <= 50:
        inst = insts[-1]
        t = time.perf_counter()
        r = O.ss_heap(inst.A, inst.d, w["key_rows"], key_base=w.get("key_base", 0))
        dt = time.perf_counter() - t
        return {"value": r.H / dt, "unit": "hits/s", "cores": 1, "kind": "oracle",
                "sample": f"{inst.name}: whole solve by the heap Schroeppel-Shamir oracle, "
                          f"H={r.H}, {dt:.2f} s", **host_cpu()}
    inst = insts[0]
    lm = {70: 20, 80: 24, 90: 26, 100: 30}.get(w["n"], 20)
    t = time.perf_counter()
    H, k = 0, 0
    while time.perf_counter() - t < budget_s and k < 64:
        rho = (12345 + 64 * k) % (1 << lm)     # classes inside the k_L mod 64 = 0 slice family
        H += O.mitm(inst.A, inst.d, w["key_rows"], lm, rho, rho + 1,
                    key_base=w.get("key_base", 0)).H
        k += 1
    dt = time.perf_counter() - t
    return {"value": H / dt, "unit": "hits/s", "cores": 1, "kind": "oracle",
            "sample": f"{inst.name}: {k} residue classes mod 2^{lm} by the residue "
                      f"meet-in-the-middle oracle, H={H}, {dt:.2f} s", **host_cpu()}


def _pct(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs, dtype=float), q)) if len(xs) else None


def run_stream(args):
    out = stream_results(args.stream_count, not args.no_closed_loop, args.stream_max_m)
    print(json.dumps(out), flush=True)


def stream_results(count, closed_loop=True, max_m=8):
    """Uneven stream (m in {5..8}, n = 10(m-1), r = m - 4, odd instances
    planted): plain one-at-a-time solves, one batched solve, served runs
    with Poisson arrivals at 0.5 and 0.9 of the plain throughput (each beside
    the plain path's latencies for the same arrivals, solved one at a time in
    arrival order), plus a closed-loop served run with every request at
    t = 0."""
    import threading
    import torch
    from paper_2507_05045_amd import autotune, msp
    from paper_2507_05045_amd.inputs import poisson_arrivals, stream_instances

    def say(*a):                     # progress on stderr; the JSON line stays alone on stdout
        print(*a, file=sys.stderr, flush=True)

    insts = [i for i in stream_instances(count) if i.m <= max_m]
    opts = []
    for i in insts:
        o = dict(key_rows=i.key_rows)
        t = autotune.lookup(i.A, i.key_rows)
        if t:
            o.update(t)
        opts.append(o)
    # Warm-up: one solve per (m, n) class.
    seen = set()
    for i, o in zip(insts, opts):
        if i.m not in seen:
            seen.add(i.m)
            c = msp.Context(i.A, i.d)
            c.solve(**o)
            c.close()
    torch.cuda.synchronize()
    say(f"stream: {len(insts)} instances, warm-up done")

    # Plain: one instance at a time, each with its own context and the
    # binding's default workspace (PyTorch's caching allocator, so repeated
    # solves do not pay a device allocation each: a library-owned workspace
    # would add hipMalloc/hipFree of up to tens of GB per instance).
    lat, hits = [], 0
    t0 = time.perf_counter()
    ref = []
    for i, o in zip(insts, opts):
        t1 = time.perf_counter()
        c = msp.Context(i.A, i.d)
        c.solve(**o)
        ref.append((c.hits(), c.num_solutions()))
        hits += ref[-1][0]
        c.close()
        lat.append(time.perf_counter() - t1)
        if len(lat) % 32 == 0:
            say(f"plain: {len(lat)}/{len(insts)} solved, {time.perf_counter() - t0:.1f} s")
    t_plain = time.perf_counter() - t0
    plain = {"makespan_s": t_plain, "hits_per_s": hits / t_plain,
             "instances_per_s": len(insts) / t_plain,
             "p50_ms": _pct(lat, 50) * 1e3, "p99_ms": _pct(lat, 99) * 1e3}

    # Batched: msp_batch_solve over the stream, in calls of at most 128
    # instances (each call reports when it ends).
    # Batched and served arenas come from PyTorch's caching allocator as well
    # (msp_set_allocator), so each batch call does not allocate its own.
    arena = msp.TorchArena().__enter__()
    ctxs = [msp.Context(i.A, i.d) for i in insts]
    t0 = time.perf_counter()
    for k0 in range(0, len(ctxs), 128):
        rc = msp.batch_solve(ctxs[k0:k0 + 128], opts[k0:k0 + 128], max_slots=16)
        assert rc == 0, msp.strerror(rc)
        say(f"batched: {min(k0 + 128, len(ctxs))}/{len(ctxs)} solved, "
            f"{time.perf_counter() - t0:.1f} s")
    t_batch = time.perf_counter() - t0
    assert all((c.hits(), c.num_solutions()) == r for c, r in zip(ctxs, ref)), "batched != plain"
    batched = {"makespan_s": t_batch, "hits_per_s": hits / t_batch,
               "instances_per_s": len(insts) / t_batch, "calls": (len(insts) + 127) // 128}
    for c in ctxs:
        c.close()

    def served(arrivals):
        srv = msp.Server(max_slots=16)
        cs = [msp.Context(i.A, i.d) for i in insts]
        tickets = [None] * len(insts)

        def feeder():
            start = time.perf_counter()
            for k, (c, o) in enumerate(zip(cs, opts)):
                dt = arrivals[k] - (time.perf_counter() - start)
                if dt > 0:
                    time.sleep(dt)
                tickets[k] = srv.submit(c, **o)
                if (k + 1) % 64 == 0:
                    say(f"served: {k + 1}/{len(cs)} submitted, {time.perf_counter() - start:.1f} s")

        th = threading.Thread(target=feeder)
        t0 = time.perf_counter()
        th.start()
        th.join()
        for k, t in enumerate(tickets):
            assert srv.wait(t) == 0
            if (k + 1) % 64 == 0:
                say(f"served: {k + 1}/{len(tickets)} done, {time.perf_counter() - t0:.1f} s")
        make = time.perf_counter() - t0
        times = [srv.times(t) for t in tickets]
        assert all((c.hits(), c.num_solutions()) == r for c, r in zip(cs, ref)), "served != plain"
        lat = [(t[3] - t[0]) for t in times]
        first, last = min(t[0] for t in times), max(t[3] for t in times)
        srv.stop()
        for c in cs:
            c.close()
        return {"makespan_s": make, "hits_per_s": hits / (last - first),
                "p50_ms": _pct(lat, 50) * 1e3, "p99_ms": _pct(lat, 99) * 1e3,
                "mean_queue_ms": sum(t[1] - t[0] for t in times) / len(times) * 1e3}

    def plain_fifo(arrivals):
        # The plain path under the same arrivals: one solve at a time in
        # arrival order, each taking its measured plain time (waiting
        # included), p50/p99 of arrival-to-finish.
        t_free, out = 0.0, []
        for a, s_ in zip(arrivals, lat):
            start = max(a, t_free)
            t_free = start + s_
            out.append(t_free - a)
        return {"p50_ms": _pct(out, 50) * 1e3, "p99_ms": _pct(out, 99) * 1e3}

    # Poisson arrivals at half and at 0.9 of the plain path's throughput
    # (below what one GPU sustains), served with continuous batching, beside
    # the plain path's own latencies for the same arrivals.
    rate = 0.5 * plain["instances_per_s"]
    arr = poisson_arrivals(len(insts), rate, seed=7)
    poisson = served(arr)
    poisson["rate_per_s"] = rate
    poisson["plain_fifo"] = plain_fifo(arr)
    rate9 = 0.9 * plain["instances_per_s"]
    arr9 = poisson_arrivals(len(insts), rate9, seed=8)
    same = served(arr9)
    same["rate_per_s"] = rate9
    same["plain_fifo"] = plain_fifo(arr9)
    closed = served([0.0] * len(insts)) if closed_loop else None
    arena.__exit__(None, None, None)
    ms = [int(i.m) for i in insts]
    out = {
        "metric": "1-D hits verified/s (served stream) + p50/p99 latency",
        "value": poisson["hits_per_s"], "unit": "hits/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": poisson["makespan_s"] * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u16x2/i64", "data": "synthetic",
        "config": {"workload": f"stream of {len(insts)} instances, m in 5..{max_m} "
                               f"({', '.join(f'{m}:{ms.count(m)}' for m in (5, 6, 7, 8))}), "
                               "n = 10(m-1), key rows m-4, odd instances planted",
                   "instances": len(insts)},
        "hits_total": hits,
        "plain": plain, "batched": batched, "served_poisson": poisson,
        "served_poisson_0.9": same, "served_closed": closed,
        "speedup_vs_plain": {"batched": t_plain / t_batch,
                             "served_closed": t_plain / closed["makespan_s"] if closed else None},
    }
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="9_80", choices=sorted(WORKLOADS) + ["stream"])
    ap.add_argument("--no-whole", action="store_true",
                    help="skip the whole solve after the timed slice steps (9_80)")
    ap.add_argument("--no-first", action="store_true",
                    help="skip the time to the first solution of the planted twin (9_80)")
    ap.add_argument("--no-stream", action="store_true",
                    help="skip the 32-instance plain/batched/served stream (9_80)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--first-solution", action="store_true",
                    help="stop each solve at the first verified solution (time to first solution)")
    ap.add_argument("--verify-join", action="store_true",
                    help="decide exact-bucket runs by the vector hash join; the metric becomes "
                         "1-D hits covered/s (pairs decided, not compared one by one)")
    ap.add_argument("--planner-join", action="store_true",
                    help="let the planner choose how runs are decided (the vector join for large "
                         "equal-key groups); the metric becomes hits covered/s where it does")
    ap.add_argument("--stream-count", type=int, default=64,
                    help="instances of the uneven stream for --workload stream")
    ap.add_argument("--stream-max-m", type=int, default=8,
                    help="keep only the stream's instances with m <= this (5: the smallest, "
                         "sub-millisecond solves)")
    ap.add_argument("--no-closed-loop", action="store_true",
                    help="stream: skip the closed-loop served run (all requests at t = 0)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (calibrates rocprofv3 byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        x = torch.ones(1 << 30, dtype=torch.uint8, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 1 << 30, "copies": 3}), flush=True)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: --gpus must be 1 (the residue classes would "
              "shard across GPUs with one all-reduce at the end; that path is not provided)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2507_05045_amd import autotune, msp
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.workload == "stream":
        return run_stream(args)
    w = WORKLOADS[args.workload]
    insts = build_instances(w)
    ctxs = [msp.Context(i.A, i.d) for i in insts]
    kw = dict(key_rows=w["key_rows"], key_base=w.get("key_base", 0), slice_mod=w["slice_mod"],
              slice_res=0,
              first_only=1 if args.first_solution else 0,
              # The timed steps check every 1-D hit pair by pair (the metric
              # is hits verified); --verify-join decides runs by the hash join.
              verify_join=1 if args.verify_join else 0 if args.planner_join else 2)
    # The plan (modulus, cells, parts, join variant) the autotuner picked for
    # each instance class; the planner's defaults where it has no entry.
    plans = [autotune.lookup(i.A, w["key_rows"], w.get("key_base", 0)) or {} for i in insts]

    def step(res=0):
        stats = []
        for c, pl in zip(ctxs, plans):
            c.solve(**{**kw, "slice_res": res}, **pl)
            stats.append(c.stats())
        return stats

    # Sliced workloads warm up on slices of their own (residues 1, 2, ...);
    # the timed steps all solve residue 0.
    for k in range(args.warmup):
        step((1 + k) % w["slice_mod"] if w["slice_mod"] else 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    all_stats = []
    for k in range(args.steps):
        all_stats.append(step())
        if args.steps > 1:
            print(f"step {k + 1}/{args.steps}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    hits = sum(c.hits() for c in ctxs)
    nsol = [c.num_solutions() for c in ctxs]
    ms_step = dt * 1e3 / args.steps
    whole = None
    if w.get("whole") and not args.no_whole:
        # One whole solve of every instance, timed on its own.
        torch.cuda.synchronize()
        tw = time.perf_counter()
        wstats = []
        for c, pl in zip(ctxs, plans):
            # The whole solve takes the planner's choice of run check.
            c.solve(**{**kw, "slice_mod": 0, "slice_res": 0, "verify_join": 0}, **pl)
            wstats.append(c.stats())
        torch.cuda.synchronize()
        tw = time.perf_counter() - tw
        whole = {"solve_s": tw, "H": [c.hits() for c in ctxs],
                 "solutions": [c.num_solutions() for c in ctxs],
                 "hits_per_s": sum(c.hits() for c in ctxs) / tw,
                 "phase_s": {k: sum(s[k] for s in wstats) / 1e3 for k in
                             ("ms_scatter", "ms_join", "ms_count", "ms_verify", "ms_scan",
                              "ms_quarters")},
                 "windows": [s["windows"] for s in wstats],
                 "vector_join": [s["vector_join"] for s in wstats]}

    # Dominant kernel: the phase with the most time, from HIP events recorded
    # on the solve's stream inside the library (summed per step).
    flat = [s for st in all_stats for s in st]
    tot = {k: sum(s[k] for s in flat) for k in
           ("ms_verify", "ms_scatter", "ms_join", "ms_count", "ms_quarters")}
    launches_v = sum(s["verify_launches"] for s in flat)
    windows = sum(s["windows"] for s in flat)
    rec_bytes = flat[0]["record_bytes"]
    records = sum(s["records_left"] + s["records_right"] for s in flat)
    dom = max(tot, key=tot.get)
    vjoin = any(s["vector_join"] for s in flat)
    if dom == "ms_verify" and vjoin:
        # Vector join: every half record of a run is read once (insert or
        # probe) and touches one 4-byte table slot.
        vb = records * (rec_bytes + 4) / max(launches_v, 1)
        avg_s = tot["ms_verify"] / 1e3 / max(launches_v, 1)
        achieved = vb / avg_s / 1e9
        roof = {"kernel": "k_vjoin_insert+k_vjoin_probe", "bound": "hbm", "achieved": achieved,
                "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                "traffic": None, "avg_launch_ms": avg_s * 1e3,
                "algorithmic": f"{rec_bytes} B record + 4 B table slot per half record"}
    elif dom == "ms_verify":
        # One 32-bit compare of the first packed word is the least ALU work a
        # pairwise check of a 1-D hit can do.
        ops_per_launch = hits * args.steps / max(launches_v, 1)
        avg_s = tot["ms_verify"] / 1e3 / max(launches_v, 1)
        achieved = ops_per_launch / avg_s / 1e12
        roof = {"kernel": "k_verify", "bound": "alu", "achieved": achieved,
                "peak": PEAK_ALU_TOPS, "unit": "Tops/s", "frac": achieved / PEAK_ALU_TOPS,
                "traffic": measured_traffic(args.workload, "k_verify"),
                "avg_launch_ms": avg_s * 1e3,
                "algorithmic": "1 int32 compare per 1-D hit"}
    else:
        join_k = ("k_join_light", "k_join_grouped", "k_join_pairs")[flat[0]["join_grouped"]]
        # One-word records (fingerprint or one packed word) and fingerprint
        # records with a second key word (16 bytes) take k_scatter_rec.
        scat_k = ("k_scatter_rec" if flat[0]["record_bytes"] <= 12 or flat[0]["row_fingerprint"]
                  else "k_scatter_staged")
        key = {"ms_scatter": scat_k, "ms_join": join_k,
               "ms_count": "k_count", "ms_quarters": "k_quarter_gen"}.get(dom, dom)
        bytes_per_launch = records * rec_bytes / max(windows, 1)
        avg_s = tot[dom] / 1e3 / max(windows, 1)
        achieved = bytes_per_launch / avg_s / 1e9
        roof = {"kernel": key, "bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                "traffic": measured_traffic(args.workload, key),
                "avg_launch_ms": avg_s * 1e3,
                "algorithmic": f"{rec_bytes} B per half record written (scatter) or read (join)"}

    out = {
        "metric": "1-D hits covered/s" if vjoin else "1-D hits verified/s",
        "value": hits / (dt / args.steps),
        "unit": "hits/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u16x2/i64",
        "data": "synthetic",
        "config": {"workload": w["desc"], "m": w["m"], "n": w["n"], "key_rows": w["key_rows"],
                   "instances": len(insts), "slice_mod": w["slice_mod"], "plan": plans[0]},
        "hits_per_step": hits,
        "solutions": nsol,
        "first_solution": bool(args.first_solution),
        "solve_ms": [round(s["ms_total"], 3) for s in all_stats[-1]],
        "windows": [f"{s['windows']}/{s['windows_total']}" for s in all_stats[-1]],
        "phase_ms_per_step": {k: v / args.steps for k, v in tot.items()},
        "roofline": roof,
    }
    if whole is not None:
        out["whole_solve"] = whole
    if w.get("whole") and not args.no_first:
        # Time to the first solution (Algorithm 2 returns the first x) on the
        # planted twin of the same class: the paper's benchmark instances are
        # feasible, and its table times are most likely times to a first x.
        from paper_2507_05045_amd.inputs import make_instance
        tw = make_instance(w["m"], w["n"], w["seeds"][0], planted=True, key_rows=w["key_rows"])
        c = msp.Context(tw.A, tw.d)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        c.solve(**{**kw, "slice_mod": 0, "slice_res": 0, "verify_join": 0, "first_only": 1},
                **plans[0])
        torch.cuda.synchronize()
        t1 = time.perf_counter() - t1
        st = c.stats()
        sols = c.solutions()
        out["time_to_first_solution"] = {
            "instance": tw.name, "seconds": t1, "solutions": int(c.num_solutions()),
            "planted_found": bool(any((x == tw.planted).all() for x in sols)),
            "windows": f"{st['windows']}/{st['windows_total']}"}
        c.close()
    if w.get("whole") and not args.no_stream:
        # Plain, batched and served solves of an uneven stream of 32 instances.
        print("stream of 32 instances ...", file=sys.stderr, flush=True)
        out["stream"] = stream_results(32, closed_loop=True)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, insts)
    print(json.dumps(out), flush=True)
    for c in ctxs:
        c.close()


if __name__ == "__main__":
    main()
