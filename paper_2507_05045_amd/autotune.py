"""Autotuner for the solve plan: residue modulus M = 2^log2_m, residue cells
T = 2^log2_cells, work-groups per cell (parts) and the quarter split
(log2_outer).

For an instance class (m, n, key rows r, coefficient bound) it times a few
candidates around the planner's default on a residue slice of a
representative instance (the slice k_L mod 2^s = 0 keeps 1/2^s of the cells,
so timing stays short), checks that every candidate returns the same 1-D hit
count (the plan must never change the result), and caches the fastest in a
JSON file keyed by GPU architecture and class.  The cache path is
``$MSP_TUNE_CACHE`` or ``~/.cache/msp_tune.json``.

All timing goes through the C ABI (``msp_solve``); nothing here computes any
part of the solve.
"""
from __future__ import annotations

import json
import os
import time
from typing import Dict, Optional

from . import msp

CACHE = os.environ.get("MSP_TUNE_CACHE", os.path.expanduser("~/.cache/msp_tune.json"))
# Plans tuned on an MI355X for the workloads of this repository, shipped
# with the package and consulted when the user cache has no entry.
SHIPPED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_gfx950.json")


def _arch() -> str:
    try:
        import torch
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:  # no torch or no GPU: still a valid cache key
        return "gfx950"


def class_key(A, key_rows: int, key_base: int = 0) -> str:
    import numpy as np
    A = np.asarray(A)
    kb = ":kb1" if key_base else ""
    return f"{_arch()}:m{A.shape[0]}:n{A.shape[1]}:r{key_rows}{kb}:amax{int(A.max())}"


def _load() -> Dict[str, dict]:
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(cache: Dict[str, dict]):
    os.makedirs(os.path.dirname(CACHE) or ".", exist_ok=True)
    tmp = CACHE + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, CACHE)


def lookup(A, key_rows: int, key_base: int = 0) -> Optional[dict]:
    key = class_key(A, key_rows, key_base)
    hit = _load().get(key)
    if hit is None:
        try:
            with open(SHIPPED) as f:
                hit = json.load(f).get(key)
        except (OSError, ValueError):
            hit = None
    return hit["opts"] if hit else None


def tune(A, d, key_rows: int = 1, max_seconds: float = 20.0, slice_bits: Optional[int] = None,
         force: bool = False, verbose: bool = False, key_base: int = 0) -> dict:
    """Return the fastest plan options for this instance's class (cached)."""
    key = class_key(A, key_rows, key_base)
    cache = _load()
    if key in cache and not force:
        return cache[key]["opts"]
    ctx = msp.Context(A, d)
    # With a slice given, the planner's default is read off a sliced solve:
    # a whole solve of a large class can take minutes.
    ctx.solve(key_rows=key_rows, key_base=key_base,
              **(dict(slice_mod=1 << slice_bits, slice_res=0) if slice_bits else {}))
    base = ctx.stats()
    full_ms = base["ms_total"]
    lm, lc, parts = base["log2_m"], base["log2_cells"], base["parts"]
    qa = base["log2_outer"]
    if slice_bits is None:
        # Aim at ~0.2 s per timed solve; the slice must stay a set of cells.
        s = 0
        while full_ms / (1 << s) > 200.0 and s < min(lc, 10):
            s += 1
        slice_bits = s
    sl = dict(slice_mod=(1 << slice_bits) if slice_bits else 0, slice_res=0)
    cands = []
    for dm in ((0,) if base["exact_buckets"] else (0, -1, 1)):
        for dc in (0, -1, 1):
            m2, c2 = lm + dm, lc + dc
            if c2 < max(slice_bits, 0) or c2 > m2 or m2 - c2 > 12 or c2 > 29 or m2 < 1:
                continue
            # multiples of 8 let the kernels map whole parts to each XCD
            for p2 in sorted({parts, parts * 2, parts * 4, 16, 32, 64}):
                for jv in ((0,) if base["exact_buckets"] else (1, 2, 3)):
                    cands.append(dict(log2_m=m2, log2_cells=c2, parts=min(p2, 256),
                                      join_variant=jv))
            # One or two variables moved to the inner quarters: more cells
            # for the same outer re-reads.
            for q2 in (qa - 1, qa - 2):
                if q2 >= 1 and dc >= 0:
                    cands.append(dict(log2_m=m2, log2_cells=c2, parts=parts, join_variant=0,
                                      log2_outer=q2))
    t_end = time.time() + max_seconds
    best, best_t, ref_h = None, float("inf"), None
    for c in cands:
        if time.time() > t_end:
            break
        try:
            ctx.solve(key_rows=key_rows, key_base=key_base, **c, **sl)
        except msp.MspError as e:
            if e.code == msp.MSP_E_DEVICE:        # the context is poisoned: start afresh
                ctx.close()
                ctx = msp.Context(A, d)
            continue
        h = ctx.hits()
        if ref_h is None:
            ref_h = h
        if h != ref_h:
            raise RuntimeError(f"plan {c} changed the hit count: {h} != {ref_h}")
        t0 = time.perf_counter()
        ctx.solve(key_rows=key_rows, key_base=key_base, **c, **sl)
        dt = time.perf_counter() - t0
        if verbose:
            print(f"  {c} {dt * 1e3:.1f} ms", flush=True)
        if dt < best_t:
            best, best_t = c, dt
    ctx.close()
    if best is None:
        best = dict(log2_m=lm, log2_cells=lc, parts=parts, join_variant=0,
                    log2_outer=qa)                                     # planner's choice
    cache = _load()
    cache[key] = {"opts": best, "slice_bits": slice_bits, "ms_slice": best_t * 1e3,
                  "default": dict(log2_m=lm, log2_cells=lc, parts=parts)}
    _save(cache)
    return best
