"""Thin ctypes binding of libmsp (include/msp.h), same names as the C ABI.

Only argument marshalling lives here: every step of the solve runs in the
HIP kernels of ``libmsp.so``.  PyTorch, when present with a GPU, supplies
the device workspace (a ``torch.uint8`` CUDA tensor) and the stream (the
current torch stream); otherwise the library allocates its own.

Importing this module loads the in-tree ``libmsp.so`` and raises if it is
missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmsp.so")

MSP_OK = 0
MSP_E_NOMEM = -5
MSP_E_DEVICE = -6
MSP_E_CANCELLED = -7
MSP_E_TRUNCATED = -8


class MspError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {strerror(code)} ({code})")
        self.code = code


class msp_opts(C.Structure):
    _fields_ = [("key_rows", C.c_int32), ("log2_m", C.c_int32), ("log2_cells", C.c_int32),
                ("parts", C.c_int32), ("slice_mod", C.c_int64), ("slice_res", C.c_int64),
                ("max_solutions", C.c_uint64), ("window_records", C.c_uint64),
                ("workspace", C.c_void_p), ("workspace_bytes", C.c_uint64),
                ("stream", C.c_void_p), ("first_only", C.c_int32), ("join_variant", C.c_int32),
                ("verify_join", C.c_int32), ("key_base", C.c_int32),
                ("row_fingerprint", C.c_int32), ("first_order", C.c_int32),
                ("log2_outer", C.c_int32), ("key_words", C.c_int32)]


class msp_stats_t(C.Structure):
    _fields_ = [("ms_total", C.c_double), ("ms_quarters", C.c_double), ("ms_count", C.c_double),
                ("ms_scan", C.c_double), ("ms_scatter", C.c_double), ("ms_join", C.c_double),
                ("ms_verify", C.c_double), ("records_left", C.c_uint64),
                ("records_right", C.c_uint64), ("windows", C.c_uint64),
                ("verify_launches", C.c_uint64), ("verify_pairs", C.c_uint64),
                ("record_bytes", C.c_uint64), ("log2_m", C.c_int32), ("log2_cells", C.c_int32),
                ("parts", C.c_int32), ("key_rows", C.c_int32), ("exact_buckets", C.c_int32),
                ("words", C.c_int32), ("complete", C.c_int32), ("vector_join", C.c_int32),
                ("windows_total", C.c_uint64), ("join_grouped", C.c_int32),
                ("key_base", C.c_int32), ("row_fingerprint", C.c_int32),
                ("cells_done", C.c_uint64), ("window_order", C.c_int32), ("log2_outer", C.c_int32),
                ("first_cell", C.c_uint64), ("key_words", C.c_int32), ("key_bits", C.c_int32)]


class msp_batch_opts(C.Structure):
    _fields_ = [("hbm_budget", C.c_uint64), ("max_slots", C.c_int32), ("reserved", C.c_int32)]


class msp_plan_t(C.Structure):
    _fields_ = [("key_rows", C.c_int32), ("log2_m", C.c_int32), ("log2_cells", C.c_int32),
                ("log2_fine", C.c_int32), ("parts", C.c_int32), ("exact_buckets", C.c_int32),
                ("words", C.c_int32), ("join_variant", C.c_int32), ("vector_join", C.c_int32),
                ("key_base", C.c_int32), ("infeasible", C.c_int32), ("row_fingerprint", C.c_int32),
                ("log2_outer", C.c_int32), ("log2_inner", C.c_int32),
                ("cells", C.c_uint64), ("cells_per_window", C.c_uint64), ("windows", C.c_uint64),
                ("window_records", C.c_uint64), ("record_bytes", C.c_uint64),
                ("workspace_bytes", C.c_uint64), ("max_grid_items", C.c_uint64),
                ("key_words", C.c_int32), ("key_bits", C.c_int32)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
RELEASE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


# Every symbol include/msp.h declares (checked by the CPU test suite).
EXPORTS = ["msp_create", "msp_default_opts", "msp_solve", "msp_num_solutions", "msp_hits",
           "msp_get_solutions", "msp_stats", "msp_destroy", "msp_strerror",
           "msp_workspace_bytes", "msp_batch_solve", "msp_server_start", "msp_server_submit",
           "msp_server_poll", "msp_server_wait", "msp_server_cancel", "msp_server_times",
           "msp_server_stop", "msp_plan", "msp_set_allocator", "msp_solve_noalloc"]

# PyTorch-ROCm ships its own HIP runtime with the same soname as the system
# one.  Load torch first so that libmsp binds to the runtime torch uses:
# two HIP runtimes in one process do not share devices, memory or streams.
try:
    import torch  # noqa: F401
except ImportError:  # the library also runs without torch
    torch = None

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with "
                      "`python paper_2507_05045_amd/build.py` (no CPU fallback)")
lib = C.CDLL(LIB_PATH)
_p = C.POINTER
lib.msp_create.argtypes = [_p(C.c_int32), _p(C.c_int32), C.c_int32, C.c_int32, _p(C.c_void_p)]
lib.msp_create.restype = C.c_int
lib.msp_default_opts.argtypes = [_p(msp_opts)]
lib.msp_default_opts.restype = None
lib.msp_solve.argtypes = [C.c_void_p, _p(msp_opts)]
lib.msp_solve.restype = C.c_int
lib.msp_num_solutions.argtypes = [C.c_void_p, _p(C.c_uint64)]
lib.msp_num_solutions.restype = C.c_int
lib.msp_hits.argtypes = [C.c_void_p, _p(C.c_uint64), _p(C.c_uint64)]
lib.msp_hits.restype = C.c_int
lib.msp_get_solutions.argtypes = [C.c_void_p, _p(C.c_uint8), C.c_uint64, _p(C.c_uint64)]
lib.msp_get_solutions.restype = C.c_int
lib.msp_stats.argtypes = [C.c_void_p, _p(msp_stats_t)]
lib.msp_stats.restype = C.c_int
lib.msp_destroy.argtypes = [C.c_void_p]
lib.msp_destroy.restype = None
lib.msp_strerror.argtypes = [C.c_int]
lib.msp_strerror.restype = C.c_char_p
lib.msp_workspace_bytes.argtypes = [C.c_void_p, _p(msp_opts)]
lib.msp_workspace_bytes.restype = C.c_uint64
lib.msp_batch_solve.argtypes = [_p(C.c_void_p), _p(msp_opts), C.c_int32, _p(msp_batch_opts)]
lib.msp_batch_solve.restype = C.c_int
lib.msp_server_start.argtypes = [_p(msp_batch_opts), _p(C.c_void_p)]
lib.msp_server_start.restype = C.c_int
lib.msp_server_submit.argtypes = [C.c_void_p, C.c_void_p, _p(msp_opts), _p(C.c_uint64)]
lib.msp_server_submit.restype = C.c_int
lib.msp_server_poll.argtypes = [C.c_void_p, C.c_uint64, _p(C.c_int32), _p(C.c_int32)]
lib.msp_server_poll.restype = C.c_int
lib.msp_server_wait.argtypes = [C.c_void_p, C.c_uint64, _p(C.c_int32)]
lib.msp_server_wait.restype = C.c_int
lib.msp_server_cancel.argtypes = [C.c_void_p, C.c_uint64]
lib.msp_server_cancel.restype = C.c_int
lib.msp_server_times.argtypes = [C.c_void_p, C.c_uint64, _p(C.c_double)]
lib.msp_server_times.restype = C.c_int
lib.msp_server_stop.argtypes = [C.c_void_p]
lib.msp_server_stop.restype = C.c_int
lib.msp_solve_noalloc.argtypes = [C.c_void_p, _p(msp_opts)]
lib.msp_solve_noalloc.restype = C.c_int
lib.msp_plan.argtypes = [C.c_void_p, _p(msp_opts), _p(msp_plan_t)]
lib.msp_plan.restype = C.c_int
lib.msp_set_allocator.argtypes = [ALLOC_FN, RELEASE_FN, C.c_void_p]
lib.msp_set_allocator.restype = C.c_int


def strerror(code: int) -> str:
    return lib.msp_strerror(code).decode()


def _check(rc: int, what: str):
    if rc != MSP_OK:
        raise MspError(rc, what)


def msp_default_opts(**kw) -> msp_opts:
    o = msp_opts()
    lib.msp_default_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


@dataclass
class Result:
    H: int                       # 1-D hits (128-bit, exact)
    nsol: int                    # |S|
    solutions: np.ndarray        # (stored, n) uint8, canonical order
    stats: dict


class Context:
    """Owns one msp_ctx (msp_create ... msp_destroy)."""

    def __init__(self, A, d):
        A = np.ascontiguousarray(np.asarray(A, dtype=np.int32))
        d = np.ascontiguousarray(np.asarray(d, dtype=np.int32))
        if A.ndim != 2 or d.shape != (A.shape[0],):
            raise ValueError("A must be (m, n) and d (m,)")
        self.m, self.n = A.shape
        self._ctx = C.c_void_p()
        _check(lib.msp_create(A.ctypes.data_as(_p(C.c_int32)), d.ctypes.data_as(_p(C.c_int32)),
                              self.m, self.n, C.byref(self._ctx)), "msp_create")
        self._ws = None

    def close(self):
        if self._ctx:
            lib.msp_destroy(self._ctx)
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self, opts: msp_opts) -> int:
        return int(lib.msp_workspace_bytes(self._ctx, C.byref(opts)))

    def plan(self, budget: int = 0, **kw) -> dict:
        """msp_plan: the plan msp_solve would run (host only, no GPU)."""
        opts = msp_default_opts(**kw)
        opts.workspace_bytes = budget
        out = msp_plan_t()
        _check(lib.msp_plan(self._ctx, C.byref(opts), C.byref(out)), "msp_plan")
        return {k: getattr(out, k) for k, _ in msp_plan_t._fields_}

    def solve(self, use_torch: bool = True, budget: Optional[int] = None, **kw) -> "Context":
        """msp_solve.  With torch and a GPU, the workspace is a torch tensor
        and the work runs on torch's current stream."""
        opts = msp_default_opts(**kw)
        if use_torch and torch is not None:
            if torch.cuda.is_available():
                if budget is None:
                    free, _ = torch.cuda.mem_get_info()
                    budget = min(int(free * 0.6), 64 << 30)
                opts.workspace_bytes = budget
                need = self.workspace_bytes(opts)
                if need == 0:
                    raise MspError(-5, "msp_workspace_bytes")
                if self._ws is None or self._ws.numel() < need:
                    self._ws = None
                    self._ws = torch.empty(need, dtype=torch.uint8, device="cuda")
                opts.workspace = self._ws.data_ptr()
                opts.workspace_bytes = self._ws.numel()
                opts.stream = torch.cuda.current_stream().cuda_stream
        elif budget is not None:
            opts.workspace_bytes = budget
        _check(lib.msp_solve(self._ctx, C.byref(opts)), "msp_solve")
        return self

    def solve_noalloc(self, **kw) -> "Context":
        """msp_solve_noalloc: the library's fixed scratch array as workspace;
        no device allocation (stream: kw ``stream`` or the null stream)."""
        opts = msp_default_opts(**kw)
        _check(lib.msp_solve_noalloc(self._ctx, C.byref(opts)), "msp_solve_noalloc")
        return self

    def hits(self) -> int:
        lo, hi = C.c_uint64(), C.c_uint64()
        _check(lib.msp_hits(self._ctx, C.byref(lo), C.byref(hi)), "msp_hits")
        return (hi.value << 64) | lo.value

    def num_solutions(self) -> int:
        c = C.c_uint64()
        _check(lib.msp_num_solutions(self._ctx, C.byref(c)), "msp_num_solutions")
        return c.value

    def solutions(self) -> np.ndarray:
        cnt = self.num_solutions()
        buf = np.zeros(max(cnt, 1) * self.n, dtype=np.uint8)
        w = C.c_uint64()
        rc = lib.msp_get_solutions(self._ctx, buf.ctypes.data_as(_p(C.c_uint8)), cnt, C.byref(w))
        if rc not in (MSP_OK, MSP_E_TRUNCATED):
            _check(rc, "msp_get_solutions")
        return buf[: w.value * self.n].reshape(w.value, self.n).copy()

    def stats(self) -> dict:
        s = msp_stats_t()
        _check(lib.msp_stats(self._ctx, C.byref(s)), "msp_stats")
        return {k: getattr(s, k) for k, _ in msp_stats_t._fields_}

    def result(self) -> Result:
        return Result(self.hits(), self.num_solutions(), self.solutions(), self.stats())


def solve(A, d, **kw) -> Result:
    """One-shot: msp_create, msp_solve, read results, msp_destroy."""
    ctx = Context(A, d)
    try:
        ctx.solve(**kw)
        return ctx.result()
    finally:
        ctx.close()


def batch_solve(contexts, opts=None, hbm_budget: int = 0, max_slots: int = 0) -> int:
    """msp_batch_solve over Context objects; opts is None, one dict for all,
    or a list of dicts (msp_opts fields).  Returns the status code; each
    context holds its own result (or raises on read if it failed)."""
    n = len(contexts)
    arr = (C.c_void_p * max(n, 1))(*[c._ctx.value for c in contexts])
    if opts is None:
        oarr = None
    else:
        lst = opts if isinstance(opts, (list, tuple)) else [opts] * n
        oarr = (msp_opts * max(n, 1))(*[msp_default_opts(**o) for o in lst])
    bo = msp_batch_opts(hbm_budget, max_slots, 0)
    return lib.msp_batch_solve(arr, oarr, n, C.byref(bo))


class Server:
    """msp_server_*: a continuous-batching request loop on its own thread."""

    def __init__(self, hbm_budget: int = 0, max_slots: int = 0):
        self._s = C.c_void_p()
        bo = msp_batch_opts(hbm_budget, max_slots, 0)
        _check(lib.msp_server_start(C.byref(bo), C.byref(self._s)), "msp_server_start")
        self._keep = {}

    def submit(self, ctx: Context, **kw) -> int:
        t = C.c_uint64()
        _check(lib.msp_server_submit(self._s, ctx._ctx, C.byref(msp_default_opts(**kw)),
                                     C.byref(t)), "msp_server_submit")
        self._keep[t.value] = ctx
        return t.value

    def poll(self, ticket: int):
        done, st = C.c_int32(), C.c_int32()
        _check(lib.msp_server_poll(self._s, ticket, C.byref(done), C.byref(st)), "msp_server_poll")
        return bool(done.value), st.value

    def wait(self, ticket: int) -> int:
        st = C.c_int32()
        _check(lib.msp_server_wait(self._s, ticket, C.byref(st)), "msp_server_wait")
        return st.value

    def cancel(self, ticket: int):
        _check(lib.msp_server_cancel(self._s, ticket), "msp_server_cancel")

    def times(self, ticket: int):
        t4 = (C.c_double * 4)()
        _check(lib.msp_server_times(self._s, ticket, t4), "msp_server_times")
        return tuple(t4)

    def stop(self):
        if self._s:
            _check(lib.msp_server_stop(self._s), "msp_server_stop")
            self._s = C.c_void_p()


_allocator_keep = None


def set_allocator(alloc=None, release=None):
    """msp_set_allocator.  ``alloc(bytes) -> device pointer (int) or 0`` and
    ``release(ptr)`` are Python callables; both None restores hipMalloc."""
    global _allocator_keep
    if alloc is None and release is None:
        rc = lib.msp_set_allocator(ALLOC_FN(), RELEASE_FN(), None)
        _check(rc, "msp_set_allocator")
        _allocator_keep = None
        return
    a = ALLOC_FN(lambda nbytes, user: alloc(int(nbytes)) or None)
    r = RELEASE_FN(lambda ptr, user: release(int(ptr)))
    _check(lib.msp_set_allocator(a, r, None), "msp_set_allocator")
    _allocator_keep = (a, r, alloc, release)


class TorchArena:
    """Device memory for the library from PyTorch's caching allocator: each
    request is a torch.uint8 CUDA tensor kept alive until the library
    releases it.  Use as ``with TorchArena(): ...``."""

    def __init__(self):
        self.live = {}
        self.requests = 0

    def alloc(self, nbytes: int) -> int:
        try:
            t = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        except RuntimeError:
            return 0
        self.live[t.data_ptr()] = t
        self.requests += 1
        return t.data_ptr()

    def release(self, ptr: int):
        self.live.pop(ptr, None)

    def __enter__(self):
        set_allocator(self.alloc, self.release)
        return self

    def __exit__(self, *exc):
        set_allocator(None, None)
        return False
