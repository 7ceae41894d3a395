"""ctypes wrapper of the C oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this module.  The GPU library never does.  It shares no code with
the GPU path; the two meet only at the seeded input generators.

Routines (each documented in ``msp_oracle.h``):

* ``brute``       -- the definition of S and H written out (2^n walk, n <= 30);
* ``dp_count``    -- textbook subset-sum counting DP (exact H for one row);
* ``dp_count2``   -- 2-D counting DP (H for two rows);
* ``ss_heap``     -- Schroeppel-Shamir with heaps, Algorithm 1, each equal-key
  group verified by the exact sort-and-search join of Algorithms 2-3;
* ``mitm``        -- meet in the middle one residue class of the left key at a
  time (summed over all classes it is the whole solve; a subset of classes
  gives a sampled slice).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "msp_oracle.c")

ERRORS = {-1: "invalid argument", -2: "row sum exceeds 65534",
          -3: "key overflows int64", -4: "problem too large for this routine",
          -5: "out of memory"}


class OracleError(RuntimeError):
    pass


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (it is plain C, no GPU code)."""
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC",
                               "-o", _LIB_PATH, _SRC])
    return _LIB_PATH


class _Res(C.Structure):
    _fields_ = [("h_lo", C.c_uint64), ("h_hi", C.c_uint64),
                ("nsol", C.c_uint64), ("stored", C.c_uint64)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = C.CDLL(_LIB_PATH)
        i32p = C.POINTER(C.c_int32)
        u8p = C.POINTER(C.c_uint8)
        u64p = C.POINTER(C.c_uint64)
        i64p = C.POINTER(C.c_int64)
        lib.orc_brute.argtypes = [i32p, i32p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int64,
                                  C.c_int64, u64p, u8p, C.c_uint64, C.POINTER(_Res)]
        lib.orc_dp_count_row.argtypes = [i32p, C.c_int, C.c_int64, u64p, u64p]
        lib.orc_dp_count_2rows.argtypes = [i32p, i32p, C.c_int, C.c_int64, C.c_int64, u64p]
        lib.orc_ss_heap.argtypes = [i32p, i32p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int64,
                                    C.c_int64, u8p, C.c_uint64, C.POINTER(_Res)]
        lib.orc_mitm_residues.argtypes = [i32p, i32p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                          C.c_int64, C.c_int64, C.c_int64, C.c_int64,
                                          u8p, C.c_uint64, C.POINTER(_Res)]
        lib.orc_key_setup.argtypes = [i32p, i32p, C.c_int, C.c_int, C.c_int, C.c_int, i64p, i64p,
                                      i64p, C.POINTER(C.c_int)]
        lib.orc_key_setup_wide.argtypes = [i32p, i32p, C.c_int, C.c_int, C.c_int, C.c_int, i64p,
                                           i64p, i64p, C.POINTER(C.c_int), C.POINTER(C.c_int)]
        for f in (lib.orc_brute, lib.orc_dp_count_row, lib.orc_dp_count_2rows,
                  lib.orc_ss_heap, lib.orc_mitm_residues, lib.orc_key_setup,
                  lib.orc_key_setup_wide):
            f.restype = C.c_int
        _lib = lib
    return _lib


@dataclass
class OracleResult:
    H: int                      # 1-D hits (exact, arbitrary precision)
    nsol: int                   # |S|
    solutions: np.ndarray       # (stored, n) uint8, canonical (lexicographic) order
    hr: Optional[np.ndarray] = None   # brute force only: H for r = 1..m

    def solution_set(self):
        return {bytes(r) for r in self.solutions}


def _ptr(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def _prep(A, d):
    A = np.ascontiguousarray(np.asarray(A, dtype=np.int32))
    d = np.ascontiguousarray(np.asarray(d, dtype=np.int32))
    if A.ndim != 2 or d.shape != (A.shape[0],):
        raise ValueError("A must be (m, n) and d (m,)")
    return A, d


def canonical(sol: np.ndarray) -> np.ndarray:
    """Lexicographic order on (x_1, ..., x_n) with 0 < 1."""
    if sol.shape[0] == 0:
        return sol
    keys = [sol[:, j] for j in range(sol.shape[1] - 1, -1, -1)]
    return sol[np.lexsort(keys)]


def _check(rc):
    if rc != 0:
        raise OracleError(ERRORS.get(rc, f"error {rc}"))


def _finish(res, buf, n, hr=None):
    stored = int(res.stored)
    sol = canonical(buf[:stored * n].reshape(stored, n).copy())
    return OracleResult((int(res.h_hi) << 64) | int(res.h_lo), int(res.nsol), sol, hr)


def brute(A, d, key_rows=1, slice_mod=0, slice_res=0, capacity=1 << 16,
          key_base=0) -> OracleResult:
    A, d = _prep(A, d)
    m, n = A.shape
    hr = np.zeros(m, dtype=np.uint64)
    buf = np.zeros(capacity * n, dtype=np.uint8)
    res = _Res()
    _check(_load().orc_brute(_ptr(A, C.c_int32), _ptr(d, C.c_int32), m, n, key_rows,
                             key_base, slice_mod, slice_res, _ptr(hr, C.c_uint64),
                             _ptr(buf, C.c_uint8), capacity, C.byref(res)))
    return _finish(res, buf, n, hr.astype(object))


def dp_count(a, target) -> int:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.int32))
    lo, hi = C.c_uint64(), C.c_uint64()
    _check(_load().orc_dp_count_row(_ptr(a, C.c_int32), a.size, int(target),
                                    C.byref(lo), C.byref(hi)))
    return (hi.value << 64) | lo.value


def dp_count2(a1, a2, t1, t2) -> int:
    a1 = np.ascontiguousarray(np.asarray(a1, dtype=np.int32))
    a2 = np.ascontiguousarray(np.asarray(a2, dtype=np.int32))
    out = C.c_uint64()
    _check(_load().orc_dp_count_2rows(_ptr(a1, C.c_int32), _ptr(a2, C.c_int32), a1.size,
                                      int(t1), int(t2), C.byref(out)))
    return out.value


def ss_heap(A, d, key_rows=1, slice_mod=0, slice_res=0, capacity=1 << 16,
            key_base=0) -> OracleResult:
    A, d = _prep(A, d)
    m, n = A.shape
    buf = np.zeros(capacity * n, dtype=np.uint8)
    res = _Res()
    _check(_load().orc_ss_heap(_ptr(A, C.c_int32), _ptr(d, C.c_int32), m, n, key_rows,
                               key_base, slice_mod, slice_res, _ptr(buf, C.c_uint8), capacity,
                               C.byref(res)))
    return _finish(res, buf, n)


def mitm(A, d, key_rows=1, log2_m=12, rho_lo=0, rho_hi=None, slice_mod=0, slice_res=0,
         capacity=1 << 16, key_base=0) -> OracleResult:
    A, d = _prep(A, d)
    m, n = A.shape
    if rho_hi is None:
        rho_hi = 1 << log2_m
    buf = np.zeros(capacity * n, dtype=np.uint8)
    res = _Res()
    _check(_load().orc_mitm_residues(_ptr(A, C.c_int32), _ptr(d, C.c_int32), m, n, key_rows,
                                     key_base, log2_m, rho_lo, rho_hi, slice_mod, slice_res,
                                     _ptr(buf, C.c_uint8), capacity, C.byref(res)))
    return _finish(res, buf, n)


def key_setup(A, d, key_rows=1, key_base=0):
    """(radix of row 1, K_d, per-column key weights, infeasible flag)."""
    A, d = _prep(A, d)
    m, n = A.shape
    base, kd = C.c_int64(), C.c_int64()
    w = np.zeros(n, dtype=np.int64)
    inf = C.c_int()
    _check(_load().orc_key_setup(_ptr(A, C.c_int32), _ptr(d, C.c_int32), m, n, key_rows,
                                 key_base, C.byref(base), C.byref(kd), _ptr(w, C.c_int64), C.byref(inf)))
    return base.value, kd.value, w, bool(inf.value)


def key_setup_wide(A, d, key_rows=1, key_base=0):
    """key_setup that also takes keys past int64: then (radix of row 1, K_d
    mod 2^64, weights mod 2^64, infeasible, True); the int64 values are the
    bit patterns of those residues."""
    A, d = _prep(A, d)
    m, n = A.shape
    base, kd = C.c_int64(), C.c_int64()
    w = np.zeros(n, dtype=np.int64)
    inf, wide = C.c_int(), C.c_int()
    _check(_load().orc_key_setup_wide(_ptr(A, C.c_int32), _ptr(d, C.c_int32), m, n, key_rows,
                                      key_base, C.byref(base), C.byref(kd), _ptr(w, C.c_int64),
                                      C.byref(inf), C.byref(wide)))
    return base.value, kd.value, w, bool(inf.value), bool(wide.value)


def left_key(A, d, x, key_rows=1, key_base=0) -> int:
    """k_L(x): the 1-D key of x restricted to the left half of the columns
    (modulo 2^64 when the key does not fit int64: exact for residues mod 2^k)."""
    _, _, w, _, wide = key_setup_wide(A, d, key_rows, key_base)
    n = len(w)
    hl = (n + 1) // 2
    k = int(sum(int(w[j]) for j in range(hl) if x[j]))
    return k % (1 << 64) if wide else k
