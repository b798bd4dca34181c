"""CPU oracle (test infrastructure only).

Loads ``liboracle.so`` built from ``ssort_oracle.c`` with gcc.  Only the tests,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may use it;
the product path never does.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ssort_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

u8p = ctypes.POINTER(ctypes.c_uint8)
u32p = ctypes.POINTER(ctypes.c_uint32)
u64p = ctypes.POINTER(ctypes.c_uint64)


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        L.ssort_oracle_sort.restype = ctypes.c_int
        L.ssort_oracle_sort.argtypes = [u8p, ctypes.c_uint64, u64p, u32p, ctypes.c_uint32,
                                        ctypes.c_uint32, u32p, u32p]
        L.ssort_oracle_stats.restype = ctypes.c_int
        L.ssort_oracle_stats.argtypes = [u8p, ctypes.c_uint64, u64p, u32p, ctypes.c_uint32,
                                         ctypes.c_uint32, u32p, u32p, u64p]
        L.ssort_oracle_check.restype = ctypes.c_int64
        L.ssort_oracle_check.argtypes = [u8p, ctypes.c_uint64, u64p, u32p, ctypes.c_uint32,
                                         ctypes.c_uint32, u32p, u32p]
        L.ssort_oracle_keys.restype = None
        L.ssort_oracle_keys.argtypes = [u8p, ctypes.c_uint64, u64p, u32p, ctypes.c_uint32,
                                        ctypes.c_uint32, u32p, ctypes.c_uint64, u32p, u64p]
        L.ssort_oracle_classify.restype = None
        L.ssort_oracle_classify.argtypes = [u64p, ctypes.c_uint64, u64p, ctypes.c_uint32, u32p]
        L.ssort_oracle_tree_ranks.restype = None
        L.ssort_oracle_tree_ranks.argtypes = [ctypes.c_uint32, u32p]
        L.ssort_oracle_splitter_lcp.restype = None
        L.ssort_oracle_splitter_lcp.argtypes = [u64p, ctypes.c_uint32, u32p]
        _lib = L
    return _lib


def _p(a: np.ndarray | None, t):
    if a is None:
        return ctypes.cast(None, t)
    return a.ctypes.data_as(t)


def _args(ss):
    chars = np.ascontiguousarray(ss.chars, dtype=np.uint8)
    if chars.size == 0:
        chars = np.zeros(1, dtype=np.uint8)
    off = np.ascontiguousarray(ss.offsets, dtype=np.uint64)
    if off.size == 0:
        off = np.zeros(1, dtype=np.uint64)
    ln = None if ss.lengths is None else np.ascontiguousarray(ss.lengths, dtype=np.uint32)
    keep = (chars, off, ln)
    return keep, [_p(chars, u8p), ctypes.c_uint64(len(ss.chars)), _p(off, u64p), _p(ln, u32p),
                  ctypes.c_uint32(ss.n), ctypes.c_uint32(ss.flags)]


def sort(ss, with_lcp: bool = True):
    """(perm, lcp) as uint32 arrays; lcp is None when with_lcp is False."""
    keep, a = _args(ss)
    perm = np.empty(max(ss.n, 1), dtype=np.uint32)
    lcp = np.empty(max(ss.n, 1), dtype=np.uint32) if with_lcp else None
    rc = lib().ssort_oracle_sort(*a, _p(perm, u32p), _p(lcp, u32p))
    if rc != 0:
        raise ValueError(f"oracle rejected input (rc={rc})")
    del keep
    return perm[: ss.n], (lcp[: ss.n] if with_lcp else None)


def stats(ss, perm, lcp) -> dict:
    keep, a = _args(ss)
    perm = np.ascontiguousarray(perm, dtype=np.uint32)
    lcp = np.ascontiguousarray(lcp, dtype=np.uint32)
    out = np.zeros(5, dtype=np.uint64)
    rc = lib().ssort_oracle_stats(*a, _p(perm, u32p), _p(lcp, u32p), _p(out, u64p))
    if rc != 0:
        raise ValueError(f"oracle rejected input (rc={rc})")
    del keep
    D, Dp, L, N, Np = (int(x) for x in out)
    return {"D": D, "D_paper": Dp, "L": L, "N": N, "N_paper": Np}


def check(ss, perm, lcp) -> int:
    """-1 when (perm, lcp) is exactly the sorted order and LCP array, else the
    first failing position (n for a permutation failure)."""
    keep, a = _args(ss)
    perm = np.ascontiguousarray(perm, dtype=np.uint32)
    lcp = np.ascontiguousarray(lcp, dtype=np.uint32)
    if perm.size != ss.n or lcp.size != ss.n:
        return ss.n
    if ss.n == 0:
        return -1
    r = lib().ssort_oracle_check(*a, _p(perm, u32p), _p(lcp, u32p))
    del keep
    return int(r)


def keys(ss, idx, depth) -> np.ndarray:
    keep, a = _args(ss)
    idx = np.ascontiguousarray(idx, dtype=np.uint32)
    depth = np.ascontiguousarray(np.broadcast_to(depth, idx.shape), dtype=np.uint32)
    out = np.zeros(max(idx.size, 1), dtype=np.uint64)
    lib().ssort_oracle_keys(*a, _p(idx, u32p), ctypes.c_uint64(idx.size), _p(depth, u32p),
                            _p(out, u64p))
    del keep
    return out[: idx.size]


def classify(keys_: np.ndarray, splitters: np.ndarray) -> np.ndarray:
    k = np.ascontiguousarray(keys_, dtype=np.uint64)
    x = np.ascontiguousarray(splitters, dtype=np.uint64)
    out = np.zeros(max(k.size, 1), dtype=np.uint32)
    lib().ssort_oracle_classify(_p(k, u64p), ctypes.c_uint64(k.size), _p(x, u64p),
                                ctypes.c_uint32(x.size), _p(out, u32p))
    return out[: k.size]


def tree_ranks(v: int) -> np.ndarray:
    out = np.zeros(v, dtype=np.uint32)
    lib().ssort_oracle_tree_ranks(ctypes.c_uint32(v), _p(out, u32p))
    return out


def splitter_lcp(splitters: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(splitters, dtype=np.uint64)
    out = np.zeros(x.size + 1, dtype=np.uint32)
    lib().ssort_oracle_splitter_lcp(_p(x, u64p), ctypes.c_uint32(x.size), _p(out, u32p))
    return out
