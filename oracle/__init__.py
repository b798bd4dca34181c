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
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-pthread", "-shared", "-fPIC",
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
                                        ctypes.c_uint32, u32p, u32p, ctypes.c_int]
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
        L.ssort_oracle_lcp_insertion_sort.restype = ctypes.c_int
        L.ssort_oracle_lcp_insertion_sort.argtypes = [u8p, ctypes.c_uint64, u64p, u32p, ctypes.c_uint32,
                                                      ctypes.c_uint32, u32p, ctypes.c_uint32, ctypes.c_uint32,
                                                      u32p, u32p, u64p]
        L.ssort_oracle_lcp_merge.restype = ctypes.c_int
        L.ssort_oracle_lcp_merge.argtypes = [u8p, ctypes.c_uint64, u64p, u32p, ctypes.c_uint32, ctypes.c_uint32,
                                             u32p, ctypes.c_uint32, ctypes.c_int, u32p, u32p, u32p, u32p, u64p]
        L.ssort_oracle_lcp_mergesort.restype = ctypes.c_int
        L.ssort_oracle_lcp_mergesort.argtypes = [u8p, ctypes.c_uint64, u64p, u32p, ctypes.c_uint32,
                                                 ctypes.c_uint32, ctypes.c_uint32, u32p, u32p, u64p]
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


def sort(ss, with_lcp: bool = True, threads: int = 1):
    """(perm, lcp) as uint32 arrays; lcp is None when with_lcp is False.
    threads > 1 runs the same multikey quicksort on that many host threads
    (a shared job queue for subproblems above 2^16 strings); the result is
    the same."""
    keep, a = _args(ss)
    perm = np.empty(max(ss.n, 1), dtype=np.uint32)
    lcp = np.empty(max(ss.n, 1), dtype=np.uint32) if with_lcp else None
    rc = lib().ssort_oracle_sort(*a, _p(perm, u32p), _p(lcp, u32p), ctypes.c_int(threads))
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


def lcp_insertion_sort(ss, idx, hbar: int = 0):
    """Algorithm 5 on the strings idx (which share the prefix hbar): (perm,
    lcp, character comparisons)."""
    keep, a = _args(ss)
    idx = np.ascontiguousarray(idx, dtype=np.uint32)
    m = idx.size
    perm = np.zeros(max(m, 1), dtype=np.uint32)
    lcp = np.zeros(max(m, 1), dtype=np.uint32)
    cnt = np.zeros(1, dtype=np.uint64)
    rc = lib().ssort_oracle_lcp_insertion_sort(*a, _p(idx, u32p), ctypes.c_uint32(m), ctypes.c_uint32(hbar),
                                               _p(perm, u32p), _p(lcp, u32p), _p(cnt, u64p))
    if rc != 0:
        raise ValueError(f"oracle rejected input (rc={rc})")
    del keep
    return perm[:m], lcp[:m], int(cnt[0])


def lcp_merge(ss, run_begin, perm_in, lcp_in, binary: bool = False):
    """K-way LCP-merge (Algorithm 4; Algorithm 3 with binary and K = 2) of
    sorted runs: (perm, lcp, character comparisons)."""
    keep, a = _args(ss)
    rb = np.ascontiguousarray(run_begin, dtype=np.uint32)
    K = rb.size - 1
    pin = np.ascontiguousarray(perm_in, dtype=np.uint32)
    hin = np.ascontiguousarray(lcp_in, dtype=np.uint32)
    n = int(rb[-1])
    if pin.size == 0:
        pin = np.zeros(1, np.uint32)
        hin = np.zeros(1, np.uint32)
    perm = np.zeros(max(n, 1), dtype=np.uint32)
    lcp = np.zeros(max(n, 1), dtype=np.uint32)
    cnt = np.zeros(1, dtype=np.uint64)
    rc = lib().ssort_oracle_lcp_merge(*a, _p(rb, u32p), ctypes.c_uint32(K), ctypes.c_int(1 if binary else 0),
                                      _p(pin, u32p), _p(hin, u32p), _p(perm, u32p), _p(lcp, u32p), _p(cnt, u64p))
    if rc != 0:
        raise ValueError(f"oracle rejected input (rc={rc})")
    del keep
    return perm[:n], lcp[:n], int(cnt[0])


def lcp_mergesort(ss, K: int = 2):
    """LCP-mergesort (binary with K = 2, else K-way): (perm, lcp, character
    comparisons)."""
    keep, a = _args(ss)
    perm = np.zeros(max(ss.n, 1), dtype=np.uint32)
    lcp = np.zeros(max(ss.n, 1), dtype=np.uint32)
    cnt = np.zeros(1, dtype=np.uint64)
    rc = lib().ssort_oracle_lcp_mergesort(*a, ctypes.c_uint32(K), _p(perm, u32p), _p(lcp, u32p), _p(cnt, u64p))
    if rc != 0:
        raise ValueError(f"oracle rejected input (rc={rc})")
    del keep
    return perm[:ss.n], lcp[:ss.n], int(cnt[0])
