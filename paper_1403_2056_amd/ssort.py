"""Thin ctypes binding of libssort.so (argument marshalling only).

Every step of the sort runs in the HIP kernels of libssort.so; PyTorch only
provides device memory and the current stream.  There is no fallback: if the
library or a GPU is missing, calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libssort.so")

SSORT_TO_END = 1
SSORT_VALIDATE = 1
SSORT_EQUAL = 2
SSORT_ALPHABET = 4

STATUS = {
    0: "SSORT_OK", 1: "SSORT_EINVAL", 2: "SSORT_ENOMEM", 3: "SSORT_EWORKSPACE", 4: "SSORT_EBOUNDS",
    5: "SSORT_EZEROBYTE", 6: "SSORT_EDEVICE", 7: "SSORT_EBUSY", 8: "SSORT_ETIMEOUT", 9: "SSORT_ENOTFOUND",
}


STATUS_CODES = {name: code for code, name in STATUS.items()}


class SsortError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        super().__init__(f"{what}: {STATUS.get(code, code)}")


class Strings(ctypes.Structure):
    _fields_ = [("chars", ctypes.c_void_p), ("nchars", ctypes.c_uint64), ("offsets", ctypes.c_void_p),
                ("lengths", ctypes.c_void_p), ("n", ctypes.c_uint32), ("flags", ctypes.c_uint32)]


class Tuning(ctypes.Structure):
    _fields_ = [("v", ctypes.c_uint32), ("keys_per_thread", ctypes.c_uint32),
                ("base_threshold", ctypes.c_uint32), ("flags", ctypes.c_uint32)]

    def as_dict(self):
        return {"v": self.v, "keys_per_thread": self.keys_per_thread,
                "base_threshold": self.base_threshold, "flags": self.flags}


class Stats(ctypes.Structure):
    _fields_ = [("segments", ctypes.c_uint64), ("strings", ctypes.c_uint64),
                ("base_groups", ctypes.c_uint64), ("max_depth", ctypes.c_uint64),
                ("phase_ticks", ctypes.c_uint64 * 16),
                ("base_chunks", ctypes.c_uint64), ("base_rounds", ctypes.c_uint64),
                ("max_task", ctypes.c_uint64), ("max_chunk", ctypes.c_uint64),
                ("published_chunks", ctypes.c_uint64), ("error_bits", ctypes.c_uint64)]


PHASES = ["wait", "sample", "classify", "scatter", "children", "base", "extend", "other",
          "base_extend", "base_keys", "base_rank", "drain", "base_split"]


class Job(ctypes.Structure):
    _fields_ = [("chars", ctypes.c_void_p), ("nchars", ctypes.c_uint64), ("offsets", ctypes.c_void_p),
                ("n", ctypes.c_uint32), ("flags", ctypes.c_uint32), ("out_perm", ctypes.c_void_p),
                ("out_lcp", ctypes.c_void_p)]


class Result(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("status", ctypes.c_int), ("latency_ms", ctypes.c_double),
                ("queue_ms", ctypes.c_double), ("device_error", ctypes.c_uint64)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("stage_bytes", ctypes.c_size_t), ("max_jobs_per_launch", ctypes.c_uint32),
                ("max_strings_per_launch", ctypes.c_uint64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("launches", ctypes.c_uint64),
                ("jobs_launched", ctypes.c_uint64), ("max_jobs_per_launch", ctypes.c_uint64),
                ("arena_used", ctypes.c_uint64), ("waiting", ctypes.c_uint64)]


_lib = None

# every entry point declared in include/ssort.h, with its ctypes signature
_SIGS = {
    "ssort_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "ssort_destroy": (None, [ctypes.c_void_p]),
    "ssort_get_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Tuning)]),
    "ssort_workspace_bytes": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                             ctypes.POINTER(ctypes.c_size_t)]),
    "ssort_sort": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Strings), ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "ssort_merge_workspace_bytes": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32), ctypes.c_uint32,
                                                   ctypes.POINTER(ctypes.c_size_t)]),
    "ssort_merge": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Strings), ctypes.POINTER(ctypes.c_uint32),
                                   ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "ssort_sort_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Strings), ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p]),
    "ssort_sort_batched": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Strings), ctypes.c_void_p,
                                          ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_size_t, ctypes.c_void_p]),
    "ssort_query_error": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "ssort_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Stats), ctypes.c_void_p]),
    "ssort_set_wait_limit": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32]),
    "ssort_device_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)]),
    "ssort_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "ssort_profile": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "ssort_phase_ms": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_float)]),
    "ssort_graph_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Strings), ctypes.c_void_p,
                                          ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_size_t, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "ssort_graph_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "ssort_graph_destroy": (None, [ctypes.c_void_p]),
    "ssort_server_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_size_t, ctypes.c_uint32, ctypes.c_void_p,
                                           ctypes.POINTER(ServerConfig), ctypes.POINTER(ctypes.c_void_p)]),
    "ssort_server_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Job), ctypes.POINTER(ctypes.c_uint64)]),
    "ssort_server_wait": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(Result)]),
    "ssort_server_cancel": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "ssort_server_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ServerStats)]),
    "ssort_server_destroy": (None, [ctypes.c_void_p]),
    "ssort_debug_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Strings), ctypes.c_uint32,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "ssort_debug_segment_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Strings), ctypes.c_uint32]
                                 + [ctypes.c_void_p] * 9 + [ctypes.c_size_t, ctypes.c_void_p]),
}


def lib():
    """Load libssort.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != 0:
        raise SsortError(rc, what)


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def strings_to_device(ss, device="cuda"):
    """Copy a host string set (workloads.StringSet-like) to device tensors."""
    import torch
    chars = torch.from_numpy(np.ascontiguousarray(ss.chars) if len(ss.chars) else np.zeros(1, np.uint8))
    off = torch.from_numpy(np.ascontiguousarray(ss.offsets).view(np.int64) if len(ss.offsets)
                           else np.zeros(1, np.int64))
    ln = None
    if ss.lengths is not None:
        ln = torch.from_numpy(np.ascontiguousarray(ss.lengths).view(np.int32)).to(device)
    return DeviceStrings(chars.to(device), len(ss.chars), off.to(device), ln, ss.n, ss.flags)


class DeviceStrings:
    """Device-resident string set: chars (uint8), offsets (int64 viewed as
    uint64), optional lengths (int32 viewed as uint32), n, flags."""

    def __init__(self, chars, nchars, offsets, lengths, n, flags):
        self.chars, self.nchars, self.offsets, self.lengths = chars, int(nchars), offsets, lengths
        self.n, self.flags = int(n), int(flags)

    def struct(self) -> Strings:
        return Strings(_ptr(self.chars), self.nchars, _ptr(self.offsets), _ptr(self.lengths), self.n, self.flags)


class Sorter:
    """One library context on one GPU plus a workspace it grows on demand."""

    def __init__(self, device: int = 0, v: int = 255, keys_per_thread: int = 4, base_threshold: int = 128,
                 flags: int = 0):
        import torch
        self.device = device
        self.tuning = Tuning(v, keys_per_thread, base_threshold, flags)
        h = ctypes.c_void_p()
        _check(lib().ssort_create(device, ctypes.byref(self.tuning), ctypes.byref(h)), "ssort_create")
        self._h = h
        self._ws = None
        self._mws = None
        self._torch = torch

    def _retire(self, t):
        """Drop a workspace being replaced only after the device has finished
        with it (a sort or merge enqueued earlier may still use it)."""
        if t is not None:
            self._torch.cuda.synchronize(t.device)

    def _used_on(self, t, stream):
        """A buffer the library uses on a stream other than the current one:
        tell the caching allocator, so that it does not hand the memory to a
        new tensor of the current stream while that work runs."""
        if stream is not None and t is not None and stream != self._torch.cuda.current_stream(t.device):
            t.record_stream(stream)

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.ssort_destroy(self._h)
            self._h = None

    def set_wait_limit(self, ms: int):
        _check(lib().ssort_set_wait_limit(self._h, ms), "ssort_set_wait_limit")

    def profile(self, enable: bool = True):
        _check(lib().ssort_profile(self._h, 1 if enable else 0), "ssort_profile")

    def phase_ms(self) -> dict:
        a = (ctypes.c_float * 4)()
        _check(lib().ssort_phase_ms(self._h, a), "ssort_phase_ms")
        return {"root": a[0], "worker": a[1], "seam": a[2], "total": a[3]}

    def device_info(self) -> dict:
        a = (ctypes.c_uint64 * 4)()
        _check(lib().ssort_device_info(self._h, a), "ssort_device_info")
        return {"cus": a[0], "worker_blocks": a[1], "wall_khz": a[2], "device": a[3]}

    def workspace_bytes(self, n: int, m: int = 1) -> int:
        b = ctypes.c_size_t()
        _check(lib().ssort_workspace_bytes(self._h, n, m, ctypes.byref(b)), "ssort_workspace_bytes")
        return b.value

    def workspace(self, n: int, m: int = 1):
        need = self.workspace_bytes(n, m)
        if self._ws is None or self._ws.numel() < need:
            self._retire(self._ws)
            self._ws = self._torch.empty(need, dtype=self._torch.uint8, device=f"cuda:{self.device}")
        return self._ws

    def sort(self, s: DeviceStrings, with_lcp: bool = True, out_perm=None, out_lcp=None, ws=None, stream=None):
        """Enqueue a sort; returns (perm, lcp) int32 tensors holding uint32 values."""
        torch = self._torch
        dev = f"cuda:{self.device}"
        n = s.n
        if out_perm is None:
            out_perm = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        if with_lcp and out_lcp is None:
            out_lcp = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        if ws is None:
            ws = self.workspace(n)
        for t in (ws, out_perm, out_lcp):
            self._used_on(t, stream)
        st = s.struct()
        _check(lib().ssort_sort(self._h, ctypes.byref(st), _ptr(out_perm), _ptr(out_lcp) if with_lcp else None,
                                _ptr(ws), ws.numel(), _stream(stream)), "ssort_sort")
        return out_perm[:n], (out_lcp[:n] if with_lcp else None)

    def sort_noalloc(self, s: DeviceStrings, out_perm, out_lcp=None, stream=None):
        """Enqueue a sort that uses the library's own per-GPU scratch array as
        its workspace (ssort_sort_noalloc: the call allocates nothing; the
        caller passes the output tensors)."""
        for t in (out_perm, out_lcp):
            self._used_on(t, stream)
        st = s.struct()
        _check(lib().ssort_sort_noalloc(self._h, ctypes.byref(st), _ptr(out_perm), _ptr(out_lcp), _stream(stream)),
               "ssort_sort_noalloc")
        return out_perm[: s.n], (out_lcp[: s.n] if out_lcp is not None else None)

    def sort_batched(self, s: DeviceStrings, set_begin, with_lcp: bool = True, out_perm=None, out_lcp=None,
                     ws=None, stream=None):
        torch = self._torch
        dev = f"cuda:{self.device}"
        n = s.n
        m = set_begin.numel() - 1
        if out_perm is None:
            out_perm = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        if with_lcp and out_lcp is None:
            out_lcp = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        if ws is None:
            ws = self.workspace(n, m)
        for t in (ws, out_perm, out_lcp):
            self._used_on(t, stream)
        st = s.struct()
        _check(lib().ssort_sort_batched(self._h, ctypes.byref(st), _ptr(set_begin), m, _ptr(out_perm),
                                        _ptr(out_lcp) if with_lcp else None, _ptr(ws), ws.numel(),
                                        _stream(stream)), "ssort_sort_batched")
        return out_perm[:n], (out_lcp[:n] if with_lcp else None)

    def merge(self, s: DeviceStrings, run_begin, perm_in, lcp_in, with_lcp: bool = True, out_perm=None,
              out_lcp=None, ws=None, stream=None):
        """K-way LCP-merge of sorted runs: run_begin is a host sequence of K+1
        positions into perm_in/lcp_in (device int32 tensors)."""
        torch = self._torch
        dev = f"cuda:{self.device}"
        K = len(run_begin) - 1
        rb = (ctypes.c_uint32 * (K + 1))(*[int(x) for x in run_begin])
        n = int(run_begin[-1])
        if out_perm is None:
            out_perm = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        if with_lcp and out_lcp is None:
            out_lcp = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        for t in (out_perm, out_lcp):
            self._used_on(t, stream)
        if ws is None:
            # kept on the Sorter until a larger one is needed: the library's
            # error word and statistics live in it after the call returns
            b = ctypes.c_size_t()
            _check(lib().ssort_merge_workspace_bytes(self._h, rb, K, ctypes.byref(b)), "ssort_merge_workspace_bytes")
            if self._mws is None or self._mws.numel() < b.value:
                self._retire(self._mws)
                self._mws = torch.empty(max(b.value, 1), dtype=torch.uint8, device=dev)
            ws = self._mws
        self._used_on(ws, stream)
        st = s.struct()
        _check(lib().ssort_merge(self._h, ctypes.byref(st), rb, K, _ptr(perm_in), _ptr(lcp_in), _ptr(out_perm),
                                 _ptr(out_lcp) if with_lcp else None, _ptr(ws), ws.numel(), _stream(stream)),
               "ssort_merge")
        return out_perm[:n], (out_lcp[:n] if with_lcp else None)

    def query_error(self, stream=None) -> int:
        return lib().ssort_query_error(self._h, _stream(stream))

    def stats(self, stream=None) -> dict:
        st = Stats()
        _check(lib().ssort_stats(self._h, ctypes.byref(st), _stream(stream)), "ssort_stats")
        return {"segments": st.segments, "strings": st.strings, "base_groups": st.base_groups,
                "max_depth": st.max_depth, "base_chunks": st.base_chunks, "base_rounds": st.base_rounds,
                "published_chunks": st.published_chunks, "error_bits": st.error_bits,
                "max_task": {"ticks": st.max_task >> 24, "strings": st.max_task & 0xFFFFFF},
                "max_chunk": {"ticks": st.max_chunk >> 24, "rounds": (st.max_chunk >> 12) & 0xFFF,
                              "strings": st.max_chunk & 0xFFF},
                "phase_ticks": dict(zip(PHASES, list(st.phase_ticks)))}

    def debug_step(self, s: DeviceStrings, depth: int = 0, stream=None) -> dict:
        torch = self._torch
        dev = f"cuda:{self.device}"
        n = s.n
        keys = torch.empty(n, dtype=torch.int64, device=dev)
        split = torch.empty(4096, dtype=torch.int64, device=dev)
        tree = torch.empty(4096, dtype=torch.int64, device=dev)
        jump = torch.zeros(4096, dtype=torch.int16, device=dev)
        info = torch.empty(4, dtype=torch.int32, device=dev)
        bucket = torch.empty(n, dtype=torch.int16, device=dev)
        hist = torch.empty(8192, dtype=torch.int32, device=dev)
        perm = torch.empty(n, dtype=torch.int32, device=dev)
        ws = self.workspace(n)
        st = s.struct()
        _check(lib().ssort_debug_step(self._h, ctypes.byref(st), depth, _ptr(keys), _ptr(split), _ptr(tree),
                                      _ptr(jump), _ptr(info), _ptr(bucket), _ptr(hist), _ptr(perm), _ptr(ws),
                                      ws.numel(), _stream(stream)), "ssort_debug_step")
        torch.cuda.synchronize()
        out = {"keys": keys.cpu().numpy().view(np.uint64), "split": split.cpu().numpy().view(np.uint64),
               "tree": tree.cpu().numpy().view(np.uint64), "info": info.cpu().numpy().view(np.uint32),
               "bucket": bucket.cpu().numpy().view(np.uint16), "hist": hist.cpu().numpy().view(np.uint32),
               "perm": perm.cpu().numpy().view(np.uint32), "jump": jump.cpu().numpy().view(np.uint16)}
        v = int(out["info"][0])
        out["split"] = out["split"][:v]
        out["tree"] = out["tree"][:v]
        out["hist"] = out["hist"][:2 * v + 1]
        return out


    def debug_segment_step(self, s: DeviceStrings, depth: int = 0, stream=None) -> dict:
        """One persistent-worker segment step on the whole input: splitters,
        splitter LCPs, end flags, classification depth, per-bucket start, size
        and child depth, and the redistributed permutation (host arrays)."""
        torch = self._torch
        dev = f"cuda:{self.device}"
        n = s.n
        u32 = dict(dtype=torch.int32, device=dev)
        split = torch.empty(256, dtype=torch.int64, device=dev)
        info = torch.empty(4, **u32)
        hl = torch.empty(256, **u32)
        zr = torch.empty(256, **u32)
        bst = torch.empty(512, **u32)
        bsz = torch.empty(512, **u32)
        bdep = torch.empty(512, **u32)
        perm = torch.empty(n, **u32)
        ws = self.workspace(n)
        st = s.struct()
        _check(lib().ssort_debug_segment_step(self._h, ctypes.byref(st), depth, _ptr(split), _ptr(info), _ptr(hl),
                                              _ptr(zr), _ptr(bst), _ptr(bsz), _ptr(bdep), _ptr(perm), _ptr(ws),
                                              ws.numel(), _stream(stream)), "ssort_debug_segment_step")
        torch.cuda.synchronize()
        info = info.cpu().numpy().view(np.uint32)
        v = int(info[0])
        nb = 2 * v + 1
        return {"split": split.cpu().numpy().view(np.uint64)[:v], "info": info,
                "hl": hl.cpu().numpy().view(np.uint32)[: v + 1], "zr": zr.cpu().numpy().view(np.uint32)[:v],
                "start": bst.cpu().numpy().view(np.uint32)[:nb], "size": bsz.cpu().numpy().view(np.uint32)[:nb],
                "depth": bdep.cpu().numpy().view(np.uint32)[:nb], "perm": perm.cpu().numpy().view(np.uint32)}


class Graph:
    """A captured sort (plain or batched) replayed with one graph launch."""

    def __init__(self, sorter, s: DeviceStrings, set_begin=None, with_lcp=True, stream=None):
        torch = sorter._torch
        dev = f"cuda:{sorter.device}"
        n = s.n
        m = 1 if set_begin is None else set_begin.numel() - 1
        self.perm = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        self.lcp = torch.empty(max(n, 1), dtype=torch.int32, device=dev) if with_lcp else None
        self.ws = torch.empty(sorter.workspace_bytes(n, m), dtype=torch.uint8, device=dev)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=dev)
        self._keep = (s, set_begin)
        st = s.struct()
        h = ctypes.c_void_p()
        with torch.cuda.stream(self.stream):
            _check(lib().ssort_graph_create(sorter._h, ctypes.byref(st), _ptr(set_begin), m, _ptr(self.perm),
                                            _ptr(self.lcp), _ptr(self.ws), self.ws.numel(),
                                            ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
                   "ssort_graph_create")
        self._h = h
        self.n = n

    def launch(self):
        _check(lib().ssort_graph_launch(self._h, ctypes.c_void_p(self.stream.cuda_stream)), "ssort_graph_launch")

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.ssort_graph_destroy(self._h)
            self._h = None


class Server:
    """Request loop with continuous batching (host-side jobs)."""

    def __init__(self, device=0, budget_bytes=1 << 30, slots=4, v=255, keys_per_thread=4, base_threshold=128,
                 stage_bytes=0, max_jobs_per_launch=0, max_strings_per_launch=0):
        self.tuning = Tuning(v, keys_per_thread, base_threshold, 0)
        cfg = ServerConfig(stage_bytes, max_jobs_per_launch, max_strings_per_launch)
        h = ctypes.c_void_p()
        _check(lib().ssort_server_create(device, budget_bytes, slots, ctypes.byref(self.tuning),
                                         ctypes.byref(cfg), ctypes.byref(h)), "ssort_server_create")
        self._h = h
        self._jobs = {}

    def submit(self, ss, with_lcp=True) -> int:
        chars = np.ascontiguousarray(ss.chars, dtype=np.uint8)
        if chars.size == 0:
            chars = np.zeros(1, np.uint8)
        off = np.ascontiguousarray(ss.offsets, dtype=np.uint64)
        if ss.lengths is not None:
            raise ValueError("server jobs use CSR offsets or SSORT_TO_END starts")
        perm = np.empty(max(ss.n, 1), dtype=np.uint32)
        lcp = np.empty(max(ss.n, 1), dtype=np.uint32) if with_lcp else None
        job = Job(chars.ctypes.data, len(ss.chars), off.ctypes.data, ss.n, ss.flags, perm.ctypes.data,
                  lcp.ctypes.data if with_lcp else None)
        t = ctypes.c_uint64()
        _check(lib().ssort_server_submit(self._h, ctypes.byref(job), ctypes.byref(t)), "ssort_server_submit")
        self._jobs[t.value] = (chars, off, perm, lcp, ss.n)
        return t.value

    def wait(self, ticket: int, timeout_ms: int = -1):
        r = Result()
        rc = lib().ssort_server_wait(self._h, ticket, timeout_ms, ctypes.byref(r))
        chars, off, perm, lcp, n = self._jobs.pop(ticket)
        _check(rc, f"ssort_server_wait (device error mask {r.device_error:#x})" if r.device_error
               else "ssort_server_wait")
        return perm[:n], (lcp[:n] if lcp is not None else None), {"latency_ms": r.latency_ms, "queue_ms": r.queue_ms}

    def cancel(self, ticket: int) -> bool:
        ok = lib().ssort_server_cancel(self._h, ticket) == 0
        if ok:
            self._jobs.pop(ticket, None)
        return ok

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().ssort_server_stats(self._h, ctypes.byref(st)), "ssort_server_stats")
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.ssort_server_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()


def to_numpy_u32(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)
