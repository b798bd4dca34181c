"""Benchmark: one step = one full sort (all rows of the hot path) of the
long-shared-prefix workload, n = 2^24 strings (4096 random prefixes of
length 10..60 plus a random suffix of length 5..80 over a 64-symbol alphabet,
20 % exact duplicates), inputs resident in HBM.

Prints one JSON line: strings/s over K timed sorts, the distinguishing-prefix
rate, the roofline of the dominant kernel (the persistent worker, timed with
HIP events on the sort's own stream) and the CPU oracle timed on the same
input on one host core.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E peak
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "worker_traffic_prefixes_n16M.json")


def source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1403_2056_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h")):
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def dist_bytes(lens_sorted: np.ndarray, lcp: np.ndarray) -> np.ndarray:
    """Distinguishing characters of each string in sorted order:
    min(|s|, 1 + max(lcp with left neighbour, lcp with right neighbour))."""
    h = lcp.astype(np.int64)
    left = h
    right = np.zeros_like(h)
    right[:-1] = h[1:]
    return np.minimum(lens_sorted.astype(np.int64), 1 + np.maximum(left, right))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n-log2", type=int, default=24)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--copy-probe-gib", type=float, default=0.0,
                    help="also run a device copy of this many GiB (counter scaling runs)")
    ap.add_argument("--v", type=int, default=255)
    ap.add_argument("--k", type=int, default=4)
    ap.add_argument("--tb", type=int, default=128)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import torch
    from paper_1403_2056_amd import ssort, workloads

    n = 1 << args.n_log2
    t0 = time.time()
    ss = workloads.prefixes(n) if n == 1 << 24 else workloads.by_name("prefixes", n)
    print(f"[bench] generated n={ss.n} N={len(ss.chars)} in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    d = ssort.strings_to_device(ss)
    sorter = ssort.Sorter(0, v=args.v, keys_per_thread=args.k, base_threshold=args.tb)
    sorter.profile(True)
    perm = torch.empty(n, dtype=torch.int32, device="cuda")
    lcp = torch.empty(n, dtype=torch.int32, device="cuda")
    ws = sorter.workspace(n)
    for _ in range(args.warmup):
        sorter.sort(d, out_perm=perm, out_lcp=lcp, ws=ws)
    torch.cuda.synchronize()
    if sorter.query_error() != 0:
        raise SystemExit("device error during warm-up")
    print("[bench] warm-up done", file=sys.stderr, flush=True)

    worker_ms, root_ms, seam_ms = [], [], []
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(args.steps):
        sorter.sort(d, out_perm=perm, out_lcp=lcp, ws=ws)
        ph = sorter.phase_ms()          # waits for this sort's last event
        worker_ms.append(ph["worker"])
        root_ms.append(ph["root"])
        seam_ms.append(ph["seam"])
    end.record()
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(end)
    if sorter.query_error() != 0:
        raise SystemExit("device error during timed sorts")
    st = sorter.stats()
    ms_per_step = total_ms / args.steps

    if args.copy_probe_gib > 0:
        nb = int(args.copy_probe_gib * (1 << 30))
        a = torch.empty(nb, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()

    p = perm.cpu().numpy().view(np.uint32)
    h = lcp.cpu().numpy().view(np.uint32)
    lens = ss.lens()
    dist = dist_bytes(lens[p], h)
    D = int(dist.sum())
    N = int(lens.sum())
    t_s = ms_per_step / 1000.0

    # dominant kernel: the persistent worker.  Algorithmic bytes per launch:
    # the distinguishing characters beyond the first 8 (the root step reads
    # those), 10 B of index traffic per string per classification step it runs
    # (4 B read, 4 B written, 2 B bucket number), and the 4 B + 4 B of
    # permutation and LCP output per string.
    w_ms = float(np.mean(worker_ms))
    b_worker = int(np.maximum(dist - 8, 0).sum()) + 10 * int(st["strings"]) + 8 * n
    achieved = b_worker / (w_ms / 1000.0) / 1e9
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        tf = json.load(open(TRAFFIC_FILE))
        if tf.get("source_hash") == source_hash():
            traffic = tf.get("bytes_per_launch")
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic,
                "kernel": "k_worker", "avg_launch_ms": round(w_ms, 4), "algorithmic_bytes": b_worker}

    cpu = None
    if not args.no_cpu:
        import oracle
        chk = oracle.check(ss, p, h)
        if chk != -1:
            raise SystemExit(f"GPU output fails the oracle's checker at position {chk}")
        t1 = time.perf_counter()
        oracle.sort(ss)
        tc = time.perf_counter() - t1
        cpu = {"value": round(n / tc, 1), "unit": "strings/s", "cores": 1, "kind": "oracle",
               "sample": f"the same {n}-string input, whole sort with LCP array, single thread",
               "seconds": round(tc, 3), "checked_gpu_output": True}

    out = {
        "metric": "strings/sec + distinguishing-prefix GB/s (frac of HBM peak); batched vs plain",
        "value": round(n / t_s, 1),
        "unit": "strings/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "long shared prefixes: n=2^24 strings, 4096 random prefixes (len 10-60) + "
                               "random suffix (len 5-80), 64-symbol alphabet, 20% exact duplicates, CSR u64 offsets",
                   "n": n, "N": N, "D": D, "D_over_N": round(D / N, 4),
                   "tuning": sorter.tuning.as_dict()},
        "d_gbps": round(D / t_s / 1e9, 3),
        "d_frac_of_hbm_peak": round(D / t_s / 1e9 / HBM_PEAK_GBS, 6),
        "phase_ms": {"root": round(float(np.mean(root_ms)), 4), "worker": round(w_ms, 4),
                     "seam": round(float(np.mean(seam_ms)), 4)},
        "device_stats": st,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
