"""Benchmark: one step = one full sort (all rows of the hot path) of the
long-shared-prefix workload, n = 2^24 strings (4096 random prefixes of
length 10..60 plus a random suffix of length 5..80 over a 64-symbol alphabet,
20 % exact duplicates), inputs resident in HBM.

Prints one JSON line: strings/s over K timed sorts, the distinguishing-prefix
rate, the roofline of the dominant kernel (the persistent worker, timed with
HIP events on the sort's own stream), the attainable rates of the sort's two
access patterns measured on the same GPU (a device copy, random 8-byte
gathers), and the CPU oracle timed on the same input on all host threads and
on one; by default also the batched and served forms.
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


WORKLOAD_TEXT = {
    "prefixes": "long shared prefixes: n=2^{n} strings, 4096 strings per random prefix (len 10-60) + "
                "random suffix (len 5-80), 64-symbol alphabet, 20% exact duplicates, CSR u64 offsets",
    "suffixes": "suffix sort: all 2^{n} suffixes of a DNA text of copied, 1%-mutated 2 KiB blocks (strings run to the text's end)",
    "plain": "2^{n} strings of uniform length 8-32 over a-z, 5% duplicates",
}


# the files that define the sort's kernels and their launches (the merge and
# the server are host code and kernels of their own, outside the profiled sort)
SORT_SOURCES = ("ssort_dev.h", "ssort_kernels.h", "ssort_kernels.hip", "ssort_wide.hip", "ssort_api.hip")


def source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1403_2056_amd", "csrc")
    for f in SORT_SOURCES:
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


def attainable_probes(torch, w_ms: float, traffic_file: dict | None) -> dict:
    """Measured ceilings on this GPU for the sort's two access patterns: a
    1 GiB device copy (sequential read and write) and random 8-byte gathers
    from a 1 GiB table (torch index_select of 2^26 random indices: each gather
    one line fill, plus the in-order index reads and word writes).  With the
    worker's counted fetch bytes (at the copy's scale, 128 bytes per random
    line fill), also the worker's line fills per second against the probe."""
    ev = lambda: torch.cuda.Event(enable_timing=True)
    nb = 1 << 30
    a = torch.empty(nb, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    s, e = ev(), ev()
    s.record()
    for _ in range(5):
        b.copy_(a)
    e.record()
    torch.cuda.synchronize()
    copy_gbps = 2 * nb * 5 / (s.elapsed_time(e) / 1e3) / 1e9
    del a, b
    m = 1 << 26
    table = torch.zeros(1 << 27, dtype=torch.int64, device="cuda")
    idx = torch.randint(0, 1 << 27, (m,), dtype=torch.int64, device="cuda")
    g = torch.index_select(table, 0, idx)
    s, e = ev(), ev()
    s.record()
    for _ in range(3):
        g = torch.index_select(table, 0, idx)
    e.record()
    torch.cuda.synchronize()
    gathers = 3 * m / (s.elapsed_time(e) / 1e3)
    del table, idx, g
    torch.cuda.empty_cache()
    out = {"copy_gbps": round(copy_gbps, 1), "copy_frac_of_hbm_peak": round(copy_gbps / HBM_PEAK_GBS, 4),
           "random_gathers_per_s": round(gathers, 1)}
    if traffic_file is not None:
        fills = traffic_file["fetch_bytes"] / 128.0
        rate = fills / (w_ms / 1000.0)
        out["worker_line_fills_per_launch"] = round(fills)
        out["worker_line_fills_per_s"] = round(rate, 1)
        out["worker_frac_of_gather_probe"] = round(rate / gathers, 4)
    return out


def bench_merge(args):
    """K-way LCP-merge: the long-prefix input split into K contiguous shards,
    each sorted by the GPU (untimed, as K independent sorters would deliver
    them), then merged; timed: the merge alone, and a full sort for scale."""
    import torch
    from paper_1403_2056_amd import ssort, workloads
    n = 1 << args.n_log2
    K = args.runs
    ss = workloads.by_name(args.workload, n)
    d = ssort.strings_to_device(ss)
    s = ssort.Sorter(0)
    bounds = [n * k // K for k in range(K + 1)]
    sb = torch.tensor(bounds, dtype=torch.int32, device="cuda")
    p, h = s.sort_batched(d, sb)
    off = torch.repeat_interleave(torch.tensor(bounds[:-1], dtype=torch.int32),
                                  torch.tensor(np.diff(bounds), dtype=torch.int64)).cuda()
    pin = (p + off).contiguous()
    hin = h.clone()
    perm = torch.empty(n, dtype=torch.int32, device="cuda")
    lcp = torch.empty(n, dtype=torch.int32, device="cuda")
    for _ in range(args.warmup):
        s.merge(d, bounds, pin, hin, out_perm=perm, out_lcp=lcp)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        s.merge(d, bounds, pin, hin, out_perm=perm, out_lcp=lcp)
    e1.record()
    torch.cuda.synchronize()
    if s.query_error() != 0:
        raise SystemExit("device error during merges")
    ms = e0.elapsed_time(e1) / args.steps
    p2, h2 = s.sort(d)
    torch.cuda.synchronize()
    same = bool(torch.equal(p2, perm) and torch.equal(h2, lcp))
    e0.record()
    for _ in range(args.steps):
        s.sort(d)
    e1.record()
    torch.cuda.synchronize()
    sort_ms = e0.elapsed_time(e1) / args.steps
    out = {"metric": "strings/sec merged (K-way LCP-merge of sorted runs with LCP arrays)",
           "value": round(n / (ms / 1000.0), 1), "unit": "strings/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "dtype": "u8",
           "data": "synthetic",
           "config": {"workload": WORKLOAD_TEXT.get(args.workload, args.workload).format(n=args.n_log2),
                      "runs": K, "run_split": "contiguous index ranges, each sorted by the GPU"},
           "full_sort_ms": round(sort_ms, 4), "identical_to_full_sort": same}
    print(json.dumps(out), flush=True)


def device_error_exit(sorter, stream, what):
    """Stop with the device error mask (which consistency check fired)."""
    rc = sorter.query_error(stream)
    if rc != 0:
        bits = sorter.stats(stream)["error_bits"]
        raise SystemExit(f"device error during {what}: status {rc}, error mask {bits:#x}")


BATCHED_FALLBACK_TUNING = {"v": 63, "keys_per_thread": 4, "base_threshold": 256}


def host_threads() -> int:
    """Host threads this process may use: its CPU affinity, capped by
    OMP_NUM_THREADS when that is set (the share of a shared host)."""
    t = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        t = min(t, int(env))
    return max(1, t)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def bench_batched(args, embedded: bool = False):
    """Batched form: 4096 independent sets (sizes 2^U(6,18), geometric lengths
    with mean 24, 95 printable bytes) sorted by one graph-captured launch,
    against the same sets sorted one at a time (one ssort_sort per set, each
    synchronised).  The tuning is the autotuner's cached choice for this
    workload (tuned here only with --retune, or when nothing is cached and the
    batched mode runs on its own).  Returns the result dict; exits non-zero
    when a checked set differs from the oracle or the graph's output differs
    from the one-at-a-time output."""
    import torch
    from paper_1403_2056_amd import autotune, ssort, workloads
    t0 = time.time()
    ss, sb = workloads.batched(m=args.sets, seed=5, hi=args.size_log2_max or 18)
    n = ss.n
    print(f"[bench] batched: {args.sets} sets, n={n}, N={len(ss.chars)} in {time.time() - t0:.1f}s",
          file=sys.stderr, flush=True)
    d = ssort.strings_to_device(ss)
    sbt = torch.from_numpy(sb.view(np.int32)).cuda()
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    tun = autotune.lookup(arch, "batched", n)
    table = None
    tuned_from = "cache"
    if tun is None and embedded and not args.retune:
        tun, tuned_from = dict(BATCHED_FALLBACK_TUNING), "fallback (nothing cached)"
    if tun is None or args.retune:
        tuned_from = "tuned now"
        # tune on the first quarter of the sets (same size distribution)
        q = args.sets // 4
        nq = int(sb[q])
        dq = ssort.DeviceStrings(d.chars, d.nchars, d.offsets[: nq + 1], None, nq, 0)
        sbq = sbt[: q + 1]

        def factory(c):
            s = ssort.Sorter(0, **c)
            g = ssort.Graph(s, dq, set_begin=sbq)

            def run():
                g.launch()
                g.stream.synchronize()
                device_error_exit(s, g.stream, f"autotune candidate {c}")
            run._keep = (s, g)
            return run
        tun, table = autotune.tune(factory, log=lambda m: print(m, file=sys.stderr, flush=True))
        autotune.store(arch, "batched", n, dict(tun))
    sorter = ssort.Sorter(0, **tun)
    g = ssort.Graph(sorter, d, set_begin=sbt)
    for _ in range(args.warmup):
        g.launch()
    g.stream.synchronize()
    device_error_exit(sorter, g.stream, "batched graph warm-up")
    t1 = time.perf_counter()
    for _ in range(args.steps):
        g.launch()
    g.stream.synchronize()
    t_graph = (time.perf_counter() - t1) / args.steps
    device_error_exit(sorter, g.stream, "batched graph")
    # one set at a time, each sort synchronised before the next
    plain = ssort.Sorter(0, **tun)
    perm1 = torch.empty(n, dtype=torch.int32, device="cuda")
    lcp1 = torch.empty(n, dtype=torch.int32, device="cuda")
    ws = plain.workspace(int(np.diff(sb.astype(np.int64)).max()))
    views = []
    for k in range(args.sets):
        a, b = int(sb[k]), int(sb[k + 1])
        views.append((ssort.DeviceStrings(d.chars, d.nchars, d.offsets[a: b + 1], None, b - a, 0), a, b))
    for v, a, b in views[: min(64, len(views))]:
        plain.sort(v, out_perm=perm1[a:b], out_lcp=lcp1[a:b], ws=ws)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for v, a, b in views:
        plain.sort(v, out_perm=perm1[a:b], out_lcp=lcp1[a:b], ws=ws)
        torch.cuda.synchronize()
    t_one = time.perf_counter() - t2
    device_error_exit(plain, None, "one-at-a-time sorts")
    same_perm = bool(torch.equal(g.perm[:n], perm1))
    same_lcp = bool(torch.equal(g.lcp[:n], lcp1))
    out = {"metric": "strings/sec batched (one graph launch) vs one-at-a-time", "value": round(n / t_graph, 1),
           "unit": "strings/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(t_graph * 1000, 3), "higher_is_better": True, "dtype": "u8", "data": "synthetic",
           "config": {"workload": f"batched: {args.sets} sets of 2^U(6,{args.size_log2_max or 18}) strings, geometric lengths mean 24, "
                                  "95 printable bytes", "n": n, "N": int(len(ss.chars)), "tuning": tun,
                      "tuning_from": tuned_from},
           "one_at_a_time_ms": round(t_one * 1000, 3), "one_at_a_time_strings_per_s": round(n / t_one, 1),
           "batched_vs_one_at_a_time": round(t_one / t_graph, 2),
           "identical_to_one_at_a_time": same_perm and same_lcp}
    if table:
        out["autotune"] = [{**c, "ms": round(ms, 3)} for c, ms in table]
    if not args.no_cpu:
        import oracle
        rng = np.random.default_rng(0)
        p = g.perm[:n].cpu().numpy().view(np.uint32)
        h = g.lcp[:n].cpu().numpy().view(np.uint32)
        strs = None
        bad = 0
        for k in rng.choice(args.sets, size=min(32, args.sets), replace=False):
            a, b = int(sb[k]), int(sb[k + 1])
            sub = workloads.StringSet(ss.chars, ss.offsets[a: b + 1].copy(), None, 0, b - a, {})
            rp, rh = oracle.sort(sub)
            bad += int(not (np.array_equal(p[a:b], rp) and np.array_equal(h[a:b], rh)))
        checked = min(32, args.sets)
        out["oracle_checked_sets"] = checked - bad
        out["oracle_mismatching_sets"] = bad
        if bad:
            print(json.dumps(out), flush=True)
            raise SystemExit(f"batched output differs from the oracle in {bad} of {checked} checked sets")
        if embedded:
            return out
        t3 = time.perf_counter()
        done = 0
        for k in range(args.sets):
            a, b = int(sb[k]), int(sb[k + 1])
            oracle.sort(workloads.StringSet(ss.chars, ss.offsets[a: b + 1].copy(), None, 0, b - a, {}))
            done += b - a
            if time.perf_counter() - t3 > 20:
                break
        tc = time.perf_counter() - t3
        out["cpu_baseline"] = {"value": round(done / tc, 1), "unit": "strings/s", "cores": 1, "kind": "oracle",
                               "sample": f"the first {done} strings of the batch, set by set"}
    if not (same_perm and same_lcp):
        print(json.dumps(out), flush=True)
        raise SystemExit("the graph-launched batch differs from the one-at-a-time sorts")
    if embedded:
        return out
    print(json.dumps(out), flush=True)
    return out


def bench_serve(args, embedded: bool = False):
    """Serving form: a Poisson stream of jobs (sizes 2^U(4,20) strings, each
    drawn from the plain / long-prefix / suffix generators), admitted by a
    64 GB resident-memory budget with continuous batching, against the same
    jobs one at a time (one slot, one job per launch)."""
    from paper_1403_2056_amd import ssort, workloads
    rng = np.random.default_rng(7)
    jobs = []
    t0 = time.time()
    for _ in range(args.jobs):
        nj = int(np.floor(2.0 ** rng.uniform(4, args.size_log2_max or 20)))
        jobs.append(workloads.mixed_job(rng, nj))
    ntot = sum(j.n for j in jobs)
    print(f"[bench] serve: {args.jobs} jobs, {ntot} strings, generated in {time.time() - t0:.1f}s",
          file=sys.stderr, flush=True)

    def run(slots, max_jobs, rate):
        # a launch holds at most 2^22 strings (every job here has at most
        # 2^20), so the four slots pipeline copies, sorts and copies back
        srv = ssort.Server(0, budget_bytes=args.budget_gb << 30, slots=slots, max_jobs_per_launch=max_jobs,
                           stage_bytes=512 << 20, max_strings_per_launch=1 << 22)
        for j in jobs[:8]:                     # warm-up
            srv.wait(srv.submit(j))
        lat = []
        t_start = time.perf_counter()
        tickets = []
        next_t = t_start
        for j in jobs:
            if rate:
                next_t += rng.exponential(1.0 / rate)
                while time.perf_counter() < next_t:
                    pass
            tickets.append(srv.submit(j))
        for t in tickets:
            _, _, info = srv.wait(t)
            lat.append(info["latency_ms"])
        el = time.perf_counter() - t_start
        st = srv.stats()
        srv.close()
        lat = np.array(lat)
        return {"seconds": round(el, 3), "jobs_per_s": round(len(jobs) / el, 1),
                "strings_per_s": round(ntot / el, 1), "p50_ms": round(float(np.percentile(lat, 50)), 3),
                "p99_ms": round(float(np.percentile(lat, 99)), 3), "launches": st["launches"],
                "max_jobs_per_launch": st["max_jobs_per_launch"]}
    one = run(1, 1, 0)                        # one job at a time, saturated
    mu1 = one["jobs_per_s"]
    sat = run(4, 4096, 4 * mu1)               # offered load 4x the one-at-a-time rate
    lat = run(4, 4096, 0.7 * mu1)             # offered load the one-at-a-time server sustains
    one_lat = run(1, 1, 0.7 * mu1)
    out = {"metric": "served jobs/s and p50/p99 latency, continuous batching vs one-job-at-a-time",
           "value": sat["jobs_per_s"], "unit": "jobs/s", "n_gpus": 1, "higher_is_better": True,
           "dtype": "u8", "data": "synthetic",
           "config": {"workload": f"{args.jobs} Poisson jobs, sizes 2^U(4,{args.size_log2_max or 20}), plain/long-prefix/suffix mix",
                      "strings": ntot, "budget_gb": args.budget_gb},
           "served_saturated": sat, "served_at_0.7x": lat, "one_at_a_time": one, "one_at_a_time_at_0.7x": one_lat,
           "throughput_vs_one_at_a_time": round(sat["jobs_per_s"] / mu1, 2)}
    if embedded:
        return out
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n-log2", type=int, default=24)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batched", action="store_true",
                    help="plain mode: skip the batched block (4096 sets, graph launch vs one at a time) "
                         "and the served block")
    ap.add_argument("--batched-steps", type=int, default=5, help="timed graph launches of the batched block")
    ap.add_argument("--no-served", action="store_true",
                    help="plain mode: skip the served block (Poisson jobs, continuous batching vs one at a time)")
    ap.add_argument("--no-probes", action="store_true",
                    help="plain mode: skip the attainable copy and gather rates")
    ap.add_argument("--copy-probe-gib", type=float, default=0.0,
                    help="also run a device copy of this many GiB (counter scaling runs)")
    ap.add_argument("--gather-probe-m", type=int, default=0,
                    help="also gather this many random 8-byte words from a 1 GiB table (counter scaling runs)")
    ap.add_argument("--v", type=int, default=255)
    ap.add_argument("--k", type=int, default=4)
    ap.add_argument("--tb", type=int, default=128)
    ap.add_argument("--equal", action="store_true", help="S5-Equal classification")
    ap.add_argument("--alphabet", action="store_true", help="alphabet compression (packed character codes)")
    ap.add_argument("--workload", default="prefixes", help="plain mode: prefixes, suffixes or plain")
    ap.add_argument("--mode", choices=["plain", "batched", "serve", "merge"], default="plain")
    ap.add_argument("--runs", type=int, default=8, help="merge mode: number of sorted runs K")
    ap.add_argument("--sets", type=int, default=4096)
    ap.add_argument("--size-log2-max", type=int, default=0,
                    help="batched/serve: largest set or job size exponent (default 18 / 20)")
    ap.add_argument("--retune", action="store_true")
    ap.add_argument("--jobs", type=int, default=1200)
    ap.add_argument("--budget-gb", type=int, default=64)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the sorter runs on one GPU; --gpus must be 1 (sharding is described in the design notes, not implemented)",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    if args.mode == "batched":
        return bench_batched(args)
    if args.mode == "serve":
        return bench_serve(args)
    if args.mode == "merge":
        return bench_merge(args)

    import torch
    from paper_1403_2056_amd import ssort, workloads

    n = 1 << args.n_log2
    t0 = time.time()
    ss = workloads.by_name(args.workload, n)
    print(f"[bench] generated n={ss.n} N={len(ss.chars)} in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    d = ssort.strings_to_device(ss)
    sorter = ssort.Sorter(0, v=args.v, keys_per_thread=args.k, base_threshold=args.tb,
                          flags=(ssort.SSORT_EQUAL if args.equal else 0) | (ssort.SSORT_ALPHABET if args.alphabet else 0))
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
        del a, b
    if args.gather_probe_m > 0:
        # random 8-byte reads of known count: index_select reads the indices
        # in order, one table word per index at random, writes the words in order
        table = torch.zeros(1 << 27, dtype=torch.int64, device="cuda")
        idx = torch.randint(0, 1 << 27, (args.gather_probe_m,), dtype=torch.int64, device="cuda")
        torch.cuda.synchronize()
        g = torch.index_select(table, 0, idx)
        torch.cuda.synchronize()
        del table, idx, g

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
    traffic, tf_now = None, None
    if os.path.exists(TRAFFIC_FILE):
        tf = json.load(open(TRAFFIC_FILE))
        if (tf.get("source_hash") == source_hash() and args.workload == "prefixes" and n == 1 << 24
                and sorter.tuning.as_dict() == tf.get("tuning", sorter.tuning.as_dict())):
            traffic, tf_now = tf.get("bytes_per_launch"), tf
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic,
                "kernel": "k_worker", "avg_launch_ms": round(w_ms, 4), "algorithmic_bytes": b_worker}
    if traffic is not None:
        roofline["traffic_over_algorithmic"] = round(traffic / b_worker, 2)
    probes = None if args.no_probes else attainable_probes(torch, w_ms, tf_now)

    cpu = None
    if not args.no_cpu:
        import oracle
        chk = oracle.check(ss, p, h)
        if chk != -1:
            raise SystemExit(f"GPU output fails the oracle's checker at position {chk}")
        # the oracle as it stands, on every host thread this process may use
        # (same multikey quicksort, subproblems above 2^16 strings on a shared
        # job queue), then on one thread
        T = host_threads()
        t1 = time.perf_counter()
        rp, rh = oracle.sort(ss, threads=T)
        tc = time.perf_counter() - t1
        same = bool(np.array_equal(rp, p) and np.array_equal(rh, h))
        del rp, rh
        t1 = time.perf_counter()
        oracle.sort(ss, threads=1)
        t1c = time.perf_counter() - t1
        cpu = {"value": round(n / tc, 1), "unit": "strings/s", "cores": T, "kind": "oracle",
               "sample": f"the same {n}-string input, whole sort with LCP array, {T} host threads",
               "seconds": round(tc, 3), "nproc": os.cpu_count(), "cpu_model": cpu_model(),
               "single_core": {"value": round(n / t1c, 1), "unit": "strings/s", "seconds": round(t1c, 3)},
               "checked_gpu_output": True, "identical_to_gpu_output": same}
        if not same:
            raise SystemExit("the oracle's sort differs from the GPU output")

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
        "config": {"workload": WORKLOAD_TEXT.get(args.workload, args.workload).format(n=args.n_log2),
                   "n": n, "N": N, "D": D, "D_over_N": round(D / N, 4),
                   "tuning": sorter.tuning.as_dict()},
        "d_gbps": round(D / t_s / 1e9, 3),
        "d_frac_of_hbm_peak": round(D / t_s / 1e9 / HBM_PEAK_GBS, 6),
        "phase_ms": {"root": round(float(np.mean(root_ms)), 4), "worker": round(w_ms, 4),
                     "seam": round(float(np.mean(seam_ms)), 4)},
        "device_stats": st,
        "roofline": roofline,
        "attainable": probes,
        "cpu_baseline": cpu,
    }
    if not args.no_batched:
        # the batched form (the metric's "batched vs plain"): 4096 sets at
        # full size, one graph launch against one set at a time
        del d, perm, lcp, ws, sorter
        torch.cuda.empty_cache()
        ba = argparse.Namespace(**vars(args))
        ba.sets, ba.size_log2_max, ba.steps, ba.warmup = 4096, 18, args.batched_steps, 2
        out["batched"] = bench_batched(ba, embedded=True)
    if not args.no_batched and not args.no_served:
        # the serving form: the same Poisson job stream served with
        # continuous batching and one job at a time
        torch.cuda.empty_cache()
        sa = argparse.Namespace(**vars(args))
        sa.jobs, sa.size_log2_max, sa.budget_gb = 1200, 20, 64
        sv = bench_serve(sa, embedded=True)
        out["served"] = {k: sv[k] for k in ("value", "unit", "config", "served_saturated", "served_at_0.7x",
                                           "one_at_a_time", "one_at_a_time_at_0.7x", "throughput_vs_one_at_a_time")}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
