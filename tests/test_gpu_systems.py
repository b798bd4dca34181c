"""The two systems forms through the C ABI: graph-captured launches (plain and
batched) replayed several times with eager work between replays, and the
sort server (continuous batching): every result equals the oracle's, and
each job's result is the same alone and in a mix."""
import numpy as np
import pytest

import oracle
from paper_1403_2056_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ss_mod():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1403_2056_amd import ssort
    return ssort


def u32(t):
    return t.cpu().numpy().view(np.uint32)


def test_graph_plain_replays(ss_mod):
    ssort = ss_mod
    print("[systems] graph plain", flush=True)
    s = ssort.Sorter(0)
    s.set_wait_limit(10000)
    ss = W.plain(100000, seed=31)
    d = ssort.strings_to_device(ss)
    rp, rh = oracle.sort(ss)
    g = ssort.Graph(s, d)
    for rep in range(4):
        g.perm.fill_(-1)
        g.lcp.fill_(-1)
        torch.cuda.synchronize()
        g.launch()
        g.stream.synchronize()
        assert s.query_error(g.stream) == 0, s.stats(g.stream)
        assert np.array_equal(u32(g.perm)[:ss.n], rp), rep
        assert np.array_equal(u32(g.lcp)[:ss.n], rh), rep
        # eager work between replays
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()
        p, h = s.sort(d)
        torch.cuda.synchronize()
        assert np.array_equal(u32(p), rp)


def test_graph_batched_replays(ss_mod):
    ssort = ss_mod
    print("[systems] graph batched", flush=True)
    s = ssort.Sorter(0)
    s.set_wait_limit(10000)
    ss, sb = W.batched(m=96, seed=32, lo=2, hi=12)
    d = ssort.strings_to_device(ss)
    sbt = torch.from_numpy(sb.view(np.int32)).cuda()
    g = ssort.Graph(s, d, set_begin=sbt)
    strs = ss.strings()
    refs = []
    for k in range(len(sb) - 1):
        a, b = int(sb[k]), int(sb[k + 1])
        refs.append(oracle.sort(W.from_list(strs[a:b])))
    for rep in range(3):
        g.perm.fill_(-1)
        torch.cuda.synchronize()
        g.launch()
        g.stream.synchronize()
        assert s.query_error(g.stream) == 0, s.stats(g.stream)
        p, h = u32(g.perm), u32(g.lcp)
        for k, (rp, rh) in enumerate(refs):
            a, b = int(sb[k]), int(sb[k + 1])
            assert np.array_equal(p[a:b], rp), (rep, k)
            assert np.array_equal(h[a:b], rh), (rep, k)
        torch.randn(1000, device="cuda").sum().item()


def _jobs(seed, count):
    rng = np.random.default_rng(seed)
    jobs = []
    for i in range(count):
        n = int(np.floor(2.0 ** rng.uniform(4, 14)))
        jobs.append(W.mixed_job(rng, n))
    return jobs


def _check_mix(jobs, alone, mixed):
    for j, (pa, ha), (pm, hm, info) in zip(jobs, alone, mixed):
        rp, rh = oracle.sort(j)
        assert np.array_equal(pa, rp) and np.array_equal(ha, rh)
        assert np.array_equal(pm, pa) and np.array_equal(hm, ha)
        assert info["latency_ms"] >= info["queue_ms"] >= 0


def test_server_results_alone_and_in_mix(ss_mod):
    ssort = ss_mod
    print("[systems] server", flush=True)
    jobs = _jobs(33, 40)
    srv = ssort.Server(0, budget_bytes=1 << 30, slots=4)
    alone = []
    for j in jobs:                      # one job at a time
        t = srv.submit(j)
        p, h, _ = srv.wait(t)
        alone.append((p.copy(), h.copy()))
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(jobs) and st["launches"] == len(jobs)
    # all at once on a one-slot server: the jobs queued while a launch runs
    # go out together in the next one
    srv = ssort.Server(0, budget_bytes=1 << 30, slots=1)
    tickets = [srv.submit(j) for j in jobs]
    mixed = [srv.wait(t) for t in tickets]
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(jobs)
    assert st["launches"] < len(jobs)     # the mix was batched
    _check_mix(jobs, alone, mixed)


def test_server_mix_behind_large_job(ss_mod):
    ssort = ss_mod
    jobs = _jobs(33, 40)
    srv = ssort.Server(0, budget_bytes=1 << 30, slots=1)
    tb = srv.submit(W.plain(1 << 20, seed=36))
    tickets = [srv.submit(j) for j in jobs]
    mixed = [srv.wait(t) for t in tickets]
    p, h, _ = srv.wait(tb)
    srv.close()
    rp, rh = oracle.sort(W.plain(1 << 20, seed=36))
    assert np.array_equal(p, rp) and np.array_equal(h, rh)
    for j, (pm, hm, _) in zip(jobs, mixed):
        rp, rh = oracle.sort(j)
        assert np.array_equal(pm, rp) and np.array_equal(hm, rh)


def test_server_budget_and_cancel(ss_mod):
    ssort = ss_mod
    srv = ssort.Server(0, budget_bytes=16 << 20, slots=1, stage_bytes=8 << 20)
    big = W.plain(400000, seed=34)             # > 16 MiB of device buffers
    with pytest.raises(ssort.SsortError) as e:
        srv.submit(big)
    assert e.value.code == 7
    small = [W.plain(20000, seed=35 + i) for i in range(6)]
    ts = [srv.submit(j) for j in small]
    cancelled = srv.cancel(ts[-1])              # may already have started: then it completes
    for t, j in zip(ts[:-1], small[:-1]):
        p, h, _ = srv.wait(t)
        rp, rh = oracle.sort(j)
        assert np.array_equal(p, rp) and np.array_equal(h, rh)
    if not cancelled:
        srv.wait(ts[-1])
    srv.close()
