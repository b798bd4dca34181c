"""The batched form at its full size: 4096 sets of 2^U(6,18) strings
(geometric lengths with mean 24, 95 printable bytes; about 128 M strings and
3.1 GB of characters) in one launch sequence, every set checked exactly by the
oracle's O(L+n) checker (which fixes each set's order and LCP array)."""
import numpy as np
import pytest

import oracle
from paper_1403_2056_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_batched_4096_sets_every_set_checked():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import bench
    from paper_1403_2056_amd import autotune, ssort
    print("[batched-full] generating 4096 sets", flush=True)
    ss, sb = W.batched()
    n = ss.n
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    tun = autotune.lookup(arch, "batched", n) or dict(bench.BATCHED_FALLBACK_TUNING)
    print(f"[batched-full] n={n} N={len(ss.chars)} tuning={tun}", flush=True)
    s = ssort.Sorter(0, **tun)
    s.set_wait_limit(20000)
    d = ssort.strings_to_device(ss)
    sbt = torch.from_numpy(sb.view(np.int32)).cuda()
    p, h = s.sort_batched(d, sbt)
    torch.cuda.synchronize()
    assert s.query_error() == 0, s.stats()
    p = ssort.to_numpy_u32(p)
    h = ssort.to_numpy_u32(h)
    del d
    print("[batched-full] sorted; checking every set", flush=True)
    bad = []
    for k in range(len(sb) - 1):
        a, b = int(sb[k]), int(sb[k + 1])
        sub = W.StringSet(ss.chars, ss.offsets[a: b + 1].copy(), None, 0, b - a, {})
        if oracle.check(sub, p[a:b], h[a:b]) != -1:
            bad.append(k)
    assert not bad, bad[:10]
