"""One segment step of the persistent worker, row by row (through the C ABI):
splitters, splitter LCPs (against the oracle's byte loop), end flags, the
depth the step classifies at (the exact common prefix after an extension,
against brute force), bucket numbers, sizes and starts (the lower-bound
definition), the stable redistribution, and the child depths of Algorithm 1's
output checked by their defining property (Eq. (1)): every string of a bucket
shares the claimed prefix, and an equality bucket whose splitter ends the
string holds identical strings."""
import os

import numpy as np
import pytest

import oracle
from paper_1403_2056_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sorter():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1403_2056_amd import ssort
    s = ssort.Sorter(0)
    s.set_wait_limit(10000)
    return s


def _lcp(a: bytes, b: bytes) -> int:
    return len(os.path.commonprefix([a, b]))


def check_step(sorter, ss, depth, label):
    from paper_1403_2056_amd import ssort
    print(f"[segment step] {label} n={ss.n} depth={depth}", flush=True)
    out = sorter.debug_segment_step(ssort.strings_to_device(ss), depth)
    strs = ss.strings()
    v, d, h = int(out["info"][0]), int(out["info"][1]), int(out["info"][3])
    x = out["split"]
    assert v == 2 ** d - 1
    # the classification depth: the exact common prefix when every sampled key
    # was equal (an extension), else the segment's own depth
    common = min(_lcp(strs[0], s) for s in strs)
    assert h == depth or h == common, (h, depth, common)
    if h != depth:
        assert h > depth
    keys = oracle.keys(ss, np.arange(ss.n), h)
    assert np.all(x[1:] >= x[:-1])
    assert set(x.tolist()) <= set(keys.tolist())
    ndist = len(set(x.tolist()))
    # splitters repeat only as padding of the largest one
    assert np.all(x[1:ndist] > x[: ndist - 1])
    assert np.array_equal(out["hl"][1:ndist], oracle.splitter_lcp(x[:ndist])[1:ndist])
    assert out["hl"][0] == 0 and out["hl"][v] == 0
    assert np.array_equal(out["zr"], ((x & np.uint64(0xFF)) == 0).astype(np.uint32))
    b = oracle.classify(keys, x)
    size = np.bincount(b, minlength=2 * v + 1).astype(np.uint32)
    assert np.array_equal(out["size"], size)
    nz = size > 0
    start = np.concatenate([[0], np.cumsum(size)[:-1]]).astype(np.uint32)
    assert np.array_equal(out["start"][nz], start[nz])
    perm = out["perm"]
    assert np.array_equal(perm, np.argsort(b, kind="stable").astype(np.uint32))
    # Algorithm 1's output: every string of bucket i shares the claimed prefix
    for i in np.nonzero(nz)[0]:
        members = [strs[j] for j in perm[start[i]: start[i] + size[i]]]
        cd = int(out["depth"][i])
        assert cd >= h
        if (i & 1) and out["zr"][i >> 1]:
            assert all(m == members[0] for m in members), f"bucket {i}: not identical"
            continue
        cp = len(os.path.commonprefix(members)) if len(members) > 1 else len(members[0])
        if len(members) > 1:
            assert cp >= cd, f"bucket {i}: common prefix {cp} < child depth {cd}"
        assert all(len(m) >= cd for m in members) or len(members) == 1, f"bucket {i}"
    return h


def test_step_plain(sorter):
    h = check_step(sorter, W.plain(100000, seed=60), 0, "plain")
    assert h == 0


def test_step_extension_to_common_prefix(sorter):
    """Every string shares a 27-byte prefix: the step at depth 8 finds all
    sampled keys equal and classifies at the exact common prefix."""
    rng = np.random.default_rng(61)
    pre = bytes(rng.integers(97, 123, size=27).astype(np.uint8))
    strs = [pre + bytes(rng.integers(97, 123, size=int(rng.integers(0, 20))).astype(np.uint8)) for _ in range(60000)]
    h = check_step(sorter, W.from_list(strs), 8, "shared 27-byte prefix")
    assert h == 27


def test_step_extension_few_outliers(sorter):
    """Three strings leave the shared prefix early; the sample most likely
    misses them, and the exact extension still stops where they differ."""
    rng = np.random.default_rng(62)
    strs = [b"commonprefix" + bytes(rng.integers(97, 100, size=int(rng.integers(0, 9))).astype(np.uint8))
            for _ in range(30000)]
    for k in (17, 4000, 29000):
        strs[k] = b"commonpzz" + bytes([97 + k % 3])
    h = check_step(sorter, W.from_list(strs), 0, "outliers at byte 7")
    assert h in (0, 7)   # 0 only if the sample caught an outlier


def test_step_long_prefix(sorter):
    """A 700-byte shared prefix: the extension's lane-group and per-thread
    comparisons beyond the first 32 bytes."""
    rng = np.random.default_rng(63)
    p = b"q" * 700
    strs = [p + bytes(rng.integers(97, 101, size=int(rng.integers(0, 6))).astype(np.uint8)) for _ in range(20000)]
    h = check_step(sorter, W.from_list(strs), 0, "700-byte prefix")
    assert h == 700


def test_step_terminated_and_duplicates(sorter):
    """Short strings over two letters: splitters that end their strings
    (finished identical buckets), duplicates, the empty string."""
    rng = np.random.default_rng(64)
    strs = [bytes(rng.integers(97, 99, size=int(rng.integers(0, 7))).astype(np.uint8)) for _ in range(50000)]
    check_step(sorter, W.from_list(strs), 0, "terminated keys")


def test_step_prefix_groups(sorter):
    """The long-prefix workload's shape, one prefix group per step at depth 8."""
    check_step(sorter, W.prefixes(1 << 16, seed=65, n_prefix=16), 0, "16 prefix groups")
    ss = W.prefixes(1 << 16, seed=66, n_prefix=1)
    check_step(sorter, ss, 8, "one prefix group at depth 8")
