"""K-way LCP-merge (Algorithms 2-4) through the C ABI: sorted runs with
their LCP arrays merge into exactly the oracle's sort of all strings and its
LCP array (equal strings by index)."""
import numpy as np
import pytest

import oracle
from paper_1403_2056_amd import workloads as W
from tests.cases import adversarial

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


def runs_from(ss, K, seed, contiguous=False):
    """Split the indices of ss into K runs (random assignment, or contiguous
    ranges), sort every run with the oracle and return run boundaries,
    concatenated sorted indices and LCP arrays."""
    rng = np.random.default_rng(seed)
    n = ss.n
    owner = (np.arange(n) * K // max(n, 1)) if contiguous else rng.integers(0, K, size=n)
    strs = ss.strings()
    rb, pin, hin = [0], [], []
    for k in range(K):
        idx = np.nonzero(owner == k)[0]
        if len(idx):
            rp, rh = oracle.sort(W.from_list([strs[i] for i in idx]))
            pin.append(idx[rp].astype(np.uint32))
            hin.append(rh.astype(np.uint32))
        rb.append(rb[-1] + len(idx))
    cat = lambda a: np.concatenate(a) if a else np.zeros(0, np.uint32)
    return rb, cat(pin), cat(hin)


def merge_parity(sorter, ss, K, seed, label, contiguous=False):
    from paper_1403_2056_amd import ssort
    print(f"[merge] {label} n={ss.n} K={K}", flush=True)
    rb, pin, hin = runs_from(ss, K, seed, contiguous)
    d = ssort.strings_to_device(ss)
    tp = torch.from_numpy(pin.view(np.int32)).cuda()
    th = torch.from_numpy(hin.view(np.int32)).cuda()
    p, h = sorter.merge(d, rb, tp, th)
    torch.cuda.synchronize()
    assert sorter.query_error() == 0, sorter.stats()
    rp, rh = oracle.sort(ss)
    p, h = ssort.to_numpy_u32(p), ssort.to_numpy_u32(h)
    if not np.array_equal(p, rp):
        bad = int(np.nonzero(p != rp)[0][0])
        raise AssertionError(f"{label}: perm differs at {bad}")
    if not np.array_equal(h, rh):
        bad = int(np.nonzero(h != rh)[0][0])
        raise AssertionError(f"{label}: lcp differs at {bad}: {h[bad]} vs {rh[bad]}")


@pytest.mark.parametrize("K", [1, 2, 3, 5, 8, 12, 32])
def test_merge_plain(sorter, K):
    merge_parity(sorter, W.plain(60000, seed=60 + K), K, K, f"plain K={K}")


@pytest.mark.parametrize("K", [4, 16])
def test_merge_long_prefixes(sorter, K):
    merge_parity(sorter, W.prefixes(1 << 17, seed=70, n_prefix=64), K, 3, f"prefixes K={K}")


def test_merge_suffixes_contiguous_runs(sorter):
    merge_parity(sorter, W.suffixes(1 << 16, seed=71), 8, 4, "suffixes", contiguous=True)


def test_merge_adversarial(sorter):
    for i in range(12):
        rng = np.random.default_rng(720 + i)
        strs = adversarial(rng, int(rng.integers(1, 3000)))
        if strs:
            merge_parity(sorter, W.from_list(strs), 1 + i % 6, i, f"adversarial {i}")


def test_merge_random_sweep(sorter):
    """Seeded mixes of the adversarial kinds split into K = 1..32 runs, at
    random or in contiguous ranges (many cut searches land in long runs of
    equal strings or of strings that are prefixes of one another)."""
    rng = np.random.default_rng(7300)
    for c in range(160):
        strs = []
        for _ in range(int(rng.integers(1, 4))):
            strs += adversarial(rng, int(rng.integers(1, 5000)))
        if not strs:
            continue
        rng.shuffle(strs)
        K = int(rng.integers(1, 33))
        merge_parity(sorter, W.from_list(strs), K, int(rng.integers(0, 1 << 30)), f"sweep {c}",
                     contiguous=bool(rng.random() < 0.3))


def test_merge_identical_and_empty_runs(sorter):
    from paper_1403_2056_amd import ssort
    ss = W.from_list([b"same"] * 5000 + [b"x", b""] * 100)
    merge_parity(sorter, ss, 5, 9, "identical")
    # empty runs, K = 32 with most runs empty
    rb, pin, hin = runs_from(ss, 3, 10)
    rb = rb + [rb[-1]] * 29
    d = ssort.strings_to_device(ss)
    p, h = sorter.merge(d, rb, torch.from_numpy(pin.view(np.int32)).cuda(), torch.from_numpy(hin.view(np.int32)).cuda())
    torch.cuda.synchronize()
    rp, rh = oracle.sort(ss)
    assert np.array_equal(ssort.to_numpy_u32(p), rp) and np.array_equal(ssort.to_numpy_u32(h), rh)


def test_merge_of_gpu_sorted_runs(sorter):
    """Runs sorted by the GPU sorter itself (batched), then merged."""
    from paper_1403_2056_amd import ssort
    ss = W.prefixes(1 << 18, seed=73, n_prefix=64)
    K = 8
    bounds = [ss.n * k // K for k in range(K + 1)]
    d = ssort.strings_to_device(ss)
    sb = torch.tensor(bounds, dtype=torch.int32).cuda()
    p, h = sorter.sort_batched(d, sb)     # set-local indices
    off = torch.repeat_interleave(torch.tensor(bounds[:-1], dtype=torch.int32),
                                  torch.tensor(np.diff(bounds), dtype=torch.int64)).cuda()
    pg = (p + off).contiguous()
    m, hm = sorter.merge(d, bounds, pg, h)
    torch.cuda.synchronize()
    rp, rh = oracle.sort(ss)
    assert np.array_equal(ssort.to_numpy_u32(m), rp)
    assert np.array_equal(ssort.to_numpy_u32(hm), rh)


def test_merge_rejects_bad_runs(sorter):
    from paper_1403_2056_amd import ssort
    ss = W.plain(100, seed=74)
    d = ssort.strings_to_device(ss)
    t = torch.zeros(100, dtype=torch.int32).cuda()
    with pytest.raises(ssort.SsortError):
        sorter.merge(d, [0, 60, 50, 100], t, t)
    with pytest.raises(ssort.SsortError):
        sorter.merge(d, [0] + [100] * 33, t, t)


def test_merge_index_in_two_runs_is_a_device_error(sorter):
    """An index at the start of two runs gives two samples of the same rank,
    so one cut row stays unwritten: the merge ends with SSORT_EDEVICE (error
    bit 512) instead of reading the row."""
    from paper_1403_2056_amd import ssort
    import os
    ss = W.plain(4000, seed=75)
    strs = ss.strings()
    rp = oracle.sort(ss)[0].astype(np.uint32)
    x = rp[0]                          # the set's smallest (string, index)
    runs = [rp[0::2], np.concatenate([[x], rp[1::2]]).astype(np.uint32)]   # x starts both runs
    lcps = [np.array([0] + [len(os.path.commonprefix([strs[r[i - 1]], strs[r[i]]])) for i in range(1, len(r))],
                     dtype=np.uint32) for r in runs]
    rb = [0, len(runs[0]), len(runs[0]) + len(runs[1])]
    pin, hin = np.concatenate(runs), np.concatenate(lcps)
    d = ssort.strings_to_device(ss)
    sorter.merge(d, rb, torch.from_numpy(pin.view(np.int32)).cuda(), torch.from_numpy(hin.view(np.int32)).cuda())
    torch.cuda.synchronize()
    assert sorter.query_error() == ssort.STATUS_CODES["SSORT_EDEVICE"]
    assert sorter.stats()["error_bits"] & 512
    # the context still sorts and merges correctly afterwards
    merge_parity(sorter, ss, 3, 12, "after a rejected merge")


def test_merge_error_word_outlives_the_call(sorter):
    """The merge workspace (with the error word ssort_query_error reads) stays
    allocated after the call, so an unrelated allocation filled with ones
    cannot land on it."""
    from paper_1403_2056_amd import ssort
    ss = W.plain(30000, seed=76)
    rb, pin, hin = runs_from(ss, 4, 13)
    d = ssort.strings_to_device(ss)
    sorter.merge(d, rb, torch.from_numpy(pin.view(np.int32)).cuda(), torch.from_numpy(hin.view(np.int32)).cuda())
    torch.cuda.synchronize()
    junk = [torch.full((1 << 16,), -1, dtype=torch.int64, device="cuda") for _ in range(64)]
    torch.cuda.synchronize()
    assert sorter.query_error() == 0
    assert sorter.stats()["error_bits"] == 0
    del junk


def test_merge_full_size_long_prefixes(sorter):
    """The merge at the benchmark's size: 8 runs (contiguous index ranges,
    each sorted by the GPU) of 2^24 long-prefix strings, merged twice into
    sentinel-filled outputs.  Every position is written, both merges equal
    the full sort (element by element, permutation and LCP array), and at
    sampled positions the order and LCP hold against the strings themselves
    (the oracle's byte loop, at any size)."""
    import os
    from paper_1403_2056_amd import ssort
    ss = W.prefixes(1 << 24, seed=2)
    n, K = ss.n, 8
    print(f"[merge] full size n={n} K={K}", flush=True)
    bounds = [n * k // K for k in range(K + 1)]
    d = ssort.strings_to_device(ss)
    sb = torch.tensor(bounds, dtype=torch.int32).cuda()
    p, h = sorter.sort_batched(d, sb)
    off = torch.repeat_interleave(torch.tensor(bounds[:-1], dtype=torch.int32),
                                  torch.tensor(np.diff(bounds), dtype=torch.int64)).cuda()
    pg = (p + off).contiguous()
    fp, fh = sorter.sort(d)
    torch.cuda.synchronize()
    fp, fh = ssort.to_numpy_u32(fp), ssort.to_numpy_u32(fh)
    for rep in range(2):
        m = torch.full((n,), -1, dtype=torch.int32, device="cuda")
        hm = torch.full((n,), -1, dtype=torch.int32, device="cuda")
        sorter.merge(d, bounds, pg, h, out_perm=m, out_lcp=hm)
        torch.cuda.synchronize()
        assert sorter.query_error() == 0, sorter.stats()
        mp, mh = ssort.to_numpy_u32(m), ssort.to_numpy_u32(hm)
        assert not np.any(mp == 0xFFFFFFFF) and not np.any(mh == 0xFFFFFFFF), rep
        if not np.array_equal(mp, fp):
            raise AssertionError(f"rep {rep}: perm differs from the full sort at {int(np.nonzero(mp != fp)[0][0])}")
        if not np.array_equal(mh, fh):
            bad = np.nonzero(mh != fh)[0]
            raise AssertionError(f"rep {rep}: {len(bad)} LCPs differ from the full sort, first at {int(bad[0])}")
    strs = ss.strings()
    rng = np.random.default_rng(74)
    for q in rng.integers(1, n, size=20000):
        a, b = strs[int(mp[q - 1])], strs[int(mp[q])]
        lcp = len(os.path.commonprefix([a, b]))
        assert int(mh[q]) == lcp, q
        assert a < b or (a == b and mp[q - 1] < mp[q]), q
