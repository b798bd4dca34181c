"""Parity of the HIP path with the CPU oracle, element by element (bit-exact
permutation and LCP array), through the C ABI."""
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


def gpu_sort(sorter, ss, with_lcp=True):
    from paper_1403_2056_amd import ssort
    d = ssort.strings_to_device(ss)
    perm, lcp = sorter.sort(d, with_lcp=with_lcp)
    torch.cuda.synchronize()
    err = sorter.query_error()
    assert err == 0, f"device error {err}, error mask {sorter.stats()['error_bits']:#x}, stats {sorter.stats()}"
    p = ssort.to_numpy_u32(perm).copy()
    h = ssort.to_numpy_u32(lcp).copy() if with_lcp else None
    return p, h


def assert_parity(sorter, ss, label=""):
    print(f"[parity] {label} n={ss.n}", flush=True)
    p, h = gpu_sort(sorter, ss)
    rp, rh = oracle.sort(ss)
    if not np.array_equal(p, rp):
        bad = int(np.nonzero(p != rp)[0][0])
        raise AssertionError(f"{label}: perm differs first at {bad}: gpu {p[bad-2:bad+3]} oracle {rp[bad-2:bad+3]}")
    if not np.array_equal(h, rh):
        bad = int(np.nonzero(h != rh)[0][0])
        raise AssertionError(f"{label}: lcp differs first at {bad}: gpu {h[bad-2:bad+3]} oracle {rh[bad-2:bad+3]}")


def test_device_info(sorter):
    info = sorter.device_info()
    print("[device]", info, flush=True)
    assert info["cus"] == 256
    assert 10_000 <= info["wall_khz"] <= 1_000_000


def test_debug_step_rows(sorter):
    """One classification step: keys (8-byte big-endian gather), splitters and
    level-order tree, bucket numbers, counts and the stable redistribution."""
    from paper_1403_2056_amd import ssort
    ss = W.plain(100000, seed=14)
    for depth in (0, 3):
        out = sorter.debug_step(ssort.strings_to_device(ss), depth)
        keys = oracle.keys(ss, np.arange(ss.n), depth)
        assert np.array_equal(out["keys"], keys)
        x = out["split"]
        v = len(x)
        assert v == 2 ** int(out["info"][1]) - 1
        assert np.all(x[1:] >= x[:-1])
        assert set(x.tolist()) <= set(keys.tolist())
        ranks = oracle.tree_ranks(v)
        assert np.array_equal(out["tree"], x[ranks])
        b = oracle.classify(keys, x)
        assert np.array_equal(out["bucket"].astype(np.uint32), b)
        assert np.array_equal(out["hist"], np.bincount(b, minlength=2 * v + 1).astype(np.uint32))
        assert np.array_equal(out["perm"], np.argsort(b, kind="stable").astype(np.uint32))


def test_tiny_degenerate(sorter):
    for strs in ([b"a"], [b"b", b"a"], [b"", b""], [b"x"] * 3, [b"", b"a", b""], [b"abc", b"ab", b"abd"]):
        assert_parity(sorter, W.from_list(strs), f"tiny {strs}")


def test_empty_input(sorter):
    from paper_1403_2056_amd import ssort
    d = ssort.strings_to_device(W.from_list([]))
    perm, lcp = sorter.sort(d)
    torch.cuda.synchronize()
    assert perm.numel() == 0 and lcp.numel() == 0


@pytest.mark.parametrize("seed", range(24))
def test_adversarial(sorter, seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(2, 6000))
    strs = adversarial(rng, n)
    layout = "lengths" if seed % 3 == 1 else "csr"
    assert_parity(sorter, W.from_list(strs, layout=layout, pad=3 if layout == "lengths" else 0), f"adv{seed}")


def test_plain_small_config(sorter):
    assert_parity(sorter, W.plain(131072, seed=1), "plain n=131072")


def test_prefixes_scaled(sorter):
    assert_parity(sorter, W.prefixes(1 << 18, seed=2, n_prefix=64), "prefixes 2^18")


def test_suffixes_scaled(sorter):
    assert_parity(sorter, W.suffixes(1 << 18, seed=3), "suffixes 2^18")


def test_all_identical_large(sorter):
    assert_parity(sorter, W.from_list([b"samestring"] * 200000), "identical 200000")


@pytest.mark.parametrize("n", [700, 40000])
def test_largest_keys_with_ties(sorter, n):
    """Runs of 0xFF bytes make the largest key (all 64 bits set) at many
    depths, with equal keys at earlier and later positions of a class: the
    base case's (key, position) order must hold at the top of the key range,
    next to keys that differ from it only in their last byte."""
    rng = np.random.default_rng(n)
    tails = [b"", b"\x01", b"\xfe", b"\xff\x01", b"\xfe\xff", b"\x7f"]
    strs = [b"\xff" * int(rng.integers(0, 41)) + tails[int(rng.integers(0, len(tails)))] for _ in range(n)]
    strs += [strs[int(i)] for i in rng.integers(0, n, size=n // 5)]
    assert_parity(sorter, W.from_list(strs), f"0xFF runs {len(strs)}")


def test_long_common_prefix(sorter):
    rng = np.random.default_rng(7)
    p = b"q" * 700
    strs = [p + bytes(rng.integers(97, 101, size=rng.integers(0, 6)).astype(np.uint8)) for _ in range(100000)]
    assert_parity(sorter, W.from_list(strs), "shared prefix 700")


@pytest.mark.parametrize("n", [3041, 200000])
def test_few_long_shared_prefixes(sorter, n):
    """A few strings share long prefixes (40..690 bytes) with the first one and
    each other among many that differ early: short lists of long comparisons,
    handled by lane groups in the segment and base-case extensions."""
    rng = np.random.default_rng(n)
    X = bytes(rng.integers(97, 123, size=700).astype(np.uint8))
    strs = [b"ABCDEFGH" + X]
    for i in range(n - 41):
        s = b"ABCDEFGH"
        if i % 150 == 0:
            s += X[:int(rng.integers(40, 691))]
        strs.append(s + bytes(rng.integers(97, 123, size=int(rng.integers(0, 31))).astype(np.uint8)))
    strs += [b"ABCDEFGH" + X[:600] + bytes([int(rng.integers(97, 100))]) for _ in range(40)]
    assert_parity(sorter, W.from_list(strs), f"few long prefixes {n}")


def test_determinism(sorter):
    ss = W.plain(50000, seed=8)
    a = gpu_sort(sorter, ss)
    b = gpu_sort(sorter, ss)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_perm_only(sorter):
    ss = W.plain(70000, seed=9)
    p, _ = gpu_sort(sorter, ss, with_lcp=False)
    rp, _ = oracle.sort(ss, with_lcp=False)
    assert np.array_equal(p, rp)


@pytest.mark.parametrize("v,k,tb", [(1, 4, 16), (3, 4, 64), (63, 8, 128), (127, 4, 512), (255, 8, 1024),
                                    (255, 4, 64), (31, 8, 256)])
def test_tunings_give_identical_results(v, k, tb):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1403_2056_amd import ssort
    s = ssort.Sorter(0, v=v, keys_per_thread=k, base_threshold=tb)
    s.set_wait_limit(10000)
    assert_parity(s, W.plain(100000, seed=12), f"tuning v={v} k={k} tb={tb}")
    assert_parity(s, W.suffixes(1 << 16, seed=13), f"tuning v={v} k={k} tb={tb} suffixes")


@pytest.mark.parametrize("v", [7, 255])
def test_equal_classification_variant(v):
    """S5-Equal (equality test at every node, early exit) gives the same
    buckets as the lower-bound definition and the same sorted output."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1403_2056_amd import ssort
    s = ssort.Sorter(0, v=v, flags=ssort.SSORT_EQUAL)
    s.set_wait_limit(10000)
    for ss, label in ((W.plain(90000, seed=40), "plain"), (W.prefixes(1 << 17, seed=41, n_prefix=32), "prefixes"),
                      (W.from_list([b"dup"] * 3000 + [b"a", b"zz"]), "few keys")):
        out = s.debug_step(ssort.strings_to_device(ss), 0)
        keys = oracle.keys(ss, np.arange(ss.n), 0)
        assert np.array_equal(out["bucket"].astype(np.uint32), oracle.classify(keys, out["split"])), label
        assert_parity(s, ss, f"S5-Equal v={v} {label}")


def test_validate_reports_zero_byte():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1403_2056_amd import ssort
    s = ssort.Sorter(0, flags=ssort.SSORT_VALIDATE)
    ss = W.from_list([b"ab", b"a\x00b", b"c"])
    s.sort(ssort.strings_to_device(ss))
    torch.cuda.synchronize()
    assert s.query_error() == 5


def test_workspace_too_small(sorter):
    from paper_1403_2056_amd import ssort
    d = ssort.strings_to_device(W.plain(1000, seed=1))
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(ssort.SsortError) as e:
        sorter.sort(d, ws=ws)
    assert e.value.code == 3


def test_batched_small(sorter):
    from paper_1403_2056_amd import ssort
    ss, sb = W.batched(m=48, seed=15, lo=0, hi=11)
    d = ssort.strings_to_device(ss)
    sbt = torch.from_numpy(sb.view(np.int32)).cuda()
    perm, lcp = sorter.sort_batched(d, sbt)
    torch.cuda.synchronize()
    assert sorter.query_error() == 0, sorter.stats()
    p, h = ssort.to_numpy_u32(perm), ssort.to_numpy_u32(lcp)
    strs = ss.strings()
    for s in range(len(sb) - 1):
        a, b = int(sb[s]), int(sb[s + 1])
        sub = W.from_list(strs[a:b])
        rp, rh = oracle.sort(sub)
        assert np.array_equal(p[a:b], rp), s
        assert np.array_equal(h[a:b], rh), s


def test_batched_random_sweep():
    """Seeded batches of 1..120 sets, a tenth of them empty, the others mixes
    of the adversarial kinds (1..2500 strings), under random tunings: every
    set's permutation and LCP array equal the oracle's sort of that set."""
    from paper_1403_2056_amd import ssort
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rng = np.random.default_rng(7200)
    sorters = {}
    for c in range(30):
        sets = []
        for _ in range(int(rng.integers(1, 121))):
            sets.append([] if rng.random() < 0.1 else adversarial(rng, int(rng.integers(1, 2500))))
        sb = np.zeros(len(sets) + 1, dtype=np.uint32)
        sb[1:] = np.cumsum([len(s) for s in sets])
        if sb[-1] == 0:
            continue
        ss = W.from_list([x for s in sets for x in s])
        key = (int(rng.choice([7, 63, 255])), int(rng.choice([4, 8])), int(rng.choice([16, 128, 512])))
        if key not in sorters:
            sorters[key] = ssort.Sorter(0, v=key[0], keys_per_thread=key[1], base_threshold=key[2])
            sorters[key].set_wait_limit(10000)
        s = sorters[key]
        print(f"[batched sweep] {c}: {len(sets)} sets, n={ss.n}, tuning {key}", flush=True)
        perm, lcp = s.sort_batched(ssort.strings_to_device(ss), torch.from_numpy(sb.view(np.int32)).cuda())
        torch.cuda.synchronize()
        assert s.query_error() == 0, (c, s.stats())
        p, h = ssort.to_numpy_u32(perm), ssort.to_numpy_u32(lcp)
        for i, strs in enumerate(sets):
            a, b = int(sb[i]), int(sb[i + 1])
            if a == b:
                continue
            rp, rh = oracle.sort(W.from_list(strs))
            assert np.array_equal(p[a:b], rp), (c, i)
            assert np.array_equal(h[a:b], rh), (c, i)


def _level_one_strings(seed):
    """80000 strings behind one 8-byte key (an equality bucket above the
    second whole-GPU level's threshold of 2^16), 50000 in a range, some
    duplicates."""
    rng = np.random.default_rng(seed)
    strs = [b"commonpr" + bytes(rng.integers(97, 105, size=int(rng.integers(1, 13))).astype(np.uint8))
            for _ in range(80000)]
    strs += [b"zz" + bytes(rng.integers(97, 101, size=int(rng.integers(1, 13))).astype(np.uint8))
             for _ in range(50000)]
    for _ in range(3000):
        strs[int(rng.integers(0, 130000))] = strs[int(rng.integers(0, 130000))]
    return strs


def test_second_level(sorter):
    assert_parity(sorter, W.from_list(_level_one_strings(50)), "second whole-GPU level")


def test_batched_large_sets(sorter):
    """Sets above the whole-GPU threshold go through the levels, the others
    straight to the workers; every set equals its own oracle sort."""
    from paper_1403_2056_amd import ssort
    strs = _level_one_strings(51)
    rng = np.random.default_rng(52)
    sets = [strs[:100000]]
    for _ in range(5):
        sets.append([bytes(rng.integers(97, 100, size=int(rng.integers(0, 11))).astype(np.uint8))
                     for _ in range(int(rng.integers(0, 300)))])
    sets.append(strs[50000:120000])
    flat = [x for st in sets for x in st]
    sb = np.cumsum([0] + [len(st) for st in sets]).astype(np.uint32)
    ss = W.from_list(flat)
    d = ssort.strings_to_device(ss)
    perm, lcp = sorter.sort_batched(d, torch.from_numpy(sb.view(np.int32)).cuda())
    torch.cuda.synchronize()
    assert sorter.query_error() == 0, sorter.stats()
    p, h = ssort.to_numpy_u32(perm), ssort.to_numpy_u32(lcp)
    for k, st in enumerate(sets):
        a, b = int(sb[k]), int(sb[k + 1])
        rp, rh = oracle.sort(W.from_list(st))
        assert np.array_equal(p[a:b], rp), k
        assert np.array_equal(h[a:b], rh), k


def _alphabet_inputs():
    rng = np.random.default_rng(80)
    dna = W.suffixes(1 << 18, seed=81)                      # 4 symbols: 21 characters per key
    yield dna, "DNA suffixes 2^18"
    yield W.prefixes(1 << 17, seed=82, n_prefix=64), "prefixes 2^17 (64 symbols: 9 per key)"
    yield W.plain(100000, seed=83), "plain 100000 (26 symbols: 12 per key)"
    yield W.from_list([b"a" * int(k) for k in rng.integers(0, 90, 5000)]), "one symbol (32 per key)"
    yield W.from_list([bytes(rng.integers(97, 100, size=int(rng.integers(0, 70))).astype(np.uint8))
                       for _ in range(40000)]), "three symbols (32 per key)"
    yield W.from_list([bytes(rng.integers(1, 256, size=int(rng.integers(0, 30))).astype(np.uint8))
                       for _ in range(20000)]), "255 symbols (8 per key)"
    for strs in ([b"a"], [b"", b""], [b"x"] * 3, [b"", b"a", b""], [b"abc", b"ab", b"abd"]):
        yield W.from_list(strs), f"tiny {strs}"
    for seed in range(6):
        r = np.random.default_rng(2000 + seed)
        yield W.from_list(adversarial(r, int(r.integers(2, 6000)))), f"adversarial {seed}"


@pytest.mark.parametrize("v,k,tb", [(255, 4, 128), (63, 8, 64), (7, 4, 512)])
def test_alphabet_compression(v, k, tb):
    """Keys of packed order-preserving character codes (ceil(log2(sigma'+1))
    bits each): the same permutation and LCP array as the oracle."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1403_2056_amd import ssort
    s = ssort.Sorter(0, v=v, keys_per_thread=k, base_threshold=tb, flags=ssort.SSORT_ALPHABET)
    s.set_wait_limit(10000)
    for ss, label in _alphabet_inputs():
        assert_parity(s, ss, f"alphabet v={v} k={k} tb={tb} {label}")


def test_alphabet_compression_batched(sorter):
    """Batched sets (each below the whole-GPU level threshold) with packed keys."""
    from paper_1403_2056_amd import ssort
    s = ssort.Sorter(0, flags=ssort.SSORT_ALPHABET)
    s.set_wait_limit(10000)
    ss, sb = W.batched(m=48, seed=84, lo=0, hi=12)
    d = ssort.strings_to_device(ss)
    perm, lcp = s.sort_batched(d, torch.from_numpy(sb.view(np.int32)).cuda())
    torch.cuda.synchronize()
    assert s.query_error() == 0, s.stats()
    p, h = ssort.to_numpy_u32(perm), ssort.to_numpy_u32(lcp)
    strs = ss.strings()
    for k in range(len(sb) - 1):
        a, b = int(sb[k]), int(sb[k + 1])
        rp, rh = oracle.sort(W.from_list(strs[a:b]))
        assert np.array_equal(p[a:b], rp), k
        assert np.array_equal(h[a:b], rh), k


def test_batched_many_large_sets():
    """1024 sets of up to 2^16 strings in one launch, with the tuning (v = 63,
    base threshold 256) that publishes the most base-case chunks per step:
    every set is a permutation of itself with no device error, three times
    over, and sampled sets equal their oracle sort (a regression test for
    work-queue hand-over: a publishing store overtaking the L2 write-back of
    the data it publishes)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1403_2056_amd import ssort
    ss, sb = W.batched(m=1024, seed=90, lo=6, hi=16)
    print(f"[parity] many large sets n={ss.n}", flush=True)
    s = ssort.Sorter(0, v=63, keys_per_thread=4, base_threshold=256)
    s.set_wait_limit(10000)
    d = ssort.strings_to_device(ss)
    sbt = torch.from_numpy(sb.view(np.int32).copy()).cuda()
    perm = torch.empty(ss.n, dtype=torch.int32, device="cuda")
    lcp = torch.empty(ss.n, dtype=torch.int32, device="cuda")
    sizes = np.diff(sb.astype(np.int64))
    starts = sb[:-1].astype(np.int64)
    rng = np.random.default_rng(91)
    sample = rng.choice(len(sizes), size=12, replace=False)
    for rep in range(3):
        perm.fill_(-1)
        s.sort_batched(d, sbt, out_perm=perm, out_lcp=lcp)
        torch.cuda.synchronize()
        assert s.query_error() == 0, s.stats()
        p = ssort.to_numpy_u32(perm)
        # each set's entries are a permutation of 0..size-1
        ok = (p < np.repeat(sizes, sizes).astype(np.uint32))
        assert ok.all(), (rep, int(np.argmin(ok)))
        key = np.repeat(starts, sizes) + p.astype(np.int64)
        assert np.array_equal(np.sort(key), np.arange(ss.n)), rep
    h = ssort.to_numpy_u32(lcp)
    o = ss.offsets
    for k in sample:
        a, n_k = int(starts[k]), int(sizes[k])
        sub = W.from_list([ss.chars[int(o[j]):int(o[j + 1])].tobytes() for j in range(a, a + n_k)])
        rp, rh = oracle.sort(sub)
        assert np.array_equal(p[a:a + n_k], rp), k
        assert np.array_equal(h[a:a + n_k], rh), k
