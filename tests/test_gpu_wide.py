"""Wide first level (v = 1023 ... 4095 splitters: the larger trees of the
implementation details of S5, with the jump table and the two-pass
distribution of the paper's refinements): the level-0 step row by row against
the oracle's definitions, and whole sorts element by element against the
oracle, through the C ABI."""
import numpy as np
import pytest

import oracle
from paper_1403_2056_amd import workloads as W
from tests.cases import adversarial
from tests.test_gpu_parity import assert_parity, _level_one_strings

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

JA = 12


def _sorter(**kw):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1403_2056_amd import ssort
    s = ssort.Sorter(0, **kw)
    s.set_wait_limit(10000)
    return s


def _check_jump(jump, tree, v):
    """The jump table by its defining property: for every value p of a key's
    top JA bits, the path from the root to jump[p] takes at every node the
    turn that p alone decides (p above the node's top bits: right, below:
    left, never equal), and it stops at a node (<= v) only where p equals that
    node's top bits; a stop beyond v is a leaf."""
    top = (tree >> np.uint64(64 - JA)).astype(np.int64)     # top bits of node j at top[j - 1]
    for p in range(1 << JA):
        i = int(jump[p])
        assert 1 <= i <= 2 * v + 1, (p, i)
        depth = i.bit_length() - 1
        for lev in range(depth):
            a = i >> (depth - lev)                      # ancestor at this level
            right = (i >> (depth - lev - 1)) & 1
            t = int(top[a - 1])
            assert p != t, (p, i, a)
            assert right == (1 if p > t else 0), (p, i, a)
        if i <= v:
            assert p == int(top[i - 1]), (p, i)


def _rows(s, ss, depth):
    from paper_1403_2056_amd import ssort
    out = s.debug_step(ssort.strings_to_device(ss), depth)
    keys = oracle.keys(ss, np.arange(ss.n), depth)
    assert np.array_equal(out["keys"], keys)
    x = out["split"]
    v = len(x)
    assert v == 2 ** int(out["info"][1]) - 1
    assert int(out["info"][3]) == JA
    assert np.all(x[1:] >= x[:-1])
    assert set(x.tolist()) <= set(keys.tolist())
    assert np.array_equal(out["tree"], x[oracle.tree_ranks(v)])
    _check_jump(out["jump"], out["tree"], v)
    b = oracle.classify(keys, x)
    assert np.array_equal(out["bucket"].astype(np.uint32), b)
    assert np.array_equal(out["hist"], np.bincount(b, minlength=2 * v + 1).astype(np.uint32))
    assert np.array_equal(out["perm"], np.argsort(b, kind="stable").astype(np.uint32))
    return v


@pytest.mark.parametrize("v", [1023, 4095])
def test_wide_step_rows(v):
    """Keys, splitters (sorted sample keys), level-order tree, jump table,
    bucket numbers (lower-bound definition), counts and the stable two-pass
    redistribution (= stable argsort by bucket) of one wide step."""
    s = _sorter(v=v)
    got = _rows(s, W.plain(200000, seed=90), 0)
    assert got == v
    _rows(s, W.plain(200000, seed=91), 3)
    _rows(s, W.prefixes(1 << 17, seed=92, n_prefix=3000), 0)
    # keys at both ends of the jump table: top bits all ones and all zeros
    rng = np.random.default_rng(93)
    strs = [bytes([0xFF, 0xFF]) + bytes(rng.integers(1, 256, size=int(rng.integers(0, 9))).astype(np.uint8))
            for _ in range(40000)]
    strs += [bytes([1]) + bytes(rng.integers(1, 3, size=int(rng.integers(0, 9))).astype(np.uint8))
             for _ in range(40000)]
    strs += [b"" for _ in range(5000)]
    _rows(s, W.from_list(strs), 0)


def _wide_inputs():
    rng = np.random.default_rng(94)
    yield W.plain(131072, seed=1), "plain n=131072"
    yield W.prefixes(1 << 18, seed=2, n_prefix=64), "prefixes 2^18, 64 prefixes"
    yield W.prefixes(1 << 18, seed=95, n_prefix=4096), "prefixes 2^18, 4096 prefixes"
    yield W.suffixes(1 << 18, seed=3), "suffixes 2^18"
    yield W.from_list(_level_one_strings(96)), "equality bucket above the second level's threshold"
    yield W.from_list([b"samestring"] * 100000), "identical 100000"
    yield W.from_list([b""] * 70000 + [b"a"] * 3), "empty strings"
    for seed in range(4):
        r = np.random.default_rng(3000 + seed)
        strs = []
        while len(strs) < 70000:
            strs += adversarial(r, 6000)
        yield W.from_list(strs), f"adversarial mix {seed}"


@pytest.mark.parametrize("v,k,tb", [(1023, 4, 128), (4095, 4, 128), (2047, 8, 64), (4095, 8, 1024)])
def test_wide_parity(v, k, tb):
    s = _sorter(v=v, keys_per_thread=k, base_threshold=tb)
    for ss, label in _wide_inputs():
        assert_parity(s, ss, f"wide v={v} k={k} tb={tb} {label}")


def test_wide_batched():
    """Sets above the level threshold share the wide level (one tree each),
    smaller ones go straight to the workers; each set equals its own oracle sort."""
    from paper_1403_2056_amd import ssort
    s = _sorter(v=4095)
    rng = np.random.default_rng(97)
    sets = [W.plain(100000, seed=98).strings(), _level_one_strings(99)[:90000]]
    for _ in range(6):
        sets.append([bytes(rng.integers(97, 100, size=int(rng.integers(0, 11))).astype(np.uint8))
                     for _ in range(int(rng.integers(0, 3000)))])
    sets.append(W.prefixes(1 << 17, seed=100, n_prefix=512).strings())
    flat = [x for st in sets for x in st]
    sb = np.cumsum([0] + [len(st) for st in sets]).astype(np.uint32)
    d = ssort.strings_to_device(W.from_list(flat))
    perm, lcp = s.sort_batched(d, torch.from_numpy(sb.view(np.int32)).cuda())
    torch.cuda.synchronize()
    assert s.query_error() == 0, s.stats()
    p, h = ssort.to_numpy_u32(perm), ssort.to_numpy_u32(lcp)
    for k, st in enumerate(sets):
        a, b = int(sb[k]), int(sb[k + 1])
        rp, rh = oracle.sort(W.from_list(st))
        assert np.array_equal(p[a:b], rp), k
        assert np.array_equal(h[a:b], rh), k


def test_wide_with_alphabet_and_equal():
    from paper_1403_2056_amd import ssort
    s = _sorter(v=4095, flags=ssort.SSORT_ALPHABET)
    assert_parity(s, W.suffixes(1 << 18, seed=101), "wide + alphabet, DNA suffixes")
    assert_parity(s, W.prefixes(1 << 17, seed=102, n_prefix=256), "wide + alphabet, prefixes")
    s = _sorter(v=1023, flags=ssort.SSORT_EQUAL)
    assert_parity(s, W.prefixes(1 << 17, seed=103, n_prefix=1024), "wide + S5-Equal steps, prefixes")


def test_wide_tuning_validation():
    from paper_1403_2056_amd import ssort
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    for v in (511, 8191, 1000):
        with pytest.raises(ssort.SsortError):
            ssort.Sorter(0, v=v)
