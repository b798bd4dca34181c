"""Pins of the CPU oracle against facts it does not compute itself:
textbook sorting of python byte strings, brute force on tiny inputs, the
paper's printed dataset statistics through closed forms, Fig. 1, and
library routines for the single-step helpers."""
import bisect
import itertools
import math
import os

import numpy as np
import pytest

import oracle
from paper_1403_2056_amd import workloads as W
from tests.cases import adversarial

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def brute(strs):
    """Python's own ordering of bytes objects is the canonical lexicographic
    order over unsigned bytes with a proper prefix first."""
    perm = sorted(range(len(strs)), key=lambda i: (strs[i], i))
    lcp = [0] * len(strs)
    for i in range(1, len(strs)):
        lcp[i] = len(os.path.commonprefix([strs[perm[i - 1]], strs[perm[i]]]))
    return perm, lcp


def run(strs, layout="csr", pad=0):
    ss = W.from_list(strs, layout=layout, pad=pad)
    perm, lcp = oracle.sort(ss)
    return ss, list(perm), list(lcp)


def test_exhaustive_tiny():
    alphabet = [b""] + [bytes(p) for k in (1, 2, 3) for p in itertools.product(b"ab", repeat=k)]
    assert len(alphabet) == 15
    count = 0
    for n in range(0, 4):
        for combo in itertools.product(alphabet, repeat=n):
            strs = list(combo)
            ss, perm, lcp = run(strs)
            assert (perm, lcp) == brute(strs), strs
            assert oracle.check(ss, perm, lcp) == -1
            count += 1
    assert count == 1 + 15 + 225 + 3375


@pytest.mark.parametrize("seed", range(40))
def test_random_adversarial(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(0, 2000))
    strs = adversarial(rng, n)
    layout = "lengths" if seed % 3 == 1 else "csr"
    ss, perm, lcp = run(strs, layout=layout, pad=5 if layout == "lengths" else 0)
    assert (perm, lcp) == brute(strs)
    assert oracle.check(ss, perm, lcp) == -1


def test_to_end_layout_suffixes():
    text = W.suffix_text(3000, seed=9, block=256)
    ss = W.StringSet(text, np.arange(len(text), dtype=np.uint64), None, W.FLAG_TO_END, len(text), {})
    perm, lcp = oracle.sort(ss)
    strs = [bytes(text[i:]) for i in range(len(text))]
    bp, bl = brute(strs)
    assert list(perm) == bp and list(lcp) == bl


def test_generators_plain_against_brute():
    ss = W.plain(3000, seed=11)
    perm, lcp = oracle.sort(ss)
    bp, bl = brute(ss.strings())
    assert list(perm) == bp and list(lcp) == bl


@pytest.mark.parametrize("planted", ["swap", "lcp_up", "lcp_down", "tie", "dup", "lcp0"])
def test_checker_rejects_planted_mistakes(planted):
    strs = [b"ab", b"abc", b"abc", b"b", b"ab", b"", b"abd", b"ba"]
    ss, perm, lcp = run(strs)
    perm, lcp = np.array(perm, dtype=np.uint32), np.array(lcp, dtype=np.uint32)
    assert oracle.check(ss, perm, lcp) == -1
    p, h = perm.copy(), lcp.copy()
    if planted == "swap":
        p[5], p[6] = p[6], p[5]
    elif planted == "lcp_up":
        h[3] += 1
    elif planted == "lcp_down":
        h[4] -= 1 if h[4] else 0
        h[2] = max(int(h[2]) - 1, 0)
    elif planted == "tie":      # identical strings out of index order
        i = [k for k in range(1, len(p)) if strs[p[k]] == strs[p[k - 1]]][0]
        p[i], p[i - 1] = p[i - 1], p[i]
    elif planted == "dup":
        p[1] = p[0]
    elif planted == "lcp0":
        h[0] = 1
    assert oracle.check(ss, p, h) != -1


# ---- closed forms for the paper's "Random" input and the DNA row ----

def random_closed_form(n, sigma=94, lmax=20):
    """Expected D/N (paper convention: one terminator per string) and L/n for
    n strings with lengths uniform in [0,lmax) and i.i.d. uniform bytes.
    A string of length l needs 1 + sum_{k<=l} P(M >= k) characters, M the
    largest lcp with another string; sum_k H >= k counts, per depth k, the
    strings of length >= k minus their distinct k-prefixes."""
    e_dist = 0.0
    for l in range(lmax):
        s = 1.0
        for k in range(1, l + 1):
            pk = (lmax - k) / lmax * sigma ** (-k)
            s += -math.expm1((n - 1) * math.log1p(-pk))
        e_dist += s / lmax
    dn = e_dist / ((lmax - 1) / 2 + 1)
    ln = 0.0
    for k in range(1, lmax):
        P = (lmax - k) / lmax
        pk = P * sigma ** (-k)
        ln += P - sigma ** k * (-math.expm1(n * math.log1p(-pk))) / n
    return dn, ln


def fixed_len_closed_form(n, length, sigma):
    e_dist = 1.0
    ln = 0.0
    for k in range(1, length + 1):
        pk = sigma ** (-k)
        e_dist += -math.expm1((n - 1) * math.log1p(-pk))
        ln += 1 - sigma ** k * (-math.expm1(n * math.log1p(-pk))) / n
    return e_dist / (length + 1), ln


def _golden_rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                rows.append(line.split())
    return rows


def test_closed_form_reproduces_paper_random_rows():
    rows = _golden_rows("paper_random_dn.txt")
    for r in rows:
        if r[0] == "Ln":
            dn, ln = random_closed_form(int(r[1]) / 10.5)
            assert round(ln, 1) == float(r[2])
        else:
            dn, _ = random_closed_form(int(r[0]) / 10.5)
            assert abs(100 * dn - float(r[1])) <= 0.05 + 1e-9, r


def test_closed_form_reproduces_dna_row():
    g = {r[0]: r[1] for r in _golden_rows("sinha_dna.txt")}
    dn, ln = fixed_len_closed_form(int(g["n"]), int(g["len"]), int(g["sigma"]))
    assert round(100 * dn) == int(g["D_over_N_percent"])
    assert round(ln, 1) == float(g["L_over_n"])


@pytest.mark.parametrize("n", [1 << 16, 1 << 20])
def test_oracle_D_L_match_closed_form_random(n):
    ss = W.paper_random(n, seed=21)
    perm, lcp = oracle.sort(ss)
    st = oracle.stats(ss, perm, lcp)
    dn, ln = random_closed_form(n)
    # within 0.1 percentage points of the closed form (measured: 0.02-0.04)
    assert abs(st["D_paper"] / st["N_paper"] - dn) < 0.001
    assert abs(st["L"] / n - ln) < 0.02
    # the two D conventions differ exactly by the strings that need their terminator
    assert st["D"] <= st["D_paper"] <= st["D"] + n
    assert st["N_paper"] == st["N"] + n


def test_oracle_D_L_match_closed_form_dna():
    n, length = 1 << 18, 9
    rng = np.random.default_rng(5)
    chars = np.frombuffer(b"ACGT", dtype=np.uint8)[rng.integers(0, 4, size=n * length)]
    off = np.arange(n + 1, dtype=np.uint64) * length
    ss = W.StringSet(chars, off, None, 0, n, {})
    perm, lcp = oracle.sort(ss)
    st = oracle.stats(ss, perm, lcp)
    dn, ln = fixed_len_closed_form(n, length, 4)
    assert abs(st["D_paper"] / st["N_paper"] - dn) < 0.003
    assert abs(st["L"] / n - ln) < 0.01


# ---- single-step helpers ----

def test_keys_big_endian_zero_padded():
    strs = [b"", b"a", b"abcdefgh", b"abcdefghij", b"\xff\x01", b"xyz" * 5]
    ss = W.from_list(strs)
    for depth in (0, 1, 3, 8, 9, 20):
        k = oracle.keys(ss, np.arange(len(strs)), depth)
        for i, s in enumerate(strs):
            ref = int.from_bytes((s[depth:depth + 8] + b"\0" * 8)[:8], "big")
            assert int(k[i]) == ref


def test_classify_is_lower_bound():
    rng = np.random.default_rng(3)
    for v in (1, 3, 7, 63, 255):
        x = np.unique(rng.integers(0, 1000, size=v * 3).astype(np.uint64))[:v]
        x.sort()
        keys = np.concatenate([x, x + 1, rng.integers(0, 1100, size=500).astype(np.uint64)])
        b = oracle.classify(keys, x)
        xs = [int(t) for t in x]
        for k, m in zip(keys, b):
            l = bisect.bisect_left(xs, int(k))
            assert m == 2 * l + (1 if l < len(xs) and xs[l] == int(k) else 0)


def test_tree_fig1():
    rows = {r[0]: r[1:] for r in _golden_rows("fig1_tree.txt")}
    v = int(rows["v"][0])
    assert list(oracle.tree_ranks(v)) == [int(t) for t in rows["level_order"]]
    assert 2 * v + 1 == int(rows["buckets"][0])


@pytest.mark.parametrize("d", range(1, 10))
def test_tree_level_order_closed_form_and_inorder(d):
    v = 2 ** d - 1
    r = oracle.tree_ranks(v)
    for j in range(1, v + 1):
        delta = j.bit_length() - 1
        p = j - 2 ** delta
        assert r[j - 1] == (2 * p + 1) * 2 ** (d - 1 - delta) - 1
    out = []

    def inorder(j):
        if j > v:
            return
        inorder(2 * j)
        out.append(int(r[j - 1]))
        inorder(2 * j + 1)
    inorder(1)
    assert out == list(range(v))


def test_splitter_lcp_byte_loop():
    rng = np.random.default_rng(4)
    x = np.sort(rng.integers(0, 2**63, size=200, dtype=np.int64).astype(np.uint64))
    x[50] = x[49]
    x[60] = x[59] ^ np.uint64(1)
    h = oracle.splitter_lcp(x)
    assert h[0] == 0 and h[len(x)] == 0
    for i in range(1, len(x)):
        a, b = int(x[i - 1]).to_bytes(8, "big"), int(x[i]).to_bytes(8, "big")
        assert h[i] == len(os.path.commonprefix([a, b]))


# ---- the distinguishing prefix D by its definition, over all pairs ----

def brute_dist(strs):
    """Distinguishing characters of each string by the definition
    (Preliminaries): the characters needed to tell it from every other
    string, 1 + the longest LCP with any other string (all pairs), but never
    more than the string itself (length-delimited form) or its terminator
    (the paper's convention, one terminator per string)."""
    out, out_paper = [], []
    for i, s in enumerate(strs):
        m = 0
        for j, t in enumerate(strs):
            if j != i:
                m = max(m, len(os.path.commonprefix([s, t])))
        out.append(min(len(s), 1 + m))
        out_paper.append(min(len(s) + 1, 1 + m))
    return out, out_paper


D_CASES = {
    "prefix_chain": [b"a", b"ab", b"abc", b"abcd", b"abcde", b"b"],
    "identical": [b"xyz", b"xyz", b"xyz", b"xy", b"x"],
    "empty_and_single": [b"", b"", b"q", b"qq"],
    "shared_then_split": [b"commonprefix" + bytes([c]) for c in b"azbyc"] + [b"commonprefix"],
    "one_string": [b"hello"],
}


@pytest.mark.parametrize("name", sorted(D_CASES) + [f"adv{k}" for k in range(12)])
def test_D_matches_all_pairs_definition(name):
    import bench
    if name in D_CASES:
        strs = D_CASES[name]
    else:
        rng = np.random.default_rng(300 + int(name[3:]))
        strs = adversarial(rng, int(rng.integers(1, 160)))
    ss = W.from_list(strs)
    perm, lcp = oracle.sort(ss)
    st = oracle.stats(ss, perm, lcp)
    dist, dist_paper = brute_dist(strs)
    assert st["D"] == sum(dist)
    assert st["D_paper"] == sum(dist_paper)
    lens = np.array([len(s) for s in strs], dtype=np.uint64)
    assert int(bench.dist_bytes(lens[perm], lcp).sum()) == sum(dist)
    assert st["N"] == int(lens.sum()) and st["N_paper"] == int(lens.sum()) + len(strs)


def test_D_cases_tell_plausible_mistakes_apart():
    """The fixed cases above fail a D computed as D_paper, or without the
    leading 1 + (the character after the longest LCP)."""
    tells_paper = tells_plus1 = False
    for strs in D_CASES.values():
        dist, dist_paper = brute_dist(strs)
        no_plus1 = []
        for i, s in enumerate(strs):
            m = max([len(os.path.commonprefix([s, t])) for j, t in enumerate(strs) if j != i] or [0])
            no_plus1.append(min(len(s), m))
        tells_paper |= sum(dist) != sum(dist_paper)
        tells_plus1 |= sum(dist) != sum(no_plus1)
    assert tells_paper and tells_plus1


# ---- the multi-threaded oracle is the same algorithm ----

@pytest.mark.parametrize("kind", ["prefixes", "suffixes", "identical", "adversarial"])
def test_threads_bit_exact(kind):
    if kind == "prefixes":
        ss = W.prefixes(1 << 18, seed=8, n_prefix=64)
    elif kind == "suffixes":
        ss = W.suffixes(1 << 17, seed=9)
    elif kind == "identical":
        ss = W.from_list([b"same"] * 150000 + [b"samf", b"sam"] * 1000)
    else:
        rng = np.random.default_rng(77)
        ss = W.from_list(adversarial(rng, 3000))
    p1, h1 = oracle.sort(ss, threads=1)
    for t in (2, 5, 8):
        pt, ht = oracle.sort(ss, threads=t)
        assert np.array_equal(p1, pt) and np.array_equal(h1, ht), t
    assert oracle.check(ss, p1, h1) == -1


# ---- Section 5: LCP-insertion sort (Algorithm 5), LCP-merge (Algorithms 2-4) ----

def _lsum(lcp):
    return int(np.asarray(lcp, dtype=np.int64)[1:].sum()) if len(lcp) else 0


@pytest.mark.parametrize("seed", range(16))
def test_lcp_insertion_sort_result_and_bound(seed):
    """Alg. 5 gives the sorted order (stable) and LCP array, within the
    theorem's L + n(n-1)/2 character comparisons."""
    rng = np.random.default_rng(500 + seed)
    strs = adversarial(rng, int(rng.integers(1, 120)))
    if seed % 4 == 0:           # a group with a common prefix hbar > 0
        pre = b"shared-prefix-"
        strs = [pre + s for s in strs]
    ss = W.from_list(strs)
    hbar = len(os.path.commonprefix(strs)) if seed % 4 == 0 else 0
    perm, lcp, cmp = oracle.lcp_insertion_sort(ss, np.arange(len(strs)), hbar)
    rp, rh = brute(strs)
    assert list(perm) == rp and list(lcp) == rh
    n = len(strs)
    assert cmp <= _lsum(lcp) + n * (n - 1) // 2


def test_lcp_insertion_sort_uses_lcps():
    """n long identical-prefix strings: without the LCPs of Alg. 5 every
    comparison would re-read the shared 200 bytes; with them the count stays
    within L + n(n-1)/2, far below n(n-1)/2 * 200."""
    rng = np.random.default_rng(3)
    strs = [b"p" * 200 + bytes(rng.integers(97, 100, size=3).astype(np.uint8)) for _ in range(60)]
    perm, lcp, cmp = oracle.lcp_insertion_sort(W.from_list(strs), np.arange(60), 0)
    assert cmp <= _lsum(lcp) + 60 * 59 // 2
    assert cmp < 60 * 59 // 2 * 50


def _runs(rng, n, K):
    owner = rng.integers(0, K, size=n)
    idx = [np.nonzero(owner == k)[0].astype(np.uint32) for k in range(K)]
    return idx


@pytest.mark.parametrize("K", [1, 2, 3, 4, 7, 8, 16])
@pytest.mark.parametrize("kind", ["adv", "prefixes", "identical"])
def test_kway_lcp_merge_result_and_bound(K, kind):
    """Alg. 4 over sorted runs equals the sort of their union, within the
    theorem's Delta L + n log2 K + K character comparisons."""
    rng = np.random.default_rng(K * 10 + len(kind))
    if kind == "adv":
        strs = adversarial(rng, 1500)
    elif kind == "prefixes":
        strs = W.prefixes(3000, seed=K, n_prefix=8).strings()
    else:
        strs = [b"dup"] * 500 + [b"du", b"dupe"] * 50
    ss = W.from_list(strs)
    pieces, lcps, rb = [], [], [0]
    Lruns = 0
    for idx in _runs(rng, len(strs), K):
        sub = [strs[i] for i in idx]
        p, h = brute(sub)
        pieces.append(idx[p])
        lcps.append(np.array(h, dtype=np.uint32))
        Lruns += sum(h)
        rb.append(rb[-1] + len(idx))
    pin = np.concatenate(pieces) if pieces else np.zeros(0, np.uint32)
    hin = np.concatenate(lcps) if lcps else np.zeros(0, np.uint32)
    perm, lcp, cmp = oracle.lcp_merge(ss, rb, pin, hin)
    rp, rh = brute(strs)
    assert list(perm) == rp and list(lcp) == rh
    KP = 1 << max(0, (K - 1).bit_length())
    n = len(strs)
    dL = _lsum(lcp) - Lruns
    assert cmp <= dL + n * int(math.log2(KP)) + KP


def test_binary_lcp_merge_equals_kway():
    rng = np.random.default_rng(9)
    strs = adversarial(rng, 900)
    ss = W.from_list(strs)
    a, b = _runs(rng, len(strs), 2)
    pa, ha = brute([strs[i] for i in a])
    pb, hb = brute([strs[i] for i in b])
    pin = np.concatenate([a[pa], b[pb]])
    hin = np.array(ha + hb, dtype=np.uint32)
    rb = [0, len(a), len(strs)]
    p2, h2, c2 = oracle.lcp_merge(ss, rb, pin, hin, binary=True)
    pk, hk, ck = oracle.lcp_merge(ss, rb, pin, hin)
    rp, rh = brute(strs)
    assert list(p2) == rp and list(h2) == rh and list(pk) == rp and list(hk) == rh
    n = len(strs)
    assert c2 <= _lsum(h2) - sum(ha) - sum(hb) + n


@pytest.mark.parametrize("K", [2, 4, 8])
def test_lcp_mergesort_bounds(K):
    """Binary LCP-mergesort: at most L + n ceil(log2 n) character
    comparisons; K-way: less than L + n ceil(log_K n) log2 K + n +
    ceil((n-1)/(K-1)) (theorems after Algorithms 3 and 4)."""
    for seed, strs in enumerate([adversarial(np.random.default_rng(40 + K), 2000),
                                 W.prefixes(4000, seed=K, n_prefix=16).strings(),
                                 [b"x" * 30] * 300]):
        ss = W.from_list(strs)
        perm, lcp, cmp = oracle.lcp_mergesort(ss, K)
        rp, rh = brute(strs)
        assert list(perm) == rp and list(lcp) == rh
        n, L = len(strs), _lsum(lcp)
        if K == 2:
            assert cmp <= L + n * math.ceil(math.log2(n))
        else:
            levels = math.ceil(math.log(n, K) - 1e-12)
            assert cmp < L + n * levels * math.log2(K) + n + math.ceil((n - 1) / (K - 1))


def test_merge_sample_ranks_collide_for_an_index_in_two_runs():
    """The merge splits its work by samples (every g-th element of every
    run): a sample's rank is the number of samples below it, counted with its
    cut (lower bound of (string, index)) in every run.  Runs that hold an
    index twice give two samples the same rank, so one rank (cut row) is never
    produced; the device merge must detect that rather than use the row."""
    strs = [b"b", b"a", b"c", b"d"]
    key = lambda i: (strs[i], i)
    runs = [[1, 0, 2], [1, 3]]          # index 1 starts both runs
    g = 2
    samples = [(k, p) for k, r in enumerate(runs) for p in range(0, len(r), g)]

    def lower_bound(run, x):
        lo, hi = 0, len(run)
        while lo < hi:
            mid = (lo + hi) // 2
            if key(run[mid]) < key(x):
                lo = mid + 1
            else:
                hi = mid
        return lo

    ranks = []
    for k, p in samples:
        x = runs[k][p]
        cuts = [p if r == k else lower_bound(runs[r], x) for r in range(len(runs))]
        ranks.append(sum((c + g - 1) // g for c in cuts))
    assert len(samples) == 3
    assert sorted(ranks) == [0, 0, 2]       # rank 1 never produced
    # with distinct indices (run 1 starts with 3 instead) the ranks are 0..nsamp-1
    runs[1] = [3]
    samples = [(k, p) for k, r in enumerate(runs) for p in range(0, len(r), g)]
    ranks = []
    for k, p in samples:
        x = runs[k][p]
        cuts = [p if r == k else lower_bound(runs[r], x) for r in range(len(runs))]
        ranks.append(sum((c + g - 1) // g for c in cuts))
    assert sorted(ranks) == list(range(len(samples)))
