"""Full-size parity in the configuration bench.py times: the 2^24-string
long-shared-prefix input (checked exactly by the oracle's O(L+n) checker,
which fixes order and LCP uniquely, plus sampled positions compared with
byte-wise comparisons) and all 2^22 suffixes of the 4 MiB text (element by
element against the oracle's full sort)."""
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
    s = ssort.Sorter(0)          # the tuning bench.py uses
    s.set_wait_limit(20000)
    return s


def run(sorter, ss):
    from paper_1403_2056_amd import ssort
    d = ssort.strings_to_device(ss)
    perm, lcp = sorter.sort(d)
    torch.cuda.synchronize()
    assert sorter.query_error() == 0, sorter.stats()
    return ssort.to_numpy_u32(perm).copy(), ssort.to_numpy_u32(lcp).copy()


def test_prefixes_full_size(sorter):
    print("[fullsize] prefixes n=2^24", flush=True)
    ss = W.prefixes()
    p, h = run(sorter, ss)
    assert oracle.check(ss, p, h) == -1
    rng = np.random.default_rng(0)
    strs_at = lambda i: ss.string(int(i))
    for i in rng.integers(1, ss.n, size=2000):
        a, b = strs_at(p[i - 1]), strs_at(p[i])
        assert (a, p[i - 1]) < (b, p[i])
        k = 0
        while k < min(len(a), len(b)) and a[k] == b[k]:
            k += 1
        assert h[i] == k


def test_suffixes_full_size(sorter):
    print("[fullsize] suffixes n=2^22", flush=True)
    ss = W.suffixes()
    p, h = run(sorter, ss)
    rp, rh = oracle.sort(ss)
    assert np.array_equal(p, rp)
    assert np.array_equal(h, rh)
