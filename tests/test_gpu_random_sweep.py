"""Randomised parity: seeded mixes of the adversarial input kinds, in both
layouts, each sorted with a random tuning (splitter count 1..4095, keys per
thread, base-case threshold, S5-Equal, alphabet compression) and compared with
the oracle element by element (permutation and LCP array)."""
import numpy as np
import pytest

import oracle
from paper_1403_2056_amd import workloads as W
from tests.cases import adversarial

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = 960


@pytest.fixture(scope="module")
def sorters():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return {}


def _sorter(cache, v, k, tb, flags):
    from paper_1403_2056_amd import ssort
    key = (v, k, tb, flags)
    if key not in cache:
        s = ssort.Sorter(0, v=v, keys_per_thread=k, base_threshold=tb, flags=flags)
        s.set_wait_limit(10000)
        cache[key] = s
    return cache[key]


@pytest.mark.parametrize("block", range(4))
def test_random_inputs_and_tunings(sorters, block):
    from paper_1403_2056_amd import ssort
    rng = np.random.default_rng(7100 + block)
    for c in range(CASES // 4):
        strs = []
        for _ in range(int(rng.integers(1, 4))):
            strs += adversarial(rng, int(rng.integers(1, 6000)))
        rng.shuffle(strs)
        layout = "lengths" if rng.random() < 0.3 else "csr"
        ss = W.from_list(strs, layout=layout, pad=int(rng.integers(0, 4)) if layout == "lengths" else 0)
        v = int(rng.choice([1, 3, 7, 63, 127, 255, 255, 1023, 4095]))
        k = int(rng.choice([4, 8]))
        tb = int(rng.choice([16, 64, 128, 256, 1024]))
        flags = ((ssort.SSORT_EQUAL if rng.random() < 0.2 else 0)
                 | (ssort.SSORT_ALPHABET if rng.random() < 0.2 else 0))
        label = f"block {block} case {c}: n={ss.n} {layout} v={v} k={k} tb={tb} flags={flags}"
        print(f"[sweep] {label}", flush=True)
        s = _sorter(sorters, v, k, tb, flags)
        perm, lcp = s.sort(ssort.strings_to_device(ss))
        torch.cuda.synchronize()
        assert s.query_error() == 0, (label, s.stats())
        p, h = ssort.to_numpy_u32(perm), ssort.to_numpy_u32(lcp)
        rp, rh = oracle.sort(ss)
        assert np.array_equal(p, rp), label
        assert np.array_equal(h, rh), label
