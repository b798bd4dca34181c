"""The allocation-free sort (ssort_sort_noalloc, the library's per-GPU scratch
array as workspace) against ssort_sort with a caller workspace, element by
element, on two calls in a row (the second with a smaller input), plus its
size limit."""
import ctypes

import numpy as np
import pytest

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


def _reference(sorter, d):
    from paper_1403_2056_amd import ssort
    perm, lcp = sorter.sort(d)
    torch.cuda.synchronize()
    assert sorter.query_error() == 0
    return ssort.to_numpy_u32(perm).copy(), ssort.to_numpy_u32(lcp).copy()


def test_noalloc_matches_sort_twice_smaller_second(sorter):
    from paper_1403_2056_amd import ssort
    # first call: above the whole-GPU level threshold; second: a smaller set
    cases = [("long prefixes", W.prefixes(300_000, seed=31, n_prefix=64)),
             ("plain", W.plain(20_000, seed=32))]
    for label, ss in cases:
        print(f"[noalloc] {label} n={ss.n}", flush=True)
        d = ssort.strings_to_device(ss)
        rp, rh = _reference(sorter, d)
        # fill the outputs with a pattern so that an unwritten entry shows
        perm = torch.full((ss.n,), -1, dtype=torch.int32, device="cuda")
        lcp = torch.full((ss.n,), -1, dtype=torch.int32, device="cuda")
        sorter.sort_noalloc(d, perm, lcp)
        torch.cuda.synchronize()
        assert sorter.query_error() == 0, f"device error mask {sorter.stats()['error_bits']:#x}"
        p = ssort.to_numpy_u32(perm)
        h = ssort.to_numpy_u32(lcp)
        assert np.array_equal(p, rp), f"{label}: permutation differs from ssort_sort"
        assert np.array_equal(h, rh), f"{label}: LCP array differs from ssort_sort"


def test_noalloc_permutation_only_and_stream(sorter):
    from paper_1403_2056_amd import ssort
    ss = W.plain(5_000, seed=33)
    d = ssort.strings_to_device(ss)
    rp, _ = _reference(sorter, d)
    perm = torch.full((ss.n,), -1, dtype=torch.int32, device="cuda")
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    sorter.sort_noalloc(d, perm, None, stream=st)
    st.synchronize()
    assert sorter.query_error(st) == 0
    assert np.array_equal(ssort.to_numpy_u32(perm), rp)


def test_noalloc_size_limit_is_a_host_error(sorter):
    from paper_1403_2056_amd import ssort
    L = ssort.lib()
    cap = 64 << 20
    # the largest n whose workspace fits, found with the library's own size query
    lo, hi = 1, 1 << 24
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if sorter.workspace_bytes(mid) <= cap:
            lo = mid
        else:
            hi = mid
    assert lo >= 1 << 20
    # a set one string larger is refused before anything is enqueued (the
    # pointers are never dereferenced: the size check comes first)
    dummy = torch.empty(8, dtype=torch.uint8, device="cuda")
    st = ssort.Strings(dummy.data_ptr(), 8, dummy.data_ptr(), None, hi, 0)
    rc = L.ssort_sort_noalloc(sorter._h, ctypes.byref(st), dummy.data_ptr(), None, None)
    assert rc == ssort.STATUS_CODES["SSORT_EWORKSPACE"]
    rc = L.ssort_sort_noalloc(sorter._h, ctypes.byref(st), None, None, None)
    assert rc in (ssort.STATUS_CODES["SSORT_EINVAL"], ssort.STATUS_CODES["SSORT_EWORKSPACE"])
