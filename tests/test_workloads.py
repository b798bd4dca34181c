"""Shape checks of the seeded synthetic inputs (no method arithmetic here)."""
import numpy as np
import pytest

from paper_1403_2056_amd import workloads as W


def test_plain_shape():
    ss = W.plain(20000, seed=1)
    ln = ss.lens()
    assert ss.n == 20000 and ln.min() >= 8 and ln.max() <= 32
    assert ss.chars.min() >= ord("a") and ss.chars.max() <= ord("z")
    strs = ss.strings()
    assert len(set(strs)) <= 20000 - 900          # about 5 % copies
    again = W.plain(20000, seed=1)
    assert np.array_equal(again.chars, ss.chars) and np.array_equal(again.offsets, ss.offsets)


def test_prefixes_shape():
    ss = W.prefixes(50000, seed=2, n_prefix=16)
    ln = ss.lens()
    assert ln.min() >= 15 and ln.max() <= 140
    assert ss.chars.min() >= 0x30 and ss.chars.max() <= 0x6F
    strs = ss.strings()
    assert len({s[:10] for s in strs}) <= 16
    assert len(set(strs)) <= 50000 - 7000          # about 20 % copies


def test_suffixes_shape():
    ss = W.suffixes(1 << 14, seed=3, block=512)
    assert ss.flags == W.FLAG_TO_END and ss.n == 1 << 14
    assert set(np.unique(ss.chars)) <= set(b"ACGT")
    assert int(ss.lens()[0]) == 1 << 14 and int(ss.lens()[-1]) == 1


def test_batched_shape():
    ss, sb = W.batched(m=64, seed=5, lo=6, hi=10)
    sizes = np.diff(sb.astype(np.int64))
    assert sizes.min() >= 64 and sizes.max() <= 1024 and int(sb[-1]) == ss.n
    assert ss.lens().min() >= 1
    assert ss.chars.min() >= 0x20 and ss.chars.max() <= 0x7E


def test_string_accessor_matches_strings():
    # string(i) reads one string directly; it must agree with strings() on
    # every layout, including empty strings and the suffix layout.
    sets = [
        W.from_list([b"ab", b"", b"abc", b"z"], "csr"),
        W.from_list([b"ab", b"", b"abc", b"z"], "lengths", pad=3),
        W.plain(500, seed=7),
        W.suffixes(1 << 10, seed=3, block=256),
    ]
    for ss in sets:
        strs = ss.strings()
        assert [ss.string(i) for i in range(ss.n)] == strs
        for bad in (-1, ss.n):
            with pytest.raises(IndexError):
                ss.string(bad)
