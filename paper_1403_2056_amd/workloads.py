"""Seeded synthetic string sets.

This module only draws random strings.  It holds none of the sorting method's
arithmetic, so both the HIP path and the CPU oracle can take their inputs from
it without sharing any code of the method.

Every generator returns a :class:`StringSet` in one of the three layouts the
library accepts:

* ``csr``     ``offsets`` has n+1 entries, string i is chars[offsets[i]:offsets[i+1]];
* ``lengths`` ``offsets`` has n start offsets and ``lengths`` n lengths;
* ``to_end``  ``offsets`` has n start offsets and string i runs to the end of
  ``chars`` (suffixes of one text, no copy).

Workloads (all bytes are non-zero: the paper's alphabet excludes the
terminator, Preliminaries):

* ``plain``     n strings, lengths uniform in [8,32], bytes uniform over
                'a'..'z', then 5 % of the positions replaced by copies of other
                strings (n = 131072 is the small parity case).
* ``prefixes``  n strings, each one of P random prefixes (length 10..60) plus a
                random suffix (length 5..80), both over a 64-symbol alphabet
                0x30..0x6F, then 20 % exact duplicates (n = 2^24, P = 4096 is
                the large single-GPU case).
* ``suffixes``  all suffixes of a {A,C,G,T} text built from 2 KiB blocks; a
                block after the first is, with probability 1/2, a copy of an
                earlier block with 1 % of its bases substituted, else i.i.d.
* ``paper_random`` the paper's "Random" input (Inputs subsection of the
                experiments): length uniform in [0,20), bytes uniform in
                [33,127).
* ``batched``   many independent sets, sizes log-uniform in [2^lo, 2^hi],
                lengths geometric with mean 24 (support >= 1), bytes uniform
                over the 95 printable ASCII bytes 0x20..0x7E.
"""
from __future__ import annotations

import dataclasses
import numpy as np

FLAG_TO_END = 1


@dataclasses.dataclass
class StringSet:
    chars: np.ndarray            # uint8 [nchars]
    offsets: np.ndarray          # uint64 [n+1] (csr) or [n] (lengths / to_end)
    lengths: np.ndarray | None   # uint32 [n] or None
    flags: int                   # FLAG_TO_END or 0
    n: int
    meta: dict

    @property
    def layout(self) -> str:
        if self.flags & FLAG_TO_END:
            return "to_end"
        return "lengths" if self.lengths is not None else "csr"

    def starts(self) -> np.ndarray:
        return self.offsets[: self.n].astype(np.uint64)

    def lens(self) -> np.ndarray:
        if self.flags & FLAG_TO_END:
            return (np.uint64(len(self.chars)) - self.offsets[: self.n]).astype(np.uint64)
        if self.lengths is not None:
            return self.lengths.astype(np.uint64)
        return (self.offsets[1:] - self.offsets[:-1]).astype(np.uint64)

    def string(self, i: int) -> bytes:
        # One string, without building the whole start and length arrays.
        if not 0 <= i < self.n:
            raise IndexError(f"string {i} of {self.n}")
        s = int(self.offsets[i])
        if self.flags & FLAG_TO_END:
            ln = len(self.chars) - s
        elif self.lengths is not None:
            ln = int(self.lengths[i])
        else:
            ln = int(self.offsets[i + 1]) - s
        return bytes(self.chars[s:s + ln])

    def strings(self) -> list[bytes]:
        st = self.starts()
        ln = self.lens()
        mv = self.chars.tobytes()
        return [mv[int(a):int(a) + int(b)] for a, b in zip(st, ln)]

    def total_len(self) -> int:
        return int(self.lens().sum()) if self.n else 0


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def from_list(strs: list[bytes], layout: str = "csr", pad: int = 0) -> StringSet:
    """Pack python byte strings (tests).  ``pad`` adds unused bytes around them."""
    n = len(strs)
    lens = np.array([len(s) for s in strs], dtype=np.uint64)
    body = b"".join(strs)
    chars = np.frombuffer(b"\x7f" * pad + body + b"\x7f" * pad, dtype=np.uint8).copy()
    starts = np.zeros(n, dtype=np.uint64)
    if n:
        starts[1:] = np.cumsum(lens)[:-1]
    starts += np.uint64(pad)
    if layout == "csr":
        if pad:
            raise ValueError("csr layout cannot skip padding between strings")
        off = np.zeros(n + 1, dtype=np.uint64)
        off[1:] = np.cumsum(lens)
        return StringSet(chars, off, None, 0, n, {"workload": "list"})
    if layout == "lengths":
        return StringSet(chars, starts, lens.astype(np.uint32), 0, n, {"workload": "list"})
    raise ValueError(layout)


def _ragged_fill(out: np.ndarray, out_starts: np.ndarray, src: np.ndarray,
                 src_starts: np.ndarray, lens: np.ndarray, chunk: int = 1 << 18) -> None:
    """out[out_starts[i] + k] = src[src_starts[i] + k] for k < lens[i]."""
    n = len(lens)
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        ln = lens[a:b].astype(np.int64)
        tot = int(ln.sum())
        if tot == 0:
            continue
        rep = np.repeat(np.arange(b - a), ln)
        first = np.zeros(b - a, dtype=np.int64)
        first[1:] = np.cumsum(ln)[:-1]
        k = np.arange(tot, dtype=np.int64) - first[rep]
        out[out_starts[a:b].astype(np.int64)[rep] + k] = src[src_starts[a:b].astype(np.int64)[rep] + k]


def _dup_sources(rng: np.random.Generator, n: int, frac: float) -> np.ndarray:
    """Source index per position: itself, or for a `frac` share of positions a
    uniformly drawn other position (the copy takes that string's original text)."""
    src = np.arange(n, dtype=np.int64)
    k = int(round(frac * n))
    if n < 2 or k == 0:
        return src
    pos = rng.choice(n, size=k, replace=False)
    other = rng.integers(0, n - 1, size=k)
    other = other + (other >= pos)          # never itself
    src[pos] = other
    return src


def _assemble(lens: np.ndarray, pool: np.ndarray, pool_starts: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    n = len(lens)
    off = np.zeros(n + 1, dtype=np.uint64)
    off[1:] = np.cumsum(lens.astype(np.uint64))
    chars = np.empty(int(off[-1]), dtype=np.uint8)
    _ragged_fill(chars, off[:-1], pool, pool_starts, lens)
    return chars, off


def plain(n: int = 131072, seed: int = 1, lo: int = 8, hi: int = 32,
          alpha: tuple[int, int] = (ord("a"), ord("z")), dup_frac: float = 0.05) -> StringSet:
    rng = _rng(seed)
    lens = rng.integers(lo, hi + 1, size=n).astype(np.int64)
    pool_starts = np.zeros(n, dtype=np.int64)
    pool_starts[1:] = np.cumsum(lens)[:-1]
    pool = rng.integers(alpha[0], alpha[1] + 1, size=int(lens.sum()), dtype=np.uint8)
    src = _dup_sources(rng, n, dup_frac)
    chars, off = _assemble(lens[src], pool, pool_starts[src])
    return StringSet(chars, off, None, 0, n, {
        "workload": "plain", "n": n, "seed": seed, "len": [lo, hi],
        "alphabet": [alpha[0], alpha[1]], "dup_frac": dup_frac})


def prefixes(n: int = 1 << 24, seed: int = 2, n_prefix: int = 4096,
             plen: tuple[int, int] = (10, 60), slen: tuple[int, int] = (5, 80),
             alpha: tuple[int, int] = (0x30, 0x6F), dup_frac: float = 0.20) -> StringSet:
    rng = _rng(seed)
    pl = rng.integers(plen[0], plen[1] + 1, size=n_prefix).astype(np.int64)
    ptab_start = np.zeros(n_prefix, dtype=np.int64)
    ptab_start[1:] = np.cumsum(pl)[:-1]
    ptab = rng.integers(alpha[0], alpha[1] + 1, size=int(pl.sum()), dtype=np.uint8)
    pid = rng.integers(0, n_prefix, size=n)
    sl = rng.integers(slen[0], slen[1] + 1, size=n).astype(np.int64)
    src = _dup_sources(rng, n, dup_frac)
    pid = pid[src]
    sl_orig = sl
    sfx_start = np.zeros(n, dtype=np.int64)
    sfx_start[1:] = np.cumsum(sl_orig)[:-1]
    sfx_pool = rng.integers(alpha[0], alpha[1] + 1, size=int(sl_orig.sum()), dtype=np.uint8)
    sl = sl_orig[src]
    sfx_start = sfx_start[src]
    plens = pl[pid]
    lens = plens + sl
    off = np.zeros(n + 1, dtype=np.uint64)
    off[1:] = np.cumsum(lens.astype(np.uint64))
    chars = np.empty(int(off[-1]), dtype=np.uint8)
    _ragged_fill(chars, off[:-1], ptab, ptab_start[pid], plens)
    _ragged_fill(chars, off[:-1] + plens.astype(np.uint64), sfx_pool, sfx_start, sl)
    return StringSet(chars, off, None, 0, n, {
        "workload": "prefixes", "n": n, "seed": seed, "n_prefix": n_prefix,
        "prefix_len": list(plen), "suffix_len": list(slen),
        "alphabet": [alpha[0], alpha[1]], "dup_frac": dup_frac})


def suffix_text(nbytes: int = 1 << 22, seed: int = 3, block: int = 2048,
                p_copy: float = 0.5, p_mut: float = 0.01) -> np.ndarray:
    rng = _rng(seed)
    acgt = np.frombuffer(b"ACGT", dtype=np.uint8)
    nb = (nbytes + block - 1) // block
    codes = np.empty(nb * block, dtype=np.uint8)
    codes[:block] = rng.integers(0, 4, size=block)
    for b in range(1, nb):
        seg = codes[b * block:(b + 1) * block]
        if rng.random() < p_copy:
            j = int(rng.integers(0, b))
            seg[:] = codes[j * block:(j + 1) * block]
            mut = rng.random(block) < p_mut
            k = int(mut.sum())
            if k:
                seg[mut] = (seg[mut] + rng.integers(1, 4, size=k)) % 4   # a different base
        else:
            seg[:] = rng.integers(0, 4, size=block)
    return acgt[codes[:nbytes]]


def suffixes(nbytes: int = 1 << 22, seed: int = 3, block: int = 2048,
             p_copy: float = 0.5, p_mut: float = 0.01) -> StringSet:
    text = suffix_text(nbytes, seed, block, p_copy, p_mut)
    off = np.arange(nbytes, dtype=np.uint64)
    return StringSet(text, off, None, FLAG_TO_END, nbytes, {
        "workload": "suffixes", "n": nbytes, "seed": seed, "block": block,
        "p_copy": p_copy, "p_mut": p_mut, "alphabet": "ACGT"})


def paper_random(n: int, seed: int = 4) -> StringSet:
    rng = _rng(seed)
    lens = rng.integers(0, 20, size=n).astype(np.int64)
    off = np.zeros(n + 1, dtype=np.uint64)
    off[1:] = np.cumsum(lens.astype(np.uint64))
    chars = rng.integers(33, 127, size=int(off[-1]), dtype=np.uint8)
    return StringSet(chars, off, None, 0, n, {"workload": "paper_random", "n": n, "seed": seed})


def batched(m: int = 4096, seed: int = 5, lo: int = 6, hi: int = 18,
            mean_len: float = 24.0, alpha: tuple[int, int] = (0x20, 0x7E)):
    """Flattened batch: returns (StringSet over all strings, set_begin[m+1] uint32)."""
    rng = _rng(seed)
    sizes = np.floor(2.0 ** rng.uniform(lo, hi, size=m)).astype(np.int64)
    n = int(sizes.sum())
    lens = rng.geometric(1.0 / mean_len, size=n).astype(np.int64)
    off = np.zeros(n + 1, dtype=np.uint64)
    off[1:] = np.cumsum(lens.astype(np.uint64))
    chars = rng.integers(alpha[0], alpha[1] + 1, size=int(off[-1]), dtype=np.uint8)
    set_begin = np.zeros(m + 1, dtype=np.uint32)
    set_begin[1:] = np.cumsum(sizes).astype(np.uint32)
    return StringSet(chars, off, None, 0, n, {
        "workload": "batched", "sets": m, "seed": seed, "size_log2": [lo, hi],
        "mean_len": mean_len, "alphabet": [alpha[0], alpha[1]]}), set_begin


def mixed_job(rng: np.random.Generator, n: int) -> StringSet:
    """One serving job of n strings from one of the three plain distributions."""
    kind = int(rng.integers(0, 3))
    seed = int(rng.integers(0, 2**31))
    if kind == 0:
        return plain(n, seed)
    if kind == 1:
        return prefixes(n, seed, n_prefix=max(1, -(-n // 4096)))
    return suffixes(max(n, 1), seed)


def by_name(name: str, n: int | None = None, seed: int | None = None) -> StringSet:
    kw = {}
    if seed is not None:
        kw["seed"] = seed
    if name == "plain":
        return plain(n or 131072, **kw)
    if name == "prefixes":
        if n is None:
            return prefixes(**kw)
        # keep 4096 strings per prefix group when scaled down
        return prefixes(n, n_prefix=max(1, n // 4096), **kw)
    if name == "suffixes":
        return suffixes(n or (1 << 22), **kw)
    if name == "paper_random":
        return paper_random(n or (1 << 20), **kw)
    raise ValueError(name)
