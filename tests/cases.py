"""Adversarial string lists shared by the oracle pins and the GPU parity tests
(inputs only: no sorting arithmetic here)."""
import numpy as np


def adversarial(rng, n):
    kind = int(rng.integers(0, 9))
    if kind == 0:       # heavy duplicates over a tiny alphabet
        pool = [bytes(rng.integers(97, 99, size=rng.integers(0, 6)).astype(np.uint8)) for _ in range(5)]
        return [pool[rng.integers(0, 5)] for _ in range(n)]
    if kind == 1:       # keys ending exactly at 8 / 16 bytes, shared prefixes
        base = bytes(rng.integers(65, 91, size=24).astype(np.uint8))
        return [base[: rng.choice([7, 8, 9, 15, 16, 17, 24])] + bytes([rng.integers(65, 68)]) * rng.integers(0, 2)
                for _ in range(n)]
    if kind == 2:       # extreme bytes 0x01 and 0xFF
        return [bytes(rng.choice([1, 2, 254, 255], size=rng.integers(0, 12)).astype(np.uint8)) for _ in range(n)]
    if kind == 3:       # prefix chains
        s = bytes(rng.integers(97, 123, size=40).astype(np.uint8))
        return [s[: rng.integers(0, 41)] for _ in range(n)]
    if kind == 4:       # suffixes of a tiny periodic text
        t = (b"abaab" * 400)[: rng.integers(1, 2000)]
        return [t[i:] for i in range(len(t))][:n]
    if kind == 5:       # empty strings mixed in
        return [b"" if rng.random() < 0.3 else bytes(rng.integers(33, 127, size=rng.integers(1, 30)).astype(np.uint8))
                for _ in range(n)]
    if kind == 6:       # long shared prefix, then few distinct tails
        p = bytes(rng.integers(97, 123, size=int(rng.integers(50, 300))).astype(np.uint8))
        return [p + bytes(rng.integers(97, 100, size=rng.integers(0, 4)).astype(np.uint8)) for _ in range(n)]
    if kind == 7:       # all identical
        s = bytes(rng.integers(97, 123, size=int(rng.integers(0, 30))).astype(np.uint8))
        return [s] * n
    return [bytes(rng.integers(1, 256, size=rng.integers(0, 40)).astype(np.uint8)) for _ in range(n)]
