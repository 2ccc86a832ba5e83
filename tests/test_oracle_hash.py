"""Pins of the oracle's counter-based hash (CPU only).

The workloads' "splitmix32" is read as the golden-ratio increment followed by the
MurmurHash3 32-bit finalizer.  The finalizer is pinned by MurmurHash3's published test
vectors (built here around the oracle's fmix32), the increment by its closed form
floor(2^32 / phi), and fmix32's structure by inverting it with inverse multipliers.
"""

import math
import os

import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")
M = 0xFFFFFFFF


def _rows(name):
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                yield line


def _murmur3_x86_32(data: bytes, seed: int) -> int:
    """MurmurHash3_x86_32 body; its final mixing step is the oracle's fmix32."""
    c1, c2 = 0xCC9E2D51, 0x1B873593

    def rotl(x, r):
        return ((x << r) | (x >> (32 - r))) & M

    h = seed
    nblocks = len(data) // 4
    for i in range(nblocks):
        k = int.from_bytes(data[4 * i:4 * i + 4], "little")
        k = rotl((k * c1) & M, 15)
        h ^= (k * c2) & M
        h = (rotl(h, 13) * 5 + 0xE6546B64) & M
    tail = data[4 * nblocks:]
    k = 0
    for idx in range(len(tail) - 1, -1, -1):
        k = (k << 8) | tail[idx]
    if tail:
        k = rotl((k * c1) & M, 15)
        h ^= (k * c2) & M
    h ^= len(data)
    return oracle.fmix32(h)


def test_fmix32_reproduces_published_murmur3_vectors():
    n = 0
    for line in _rows("murmur3_x86_32_vectors.txt"):
        seed_s, rest = line.split(" ", 1)
        key_s, expect_s = rest.rsplit(" ", 1)
        key = key_s.strip()[1:-1].encode("ascii")
        assert _murmur3_x86_32(key, int(seed_s, 16)) == int(expect_s, 16), line
        n += 1
    assert n >= 8


def test_increment_is_floor_two_pow_32_over_phi():
    phi = (1 + math.sqrt(5)) / 2
    gamma = int(2**32 / phi)
    assert gamma == 0x9E3779B9
    for x in [0, 1, 7, 0xDEADBEEF, 0xFFFFFFFF, 0x61C88647]:
        assert oracle.sm32(x) == oracle.fmix32((x + gamma) & M)


def _inverse_fmix32(h: int) -> int:
    """Undo fmix32 step by step: xorshift-right inverses and multiplicative inverses."""

    def unxorshift(y, s):
        x = y
        for _ in range(32 // s + 1):
            x = y ^ (x >> s)
        return x & M

    inv1 = pow(0x85EBCA6B, -1, 2**32)
    inv2 = pow(0xC2B2AE35, -1, 2**32)
    h = unxorshift(h, 16)
    h = (h * inv2) & M
    h = unxorshift(h, 13)
    h = (h * inv1) & M
    return unxorshift(h, 16)


@pytest.mark.parametrize("x", [0, 1, 2, 3, 0x80000000, 0xFFFFFFFF, 0x12345678, 0xCAFEBABE])
def test_fmix32_is_a_bijection_inverted(x):
    assert _inverse_fmix32(oracle.fmix32(x)) == x


def test_sm32_independent_vectors():
    for line in _rows("sm32_vectors.txt"):
        x, y = (int(v, 16) for v in line.split())
        assert oracle.sm32(x) == y


def test_sm32_no_collisions_on_a_window():
    vals = {oracle.sm32(x) for x in range(1 << 14)}
    assert len(vals) == 1 << 14


def test_chain_vectors_and_composition():
    for line in _rows("chain_vectors.txt"):
        x, L, h = line.split()
        assert oracle.chain(int(x), int(L)) == int(h, 16)
    for x in [0, 42, 0xFFFFFFFF]:
        assert oracle.chain(x, 0) == x
        assert oracle.chain(x, 1) == oracle.sm32(x)
        for a, b in [(3, 5), (100, 1), (0, 17)]:
            assert oracle.chain(x, a + b) == oracle.chain(oracle.chain(x, a), b)


def test_chain_batch_matches_single():
    import numpy as np
    L = np.array([0, 1, 2, 148, 1000, 65536], dtype=np.uint32)
    out = oracle.chain_batch(42, L)
    for r, l in enumerate(L):
        assert out[r] == oracle.chain(42 ^ r, int(l))


def test_key_streams_differ():
    # key(b, j, s) for different streams s and agents b must not coincide systematically
    ks = {oracle.key(42, b, j, s) for b in range(16) for j in range(16) for s in (1, 2, 3)}
    assert len(ks) == 16 * 16 * 3
