"""Pins of the oracle's closed forms (CPU only).

Each closed form is checked against something other than itself: independently computed
vectors, special cases with a known value, conservation laws and permutation invariants,
brute force on tiny inputs, and the threaded reference (which reaches the same numbers
through real atomics and real waits).
"""

import functools
import os

import numpy as np
import pytest

import oracle
import sp_inputs

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                yield line.split()


# ---- barrier hash exchange ------------------------------------------------------------

def test_barrier_independent_vectors():
    for row in _rows("barrier_hash_vectors.txt"):
        seed, N, R = (int(v) for v in row[:3])
        expect = [int(v, 16) for v in row[3:]]
        got = oracle.barrier_closed(seed, max(N, len(expect)), R)
        assert [int(x) for x in got[:len(expect)]] == expect


@pytest.mark.parametrize("seed", sp_inputs.SEEDS)
def test_barrier_one_round_reads_own_slot(seed):
    # round 0 reads slot (b + 0) mod N = b
    got = oracle.barrier_closed(seed, 37, 1)
    assert [int(x) for x in got] == [oracle.sm32(seed ^ (b << 16)) for b in range(37)]


@pytest.mark.parametrize("N,R", [(16, 1000), (5, 13), (256, 40), (1, 9)])
def test_barrier_xor_of_all_checksums_is_order_free(N, R):
    # For each round, b -> (b + r) mod N is a permutation, so the XOR over all agents of
    # the checksums equals the XOR of every published value.
    seed = 0xC0FFEE
    got = oracle.barrier_closed(seed, N, R)
    total = functools.reduce(lambda a, b: a ^ b, (int(x) for x in got), 0)
    expect = 0
    for b in range(N):
        for r in range(R):
            expect ^= oracle.sm32(seed ^ (b << 16) ^ r)
    assert total == expect


def test_barrier_full_rotation_period():
    # After N rounds every agent has read every agent's slot once per residue class:
    # with R = N, agent b reads agent (b + r) mod N in round r.
    seed, N = 7, 8
    got = oracle.barrier_closed(seed, N, N)
    for b in range(N):
        c = 0
        for s in range(N):  # source agent s is read in round (s - b) mod N
            r = (s - b) % N
            c ^= oracle.sm32(seed ^ (s << 16) ^ r)
        assert int(got[b]) == c


# ---- operation split -----------------------------------------------------------------

@pytest.mark.parametrize("nwg,total", [(1, 10), (3, 10), (2048, 1 << 20), (1000, 1 << 20), (7, 0)])
def test_ops_split_sums_to_total(nwg, total):
    parts = [oracle.ops_for_agent(nwg, total, b) for b in range(nwg)]
    assert sum(parts) == total
    assert max(parts) - min(parts) <= 1
    assert parts == sorted(parts, reverse=True)


# ---- mutex ---------------------------------------------------------------------------

@pytest.mark.parametrize("nwg", [1, 7, 64, 2048])
def test_mutex_single_lock_counts_every_acquisition(nwg):
    total = 1 << 14
    words = oracle.mutex_closed(42, nwg, total, 1, 3)
    assert (words == total).all()


@pytest.mark.parametrize("L,W", [(16, 1), (256, 16), (3, 5)])
def test_mutex_counts_sum_to_total_and_columns_agree(L, W):
    total = 1 << 16
    words = oracle.mutex_closed(0xC0FFEE, 64, total, L, W)
    assert int(words[:, 0].astype(np.int64).sum()) == total
    assert (words == words[:, :1]).all()
    # 2^16 uniform draws over L locks: every lock is hit and none is far off
    mean = total / L
    assert words[:, 0].min() > 0.7 * mean and words[:, 0].max() < 1.3 * mean


def test_mutex_brute_force_tiny():
    seed, nwg, total, L, W = 9, 3, 11, 4, 2
    expect = np.zeros((L, W), dtype=np.uint32)
    b_ops = [total // nwg + (1 if b < total % nwg else 0) for b in range(nwg)]
    for b in range(nwg):
        for j in range(b_ops[b]):
            expect[oracle.key(seed, b, j, 1) % L, :] += 1
    assert (oracle.mutex_closed(seed, nwg, total, L, W) == expect).all()


# ---- semaphore -----------------------------------------------------------------------

def test_sem_single_agent_checksum():
    seed, A = 7, 100
    c = 0
    for j in range(A):
        c ^= oracle.sm32(seed ^ j)
    assert int(oracle.sem_closed(seed, 1, A)[0]) == c


def test_sem_closed_hand_assembled_vectors():
    """Several workgroups and a ragged split: pins the per-workgroup (b << 16) term and the
    operation index j of the checksum against values assembled by hand from pinned hashes."""
    rows = [r for r in _rows("workload_vectors.txt") if r[0] == "sem"]
    assert len(rows) >= 2
    for row in rows:
        seed, nwg, total = int(row[1]), int(row[2]), int(row[3])
        expect = [int(v, 16) for v in row[4:]]
        assert [int(x) for x in oracle.sem_closed(seed, nwg, total)] == expect


def test_bounded_buffer_closed_hand_assembled_vectors():
    rows = [r for r in _rows("workload_vectors.txt") if r[0] == "bb"]
    assert len(rows) >= 2
    for row in rows:
        seed, producers, items = int(row[1]), int(row[2]), int(row[3])
        assert oracle.bb_closed(seed, producers, items) == (int(row[4], 16), int(row[5], 16))


def test_key_hand_assembled_vectors():
    """key chains three splitmix32 calls; each vector's inputs cancel the previous hash so
    that every stage lands on a pinned splitmix32 value (and a swap of b and j, or of the
    seed and the stream, would not)."""
    rows = [r for r in _rows("workload_vectors.txt") if r[0] == "key"]
    assert len(rows) >= 3
    for row in rows:
        seed, b, j, s = int(row[1]), int(row[2], 16), int(row[3], 16), int(row[4])
        assert oracle.key(seed, b, j, s) == int(row[5], 16)
        if b != j:
            assert oracle.key(seed, j, b, s) != int(row[5], 16)


# ---- microbenchmarks -----------------------------------------------------------------

@pytest.mark.parametrize("U,n,T", [(1, 1, 1), (5, 3, 7), (64, 100, 32), (8, 1000, 1024), (3, 5, 1)])
def test_bench_counts_brute_force(U, n, T):
    perm = sp_inputs.permutation(T, 42)
    counts = oracle.bench_counts(U, n, perm)
    expect = np.zeros(T, dtype=np.uint64)
    for u in range(U):
        for i in range(n):
            expect[perm[(u + i) % T]] += 1
    assert (counts == expect).all()
    assert int(counts.sum()) == U * n
    inv = np.argsort(perm)
    for t in range(T):
        assert oracle.bench_count_one(U, n, T, int(inv[t])) == int(counts[t])


@pytest.mark.parametrize("a,c", [(0, 0), (0, 1), (0, 10), (5, 7), (0xFFFFFFF0, 100),
                                  (0xFFFFFFFF, 3), (123, 70000)])
def test_sum_increments_brute_force(a, c):
    assert oracle.sum_increments(a, c) == sum((a + k) % 2**32 for k in range(c)) % 2**64


def test_sum_increments_full_wrap():
    # a full 2^32 cycle returns every 32-bit value exactly once
    assert oracle.sum_increments(12345, 2**32) == (2**32 * (2**32 - 1) // 2) % 2**64
    assert oracle.sum_increments(0, 2**33 + 5) == (2 * (2**32 * (2**32 - 1) // 2) + 10) % 2**64


def test_bench_add_closed_from_counts():
    perm = sp_inputs.permutation(32, 7)
    U, n = 96, 50
    finals, s = oracle.bench_closed("add", 7, U, n, perm)
    counts = oracle.bench_counts(U, n, perm)
    assert (finals == counts.astype(np.uint32)).all()
    assert s == sum(c * (c - 1) // 2 for c in map(int, counts)) % 2**64


def test_bench_store_load_closed():
    T, U, n, seed = 64, 10, 3, 42  # 30 ops touch at most 30 of 64 words
    perm = sp_inputs.permutation(T, seed)
    counts = oracle.bench_counts(U, n, perm)
    finals, _ = oracle.bench_closed("st", seed, U, n, perm)
    for t in range(T):
        assert int(finals[t]) == (oracle.prefill(seed, t) if counts[t] else 0)
    finals, s = oracle.bench_closed("ld", seed, U, n, perm)
    assert s == sum(int(counts[t]) * oracle.prefill(seed, t) for t in range(T))


# ---- closed forms against the threaded reference -------------------------------------

@pytest.mark.parametrize("op", ["add", "cas", "ld", "st"])
@pytest.mark.parametrize("T", [1, 32, 1000])
def test_bench_closed_matches_threaded(op, T):
    perm = sp_inputs.permutation(T, 0xC0FFEE)
    U, n = 64, 300
    finals, s = oracle.bench_closed(op, 0xC0FFEE, U, n, perm)
    tf, ts, _ = oracle.bench_threaded(op, 0xC0FFEE, U, n, perm, threads=8)
    assert (finals == tf).all()
    if op != "st":
        assert s == ts


@pytest.mark.parametrize("T", [1, 32, 1000])
def test_bench_exch_conservation_threaded(T):
    perm = sp_inputs.permutation(T, 42)
    U, n = 64, 300
    _, conserved = oracle.bench_closed("exch", 42, U, n, perm)
    tf, returned_plus_final, _ = oracle.bench_threaded("exch", 42, U, n, perm, threads=8)
    assert returned_plus_final == conserved
    written = {oracle.exch_value(42, u, i) for u in range(U) for i in range(n)}
    for t in range(T):
        if int(tf[t]) != oracle.prefill(42, t):
            assert int(tf[t]) in written


@pytest.mark.parametrize("T", [1, 32, 1000])
def test_exchange_finals_validity(T):
    """Threaded exchanges leave every word at its initial value or at a value written to
    it; a planted foreign value is caught."""
    perm = sp_inputs.permutation(T, 42)
    U, n = 64, 300
    tf, _, _ = oracle.bench_threaded("exch", 42, U, n, perm, threads=8)
    assert oracle.exch_finals_invalid(42, U, n, perm, tf) == 0
    bad = tf.copy()
    bad[0] ^= 0x5A5A5A5A
    assert oracle.exch_finals_invalid(42, U, n, perm, bad) == 1
    # untouched words must keep their initial value
    assert oracle.exch_finals_invalid(42, 1, 1, perm, np.array(
        [oracle.prefill(42, t) for t in range(T)], dtype=np.uint32)) == 0


def test_bounded_buffer_values_match_the_closed_form():
    v = oracle.bb_values(3, 5, 1001)
    x = 0
    for a in map(int, v):
        x ^= a
    assert (x, int(v.astype(np.uint64).sum())) == oracle.bb_closed(3, 5, 1001)
    rows = [r for r in _rows("workload_vectors.txt") if r[0] == "bb"]
    v = oracle.bb_values(0, 2, 3)
    assert sorted(map(int, v)) == sorted([0x92ca2f0e, 0x96a0f96b, 0x5032e8f1])
