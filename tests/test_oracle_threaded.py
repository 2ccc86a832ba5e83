"""The threaded reference (one std::thread per agent, real atomics and waits) must reach
the closed forms and hold each primitive's invariant (CPU only)."""

import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("kind", ["central", "split", "tree", "flag", "xcd"])
@pytest.mark.parametrize("N,R", [(1, 20), (2, 50), (5, 40), (16, 200), (64, 20)])
def test_barrier_threaded_matches_closed(kind, N, R):
    seed = 42
    chk, rc, _ = oracle.barrier_threaded(kind, seed, N, R, groups=3)
    assert rc == 0
    assert (chk == oracle.barrier_closed(seed, N, R)).all()


@pytest.mark.parametrize("kind", ["tree", "xcd"])
@pytest.mark.parametrize("groups", [1, 2, 8, 100])
def test_barrier_hierarchical_any_grouping(kind, groups):
    chk, rc, _ = oracle.barrier_threaded(kind, 7, 24, 30, groups=groups)
    assert rc == 0 and (chk == oracle.barrier_closed(7, 24, 30)).all()


def test_barrier_per_xcd_protocol_at_full_grid():
    """The per-XCD flag protocol with 2048 agents in 8 groups of 4 CUs each (256 members
    per group, 64 agents per CU), as on the GPU's largest co-resident grid."""
    chk, rc, _ = oracle.barrier_threaded("xcd", 42, 2048, 20, groups=8)
    assert rc == 0 and (chk == oracle.barrier_closed(42, 2048, 20)).all()


@pytest.mark.parametrize("kind", ["spin_cas", "spin_exch", "spin_backoff", "ticket", "sleep",
                                  "ring", "array", "adaptive", "cohort", "mcs", "cu_cohort"])
@pytest.mark.parametrize("L,W", [(1, 1), (1, 16), (3, 4)])
def test_mutex_threaded_matches_closed(kind, L, W):
    seed, nwg, total = 0xC0FFEE, 8, 3000
    words, rc, _ = oracle.mutex_threaded(kind, seed, nwg, total, L, W)
    assert rc == 0
    assert (words == oracle.mutex_closed(seed, nwg, total, L, W)).all()


@pytest.mark.parametrize("L", [1, 2])
def test_cohort_mutex_threaded_with_local_passes(L):
    """32 agents in 8 cohorts of 4: local hand-overs happen; counts stay exact and no two
    agents are ever inside together (the owner check)."""
    seed, nwg, total = 11, 32, 6400
    words, rc, _ = oracle.mutex_threaded("cohort", seed, nwg, total, L, 8)
    assert rc == 0
    assert (words == oracle.mutex_closed(seed, nwg, total, L, 8)).all()


@pytest.mark.parametrize("L", [1, 2])
def test_cu_cohort_mutex_threaded_with_cu_passes(L):
    """128 agents, four in each CU group of each of the 8 cohorts: hand-overs within a group
    (keeping the cohort lock), within a cohort and across cohorts all happen; counts stay
    exact and no two agents are ever inside together (the owner check)."""
    seed, nwg, total = 13, 128, 12800
    words, rc, _ = oracle.mutex_threaded("cu_cohort", seed, nwg, total, L, 8)
    assert rc == 0
    assert (words == oracle.mutex_closed(seed, nwg, total, L, 8)).all()


@pytest.mark.parametrize("kind", ["spin", "spin_backoff", "spin_backoff_wait_only", "ticket",
                                  "sleep", "counters", "adaptive", "cohort", "array",
                                  "chain"])
@pytest.mark.parametrize("K", [1, 2, 4, 32])
def test_sem_threaded_invariants(kind, K):
    seed, nwg, total = 7, 12, 2400
    r = oracle.sem_threaded(kind, K, seed, nwg, total)
    assert r["rc"] == 0
    assert 1 <= r["maxocc"] <= K
    assert (r["chk"] == oracle.sem_closed(seed, nwg, total)).all()
    s_or_count, ticket, turn, admissions = r["state"]
    assert admissions == total
    if kind.startswith("spin"):
        assert s_or_count == K + 1
    elif kind in ("counters", "adaptive", "array", "chain"):
        assert s_or_count == 0 and ticket == turn == total  # every wait drew, every post counted
    else:
        assert s_or_count == 0 and ticket == turn
        if K >= nwg:
            assert ticket == 0  # nobody ever queues


@pytest.mark.parametrize("K", [1, 32])
def test_spin_semaphore_posts_do_not_starve_at_2048_agents(K):
    """Algorithm 4 with 2048 agents: with backoff in wait only (Section 5's prose) every
    pair completes, and a post fails far less often per pair than a wait does -- posts are
    not starved by the waiters' exchanges on the one word S."""
    seed, nwg, total = 42, 2048, 1 << 13
    r = oracle.sem_threaded("spin_backoff_wait_only", K, seed, nwg, total, imin=1, imax=64)
    assert r["rc"] == 0 and r["maxocc"] <= K
    assert (r["chk"] == oracle.sem_closed(seed, nwg, total)).all()
    s, wait_fails, post_fails, admissions = r["state"]
    assert s == K + 1 and admissions == total
    assert post_fails <= max(wait_fails, 1)


@pytest.mark.parametrize("K", [1, 4, 32, 256])
def test_cohort_semaphore_at_2048_agents(K):
    """Algorithm 5's count with a queue per group: every pair completes, the bound holds,
    every local ticket is served and every grant slot taken (rc -3 otherwise)."""
    seed, nwg, total = 0xC0FFEE, 2048, 1 << 14
    r = oracle.sem_threaded("cohort", K, seed, nwg, total)
    assert r["rc"] == 0 and 1 <= r["maxocc"] <= K
    assert (r["chk"] == oracle.sem_closed(seed, nwg, total)).all()
    assert r["state"] == (0, 0, 0, total)


@pytest.mark.parametrize("K", [1, 4, 32, 256])
def test_array_semaphore_at_2048_agents(K):
    """Two counters with 16 grant slots shared by 2^14 tickets: every pair completes, the
    bound holds, every wait drew a ticket and every post counted."""
    seed, nwg, total = 0xA77A, 2048, 1 << 14
    r = oracle.sem_threaded("array", K, seed, nwg, total)
    assert r["rc"] == 0 and 1 <= r["maxocc"] <= K
    assert (r["chk"] == oracle.sem_closed(seed, nwg, total)).all()
    assert r["state"] == (0, total, total, total)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("K", [1, 3, 32, 256])
def test_chain_semaphore_at_2048_agents(K):
    """K chains over K x max(1, 16 / K) slots (K = 3: 15 slots), each waiter waiting for
    exactly its own ticket's value: a store from another chain or a later ticket of the
    same slot would leave it waiting (the timeout would fire)."""
    seed, nwg, total = 0xC4A1, 2048, 1 << 14
    r = oracle.sem_threaded("chain", K, seed, nwg, total)
    assert r["rc"] == 0 and 1 <= r["maxocc"] <= K
    assert (r["chk"] == oracle.sem_closed(seed, nwg, total)).all()
    assert r["state"] == (0, total, total, total)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("K", [8, 13, 32, 256])
def test_xcd_chain_semaphore_at_2048_agents(K):
    """Chains per group of agents (8 groups, K = 13: five groups of 2 units, three of 1):
    exact-value waits, bound, checksums and counters."""
    seed, nwg, total = 0x8C4A, 2048, 1 << 14
    r = oracle.sem_threaded("xcd_chain", K, seed, nwg, total)
    assert r["rc"] == 0 and 1 <= r["maxocc"] <= K
    assert (r["chk"] == oracle.sem_closed(seed, nwg, total)).all()
    assert r["state"] == (0, total, total, total)


def test_xcd_chain_semaphore_needs_a_unit_per_group():
    assert oracle.sem_threaded("xcd_chain", 7, 1, 16, 64)["rc"] == -1


def test_hardware_threads_reported():
    assert oracle.hardware_threads() >= 1


@pytest.mark.parametrize("K,agents,lmax", [(16384, 64, 65536), (64, 32, 1024), (1, 8, 16)])
def test_serve_threaded_matches_closed(K, agents, lmax):
    """The threaded serving queue reproduces the closed-form chain of every request and
    never holds more than K units; with K = 1 the admission is a mutex."""
    import sp_inputs
    seed = 42
    reqs = sp_inputs.request_table(3000, 1e5, seed, lmax=lmax)
    unit = 65536 if K > 1 else 1 << 40
    units = ((reqs["nbytes"] + np.uint64(unit - 1)) // np.uint64(unit)).astype(np.uint32)
    if K == 1:
        units[:] = 1
    r = oracle.serve_threaded(seed, reqs["L"], units, K, agents)
    assert r["rc"] == 0
    assert (r["out"] == oracle.chain_batch(seed, reqs["L"])).all()
    assert r["issued"] == r["released"] == int(units.sum())
    assert int(units.max()) <= r["maxuse"] <= K


def test_serve_threaded_rejects_oversized_request():
    r = oracle.serve_threaded(1, np.array([5], np.uint32), np.array([3], np.uint32), 2, 4)
    assert r["rc"] == -1


@pytest.mark.parametrize("P,C,items,cap", [(1, 1, 500, 1), (4, 3, 3000, 2), (3, 5, 2001, 16),
                                           (8, 8, 4096, 1024)])
def test_bounded_buffer_threaded_matches_closed(P, C, items, cap):
    """std::mutex + std::condition_variable producers and consumers take exactly what
    was put: the xor and sum of everything taken equal the closed form."""
    r = oracle.bb_threaded(7, P, C, items, cap)
    assert r["rc"] == 0
    assert (r["xor"], r["sum"]) == oracle.bb_closed(7, P, items)
    assert r["taken"] == r["put"] == items and r["left"] == 0
    assert 1 <= r["max_count"] <= cap


def test_bounded_buffer_closed_brute_force():
    seed, P, items = 0xC0FFEE, 3, 10
    x, s = 0, 0
    for w in range(P):
        for j in range(oracle.ops_for_agent(P, items, w)):
            v = oracle.sm32(seed ^ (w << 16) ^ j)
            x ^= v
            s += v
    assert oracle.bb_closed(seed, P, items) == (x, s)
