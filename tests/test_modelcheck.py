"""Exhaustive-interleaving checks of every algorithm on tiny instances, and mutation
tests that pin the checker itself: each planted mistake must be caught (CPU only)."""

import pytest

from oracle.modelcheck import (ArraySemModel, BarrierModel, CohortLockModel, CohortSemModel,
                               CondModel, CuCohortLockModel, FASemModel, MCSLockModel, MutexModel,
                               QueueLockModel, SpinSemModel, WeightedSemModel,
                               XcdBarrierModel, XcdChainSemModel, explore)


@pytest.mark.parametrize("kind", ["spin_cas", "spin_exch", "ticket", "sleep"])
@pytest.mark.parametrize("n,ops", [(2, 2), (3, 2), (3, 3)])
def test_mutex_correct(kind, n, ops):
    r = explore(MutexModel(kind, n, ops))
    assert r.ok, r.violation


@pytest.mark.parametrize("K", [1, 2])
@pytest.mark.parametrize("n,ops", [(3, 2), (3, 3)])
def test_spin_semaphore_correct(K, n, ops):
    r = explore(SpinSemModel(K, n, ops))
    assert r.ok, r.violation


@pytest.mark.parametrize("K", [1, 2, 3, 4])
@pytest.mark.parametrize("n,ops", [(3, 2), (3, 3)])
def test_fa_semaphore_correct(K, n, ops):
    r = explore(FASemModel(K, n, ops))
    assert r.ok, r.violation


@pytest.mark.parametrize("kind", ["central", "split", "tree", "flag"])
@pytest.mark.parametrize("n,rounds,groups", [(2, 3, 2), (3, 3, 2), (4, 3, 2), (3, 4, 3)])
def test_barrier_correct(kind, n, rounds, groups):
    r = explore(BarrierModel(kind, n, rounds, groups))
    assert r.ok, r.violation


# ---- mutation tests ------------------------------------------------------------------

def test_catches_check_then_set_lock():
    r = explore(MutexModel("sleep", 2, 1, mutant="check_then_set"))
    assert r.violation and "mutual exclusion" in r.violation


def test_catches_missing_unlock_as_deadlock():
    r = explore(MutexModel("spin_cas", 2, 1, mutant="skip_release"))
    assert r.deadlock


def test_catches_geq_comparator_in_fa_semaphore():
    # Waiters proceeding once turn >= their 0-based ticket admit K + 1 agents.
    r = explore(FASemModel(1, 2, 1, mutant="geq"))
    assert r.violation and "occupancy" in r.violation


def test_catches_unconditional_turn_bump():
    r = explore(FASemModel(2, 3, 2, mutant="always_bump"))
    assert r.violation is not None


def test_catches_spin_semaphore_off_by_one():
    r = explore(SpinSemModel(1, 3, 1, mutant="enter_at_one"))
    assert r.violation and "occupancy" in r.violation


@pytest.mark.parametrize("kind", ["central", "split", "tree", "flag"])
def test_catches_single_buffered_exchange(kind):
    r = explore(BarrierModel(kind, 2, 3, 2, mutant="single_buffer"))
    assert r.violation and "phase" in r.violation


@pytest.mark.parametrize("kind", ["central", "split", "flag"])
def test_catches_barrier_that_does_not_wait(kind):
    r = explore(BarrierModel(kind, 2, 2, mutant="no_wait"))
    assert r.violation and "phase" in r.violation


def test_catches_hierarchical_group_released_early():
    r = explore(BarrierModel("tree", 4, 2, 2, mutant="no_top_wait"))
    assert r.violation and "phase" in r.violation


def test_catches_split_barrier_published_one_arrival_early():
    r = explore(BarrierModel("split", 3, 3, mutant="split_off_by_one"))
    assert r.violation and "phase" in r.violation


# ---- weighted fetch-and-add semaphore (serving-queue admission) ---------------------

@pytest.mark.parametrize("K,weights,ops", [(1, (1, 1, 1), 2), (2, (1, 2, 2), 2),
                                           (3, (1, 2, 3), 2), (4, (3, 2, 2), 2),
                                           (5, (5, 1), 3)])
def test_weighted_semaphore_correct(K, weights, ops):
    r = explore(WeightedSemModel(K, weights, ops))
    assert r.ok, r.violation


def test_weighted_semaphore_reduces_to_algorithm5_bound():
    # unit weights: at most K inside, exactly like the fetch-and-add semaphore
    r = explore(WeightedSemModel(2, (1, 1, 1), 3))
    assert r.ok


def test_catches_weight_ignored_at_admission():
    r = explore(WeightedSemModel(3, (2, 2, 1), 2, mutant="ignore_weight"))
    assert r.violation and "units in use" in r.violation


def test_catches_strict_admission_deadlock():
    r = explore(WeightedSemModel(2, (2, 1), 1, mutant="strict"))
    assert r.deadlock


def test_catches_partial_return():
    r = explore(WeightedSemModel(3, (2, 2), 2, mutant="post_one"))
    assert not r.ok


# ---- queue mutexes -----------------------------------------------------------------------

@pytest.mark.parametrize("kind", ["ring", "array"])
@pytest.mark.parametrize("n,ops", [(2, 2), (3, 2), (3, 3)])
def test_queue_locks_correct(kind, n, ops):
    r = explore(QueueLockModel(kind, n, ops))
    assert r.ok, r.violation


@pytest.mark.parametrize("Q", [1, 2])
def test_array_lock_needs_no_slot_per_contender(Q):
    # a grant is overwritten only after its owner entered and left, so any Q works; Q
    # only spreads the polling over lines
    r = explore(QueueLockModel("array", 3, 2, Q=Q))
    assert r.ok, r.violation


def test_catches_ring_smaller_than_contenders():
    r = explore(QueueLockModel("ring", 3, 2, mutant="small_ring"))
    assert not r.ok


def test_catches_ring_without_own_id():
    r = explore(QueueLockModel("ring", 2, 1, mutant="skip_write"))
    assert r.deadlock


def test_catches_array_granting_itself():
    r = explore(QueueLockModel("array", 2, 2, mutant="grant_self"))
    assert not r.ok


# ---- condition variables (bounded buffer) ---------------------------------------------

@pytest.mark.parametrize("P,Cn,items,C", [(1, 1, 3, 1), (1, 2, 2, 1), (2, 1, 2, 1),
                                          (2, 2, 1, 1), (1, 2, 3, 2)])
def test_condition_variables_correct(P, Cn, items, C):
    r = explore(CondModel(P, Cn, items, C))
    assert r.ok, r.violation


def test_catches_lost_wakeup():
    r = explore(CondModel(1, 1, 2, 1, mutant="late_register"))
    assert r.deadlock


def test_catches_predicate_not_rechecked():
    r = explore(CondModel(1, 2, 2, 1, mutant="if_not_while"))
    assert r.violation is not None


def test_catches_missing_signal():
    r = explore(CondModel(1, 1, 2, 1, mutant="no_signal"))
    assert r.deadlock


@pytest.mark.parametrize("n,ops,B", [(4, 1, 2), (3, 2, 2), (3, 1, 3), (3, 2, 3)])
def test_cohort_lock_correct(n, ops, B):
    """Mutual exclusion, every acquisition completes, and the global and local locks end
    released, on all interleavings (two cohorts)."""
    r = explore(CohortLockModel(n, ops, C=2, B=B))
    assert r.ok, r.violation


@pytest.mark.slow
def test_cohort_lock_correct_two_per_cohort_twice():
    r = explore(CohortLockModel(4, 2, C=2, B=2))
    assert r.ok and r.states > 5 * 10 ** 5, (r.states, r.violation)


@pytest.mark.parametrize("mutant,n,ops,B", [("skip_global_wait", 4, 1, 2), ("keep_session", 3, 2, 3),
                                            ("no_waiter_check", 3, 1, 3)])
def test_cohort_lock_mutants_fail(mutant, n, ops, B):
    r = explore(CohortLockModel(n, ops, C=2, B=B, mutant=mutant))
    assert not r.ok


@pytest.mark.parametrize("n,ops,C,B", [(3, 2, 1, 3), (3, 3, 1, 2), (3, 2, 2, 2)])
def test_cohort_lock_grant_slots_shared(n, ops, C, B):
    """Two grant slots per cohort: local tickets t and t + 2 share a slot, and the grant
    for t + 2 is written only after t has entered -- the lock stays correct."""
    r = explore(CohortLockModel(n, ops, C=C, B=B, G=2))
    assert r.ok, r.violation


def test_cohort_lock_grant_into_own_slot_deadlocks():
    r = explore(CohortLockModel(3, 2, C=1, B=3, mutant="own_slot", G=2))
    assert r.deadlock


# ---- the CU-cohort lock, with an L1 per CU and an L2 per XCD ------------------------------

# (xcd, cu) per agent: agents 0 and 1 share CU 0 of XCD 0, agent 2 is on CU 1 of XCD 0,
# agent 3 on CU 2 of XCD 1.  So hand-overs within a CU, between CUs of an XCD and between
# XCDs all occur.
CU3 = ((0, 0), (0, 0), (0, 1))
CU4 = ((0, 0), (0, 0), (0, 1), (1, 2))


@pytest.mark.parametrize("pl,ops,B", [(CU3, 2, 2), (CU3, 2, 3), (CU4, 1, 2), (CU4, 1, 3)])
def test_cu_cohort_lock_correct(pl, ops, B):
    """Mutual exclusion, no stale read of the guarded word through any L1 or L2, every
    acquisition completes and every level of the lock ends released, on all interleavings:
    a holder that inherits the XCD lock within its CU reads through the L1 the previous
    holder's stores went through, with no acquire."""
    r = explore(CuCohortLockModel(pl, ops, B))
    assert r.ok, r.violation


@pytest.mark.slow
def test_cu_cohort_lock_correct_two_xcds_twice():
    r = explore(CuCohortLockModel(CU4, 2, 2))
    assert r.ok and r.states > 10 ** 6, (r.states, r.violation)


@pytest.mark.parametrize("mutant,pl,ops,B", [("no_acquire", CU3, 2, 2),
                                             ("group_by_xcd", CU3, 2, 2),
                                             ("group_by_xcd", ((0, 0), (0, 1)), 2, 2)])
def test_cu_cohort_lock_cache_mutants_read_stale(mutant, pl, ops, B):
    """Without the acquire when the XCD lock is taken, or with groups that span CUs (a
    hand-over within the group then skips the acquire between two L1s), a holder reads a
    stale copy of the word."""
    r = explore(CuCohortLockModel(pl, ops, B, mutant))
    assert not r.ok and "stale" in r.violation


def test_cu_cohort_lock_pass_without_waiter_deadlocks():
    r = explore(CuCohortLockModel(CU3, 1, 3, "no_waiter_check"))
    assert r.deadlock


# ---- the per-XCD barrier as the library runs it, with its caches ----------------------

# (xcd, cu) per agent.  TWO_XCDS: XCD 0 holds agents 0 and 2 on one CU (agent 0 is the
# master and the CU leader, agent 2 waits on the CU's release line), XCD 1 holds agent 1.
TWO_XCDS = ((0, 0), (1, 1), (0, 0))
# FOUR: XCD 0 has two CUs (agents 0 and 3 share CU 0; agent 1 is alone on CU 1, a CU
# leader that is not the master), XCD 1 has agent 2.
FOUR = ((0, 0), (0, 1), (1, 2), (0, 0))


@pytest.mark.parametrize("placement,rounds", [(TWO_XCDS, 3), (TWO_XCDS, 4), (FOUR, 3)])
@pytest.mark.parametrize("copies", [1, 2])
@pytest.mark.parametrize("mode", ["plain", "coherent"])
def test_xcd_barrier_correct(placement, rounds, copies, mode):
    r = explore(XcdBarrierModel(placement, rounds, copies, mode))
    assert r.ok, r.violation


def test_xcd_barrier_registration_round():
    """Round 0 numbers the members and CUs with fetch-and-adds, as the library does."""
    r = explore(XcdBarrierModel(TWO_XCDS, 3, 2, register=True))
    assert r.ok, r.violation
    r = explore(XcdBarrierModel(TWO_XCDS, 3, 2, "coherent", register=True))
    assert r.ok, r.violation


@pytest.mark.parametrize("block,cu_lines", [(1, 8), (8, 0)])
def test_xcd_barrier_falls_back_when_registration_overflows(block, cu_lines):
    r = explore(XcdBarrierModel(TWO_XCDS, 3, 2, register=True, block=block, cu_lines=cu_lines))
    assert r.ok, r.violation


def test_xcd_barrier_l1_invalidation_needs_coherent_l2s():
    """Every workgroup dropping only its CU's L1 is enough if a writeback removes the other
    XCDs' copies of the lines, and not otherwise."""
    r = explore(XcdBarrierModel(TWO_XCDS, 3, 2, "l1only", l2_coherent=True))
    assert r.ok, r.violation
    r = explore(XcdBarrierModel(TWO_XCDS, 3, 2, "l1only", l2_coherent=False))
    assert r.violation and "phase" in r.violation


@pytest.mark.parametrize("mutant", ["early_publish", "early_release", "no_writeback",
                                    "no_invalidate", "no_cu_wait", "flag_before_store"])
def test_xcd_barrier_mutants_read_stale_data(mutant):
    r = explore(XcdBarrierModel(TWO_XCDS, 3, 2, mutant=mutant))
    assert r.violation and "phase" in r.violation


def test_xcd_barrier_missing_stamp_copy_deadlocks():
    r = explore(XcdBarrierModel(TWO_XCDS, 3, 2, mutant="skip_copy"))
    assert r.deadlock


def test_xcd_barrier_rank_stored_late_is_caught():
    r = explore(XcdBarrierModel(((0, 0), (0, 1), (0, 0)), 2, 2, register=True,
                                mutant="rank_after_arrival"))
    assert r.violation


# ---- MCS queue lock --------------------------------------------------------------------

@pytest.mark.parametrize("n,ops", [(2, 2), (2, 3), (3, 2)])
def test_mcs_lock_correct(n, ops):
    r = explore(MCSLockModel(n, ops))
    assert r.ok, r.violation


@pytest.mark.parametrize("mutant", ["no_wait_for_next", "link_before_init", "store_tail"])
def test_mcs_lock_mutants_deadlock(mutant):
    r = explore(MCSLockModel(3, 2, mutant=mutant))
    assert not r.ok


def test_mcs_lock_entering_without_spinning_breaks_exclusion():
    r = explore(MCSLockModel(2, 2, mutant="no_spin"))
    assert r.violation and "mutual exclusion" in r.violation


# ---- cohort semaphore (Algorithm 5's count, a queue per XCD, local hand-over) -------------

@pytest.mark.parametrize("K,placement,B,small_q", [(1, (0, 1, 0), 2, False),
                                                   (1, (0, 1, 0), 3, False),
                                                   (1, (0, 1, 0), 2, True),
                                                   (1, (0, 0, 0), 2, False),
                                                   (2, (0, 1, 0), 2, True)])
def test_cohort_semaphore_correct(K, placement, B, small_q):
    """Occupancy never above K, final state quiescent, and with K = 1 no update of the
    guarded word lost through the L2s (local hand-overs skip the writeback)."""
    r = explore(CohortSemModel(K, placement, 2, B, small_q=small_q))
    assert r.ok, r.violation


@pytest.mark.parametrize("mutant", ["no_remote_writeback", "no_acquire"])
def test_cohort_semaphore_mutants_lose_updates(mutant):
    r = explore(CohortSemModel(1, (0, 1, 0), 2, 2, mutant=mutant))
    assert r.violation and "lost update" in r.violation


def test_cohort_semaphore_unchecked_claim_deadlocks():
    r = explore(CohortSemModel(1, (0, 1, 0), 2, 2, mutant="claim_unchecked"))
    assert r.deadlock


def _advance(model, sh, los, a, until, limit=64):
    """Step agent `a` alone until its program counter is `until` (or it is done)."""
    for _ in range(limit):
        if los[a][0] == until or model.done(los[a]):
            return sh, los
        sh, lo = model.step(a, sh, los[a])
        los = los[:a] + (lo,) + los[a + 1:]
    raise AssertionError(f"agent {a} did not reach {until}")


def _predict_schedule(model):
    """K = 2, five workgroups on one XCD: 0 and 1 enter, 2-4 queue; 0 leaves its critical
    section and predicts from count = 5 > 2K; then 1, 2, 3, 4 pass the other unit along
    and finish; only then does 0's decrement land."""
    M = CohortSemModel
    sh, los = model.init()
    for a in range(5):
        sh, los = _advance(model, sh, los, a, M.ACQ if a < 2 else M.W_POLL)
    sh, los = _advance(model, sh, los, 0, M.P_PRED)
    sh, lo = model.step(0, sh, los[0])  # the prediction
    los = (lo,) + los[1:]
    for a in range(1, 5):
        sh, los = _advance(model, sh, los, a, M.DONE, limit=256)
    return sh, los


def test_cohort_semaphore_count_prediction_unsafe_for_k2():
    """A post that decides from a loaded count > 2K that a waiter exists (and skips the
    writeback) can find none left: the other unit served all three waiters first."""
    model = CohortSemModel(2, (0, 0, 0, 0, 0), 1, 2, mutant="predict_2k")
    sh, los = _predict_schedule(model)
    assert all(model.done(lo) for lo in los[1:])
    for _ in range(8):  # workgroup 0 decrements, then searches every queue forever
        sh2, lo = model.step(0, sh, los[0])
        sh, los = sh2, (lo,) + los[1:]
    assert los[0][0] == CohortSemModel.P_REMOTE and sh[0] == 0
    assert model.step(0, sh, los[0]) == (sh, los[0])  # no ticket to claim: stuck


def test_cohort_semaphore_no_prediction_for_k2():
    """The shipped rule (hand-over mode only for K = 1) finishes the same schedule."""
    model = CohortSemModel(2, (0, 0, 0, 0, 0), 1, 2)
    sh, los = _predict_schedule(model)
    sh, los = _advance(model, sh, los, 0, CohortSemModel.DONE, limit=256)
    assert all(model.done(lo) for lo in los) and sh[0] == 0 and sh[6] == 0


@pytest.mark.parametrize("K,placement,M", [(1, (0, 1, 0), 1), (1, (0, 1, 0), 2),
                                          (2, (0, 1, 0), 1), (2, (0, 1, 0), 2),
                                          (2, (0, 1, 1), 4)])
def test_array_semaphore_correct(K, placement, M):
    """Grant slots shared by several tickets (M below the 6 tickets drawn), grants landing
    in any order: occupancy never above K, every waiter enters, with K = 1 no update of
    the guarded word lost through the L2s."""
    r = explore(ArraySemModel(K, placement, M, 2))
    assert r.ok, r.violation


@pytest.mark.parametrize("mutant,K,M,expect", [
    ("enter_at_k", 2, 1, "occupancy"),
    ("grant_next", 2, 2, "occupancy"),
    ("no_writeback", 1, 1, "without an earlier holder's update"),
    ("no_acquire", 1, 1, "without an earlier holder's update"),
])
def test_array_semaphore_mutants_violate_safety(mutant, K, M, expect):
    r = explore(ArraySemModel(K, (0, 1, 0), M, 2, mutant=mutant))
    assert r.violation and expect in r.violation


@pytest.mark.parametrize("mutant", ["store", "poll_eq"])
def test_array_semaphore_grant_must_be_a_maximum(mutant):
    """A plain store lets an earlier grant that lands late lower a shared slot, and an
    exact-match poll misses its grant under a later one: both strand a waiter."""
    r = explore(ArraySemModel(2, (0, 1, 0), 2, 2, mutant=mutant))
    assert r.deadlock


@pytest.mark.parametrize("K,M", [(1, 1), (1, 2), (2, 2), (2, 4), (3, 3)])
def test_chain_semaphore_correct(K, M):
    """The chain rule with M a multiple of K: the holder of ticket t grants t + K with a
    plain store; occupancy never above K, everyone enters, no lost update at K = 1."""
    r = explore(ArraySemModel(K, (0, 1, 0), M, 2, rule="chain"))
    assert r.ok, r.violation


def test_chain_semaphore_needs_slots_a_multiple_of_k():
    """With M not a multiple of K another chain's store reaches a waiter's slot: one slot
    for two chains admits a third holder, three slots for two chains strand a waiter."""
    r = explore(ArraySemModel(2, (0, 1, 0), 1, 2, rule="chain"))
    assert r.violation and "occupancy" in r.violation
    r = explore(ArraySemModel(2, (0, 1, 0), 3, 2, rule="chain"))
    assert r.deadlock


@pytest.mark.parametrize("mutant,K,M,expect", [
    ("enter_at_k", 2, 2, "occupancy"),
    ("grant_next", 2, 2, "occupancy"),
    ("no_writeback", 1, 1, "without an earlier holder's update"),
    ("no_acquire", 1, 1, "without an earlier holder's update"),
])
def test_chain_semaphore_mutants(mutant, K, M, expect):
    r = explore(ArraySemModel(K, (0, 1, 0), M, 2, mutant=mutant, rule="chain"))
    assert r.violation and expect in r.violation


@pytest.mark.parametrize("K,placement,Q,M", [(2, (0, 1, 0, 1), 2, 2), (2, (0, 1, 0, 1), 2, 1),
                                              (3, (0, 1, 0, 1), 2, 2), (2, (0, 0, 1), 2, 2),
                                              (1, (0, 1, 0), 1, 2)])
def test_xcd_chain_semaphore_correct(K, placement, Q, M):
    """Chains per XCD queue with L1s and L2s: with a queue per XCD the posts skip the
    writeback and no update is lost; with XCDs sharing a queue they write back."""
    r = explore(XcdChainSemModel(K, placement, Q, M))
    assert r.ok, r.violation


@pytest.mark.parametrize("mutant,K,placement,Q", [
    ("skip_when_shared", 1, (0, 1, 0), 1),
    ("no_acquire", 2, (0, 0, 1), 2),
    ("enter_at_k", 2, (0, 1, 0, 1), 2),
])
def test_xcd_chain_semaphore_mutants(mutant, K, placement, Q):
    r = explore(XcdChainSemModel(K, placement, Q, 2, mutant=mutant))
    assert r.violation
