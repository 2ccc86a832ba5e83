"""Exhaustive-interleaving checks of every algorithm on tiny instances, and mutation
tests that pin the checker itself: each planted mistake must be caught (CPU only)."""

import pytest

from oracle.modelcheck import (BarrierModel, CohortLockModel, CondModel, FASemModel, MutexModel,
                               QueueLockModel, SpinSemModel, WeightedSemModel, explore)


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


@pytest.mark.parametrize("kind", ["central", "xcd", "flag"])
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


@pytest.mark.parametrize("kind", ["central", "xcd", "flag"])
def test_catches_single_buffered_exchange(kind):
    r = explore(BarrierModel(kind, 2, 3, 2, mutant="single_buffer"))
    assert r.violation and "phase" in r.violation


@pytest.mark.parametrize("kind", ["central", "flag"])
def test_catches_barrier_that_does_not_wait(kind):
    r = explore(BarrierModel(kind, 2, 2, mutant="no_wait"))
    assert r.violation and "phase" in r.violation


def test_catches_hierarchical_group_released_early():
    r = explore(BarrierModel("xcd", 4, 2, 2, mutant="no_top_wait"))
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
