"""Degenerate inputs on the GPU: no work at all, fewer operations than workgroups, one
workgroup, and workgroup counts that are not powers of two.  Every result equals the
oracle's closed form and every primitive ends in its quiescent state."""

import numpy as np
import pytest

import oracle
from conftest import announce

pytestmark = pytest.mark.gpu

BARRIERS = ["central", "central_split", "tree", "flag", "xcd", "grid_sync"]
MUTEXES = ["spin_cas", "spin_exch", "spin_backoff", "ticket", "sleep", "ring", "array",
           "adaptive", "cohort", "mcs", "cu_cohort"]
SEMS = ["spin", "spin_backoff", "ticket", "sleep", "counters", "adaptive", "cohort", "array",
        "chain"]


@pytest.mark.parametrize("kind", BARRIERS)
@pytest.mark.parametrize("nwg,rounds", [(1, 0), (3, 0), (2048, 0), (1, 1), (3, 1), (2048, 1)])
def test_barrier_zero_and_one_round(ctx, kind, nwg, rounds):
    import paper_1110_4623_amd as sp
    announce("barrier", kind, f"nwg={nwg} lanes=256 rounds={rounds}")
    bar = sp.Barrier(ctx, kind, nwg)
    try:
        chk, _ = bar.run_hash(lanes=256, rounds=rounds, seed=11)
    finally:
        bar.close()
    want = oracle.barrier_closed(11, nwg, rounds)
    if rounds == 0:
        assert not want.any()
    assert (chk == want).all()


def _mutex(ctx, kind, nwg, total, L, W, seed):
    import paper_1110_4623_amd as sp
    announce("mutex", kind, f"nwg={nwg} lanes=64 total={total} L={L} W={W}")
    m = sp.Mutex(ctx, kind, L, W)
    try:
        words, _, fin = m.run(nwg=nwg, lanes=64, total=total, max_delay=100, seed=seed,
                              finish=True)
    finally:
        m.close()
    return words, fin


@pytest.mark.parametrize("kind", MUTEXES)
@pytest.mark.parametrize("nwg,total", [(1, 0), (64, 0), (64, 5), (301, 1000), (2048, 2047)])
def test_mutex_few_operations(ctx, kind, nwg, total):
    """No acquisitions leaves every word zero; with fewer acquisitions than workgroups
    most workgroups take none, and the counts are still exact."""
    words, fin = _mutex(ctx, kind, nwg, total, 7, 5, 13)
    want = oracle.mutex_closed(13, nwg, total, 7, 5)
    assert int(want.sum()) == 5 * total
    assert (words == want).all()
    assert fin is not None and len(fin) == nwg


def _sem(ctx, kind, K, nwg, total, seed):
    import paper_1110_4623_amd as sp
    announce("sem", kind, f"K={K} nwg={nwg} lanes=64 total={total}")
    s = sp.Semaphore(ctx, kind, K)
    try:
        return s.run(nwg=nwg, lanes=64, total=total, max_hold=100, seed=seed)
    finally:
        s.close()


def _sem_quiescent(r, kind, K, total):
    s_or_count, ticket, turn, adm = r["state"]
    assert adm == total and r["occ"] == 0
    assert r["maxocc"] <= K and (r["maxocc"] >= 1) == (total > 0)
    if kind.startswith("spin"):
        assert s_or_count == K + 1
    elif kind in ("counters", "adaptive", "array", "chain", "xcd_chain"):
        assert s_or_count == 0 and ticket == turn == total
    else:
        assert s_or_count == 0 and ticket == turn
    if kind == "cohort":
        assert r["unserved"] == 0


@pytest.mark.parametrize("nwg,total", [(1, 0), (64, 0), (1, 50), (64, 5), (37, 1001),
                                       (2048, 3001)])
def test_cu_lock_semaphore_few_operations(ctx, nwg, total):
    """The K = 1 CU-cohort-lock semaphore with no work, fewer pairs than workgroups and a
    ragged split."""
    r = _sem(ctx, "cu_lock", 1, nwg, total, 17)
    want = oracle.sem_closed(17, nwg, total)
    assert (r["chk"] == want).all()
    _sem_quiescent(r, "cu_lock", 1, total)


@pytest.mark.parametrize("kind", SEMS)
@pytest.mark.parametrize("K", [1, 3])
@pytest.mark.parametrize("nwg,total", [(1, 0), (64, 0), (1, 50), (64, 5), (37, 1001)])
def test_semaphore_few_operations(ctx, kind, K, nwg, total):
    r = _sem(ctx, kind, K, nwg, total, 17)
    want = oracle.sem_closed(17, nwg, total)
    if total < nwg:
        assert not want[total:].any()
    assert (r["chk"] == want).all()
    _sem_quiescent(r, kind, K, total)


@pytest.mark.parametrize("kind", ["ticket", "sleep", "counters", "adaptive", "cohort", "array",
                                  "chain"])
@pytest.mark.parametrize("K", [5, 300])
def test_semaphore_odd_grid(ctx, kind, K):
    # 300 workgroups, 12345 pairs: 45 workgroups take one pair more than the rest
    r = _sem(ctx, kind, K, 300, 12345, 19)
    assert (r["chk"] == oracle.sem_closed(19, 300, 12345)).all()
    _sem_quiescent(r, kind, K, 12345)


@pytest.mark.parametrize("kind", ["ticket", "sleep", "counters", "adaptive", "cohort", "array",
                                  "chain", "xcd_chain"])
def test_semaphore_capacity_above_agents(ctx, kind):
    r = _sem(ctx, kind, 64, 16, 4000, 7)
    assert (r["chk"] == oracle.sem_closed(7, 16, 4000)).all()
    _sem_quiescent(r, kind, 64, 4000)
    if kind in ("ticket", "sleep"):
        assert r["state"][1] == 0  # a wait never had to queue: no ticket was drawn


@pytest.mark.parametrize("nwg,total", [(1, 0), (8, 5), (37, 1001), (300, 12345)])
def test_xcd_chain_few_operations_and_odd_grids(ctx, nwg, total):
    # K = 9: one XCD's queue has two units, the others one
    r = _sem(ctx, "xcd_chain", 9, nwg, total, 17)
    assert (r["chk"] == oracle.sem_closed(17, nwg, total)).all()
    _sem_quiescent(r, "xcd_chain", 9, total)
