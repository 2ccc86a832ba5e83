"""Recorded batches: a barrier, a mutex and a semaphore run recorded into one HIP graph
give the oracle's results on every replay, with eager work and host waits between the
replays; calls that cannot be recorded are refused."""

import numpy as np
import pytest

import oracle
from conftest import announce

pytestmark = pytest.mark.gpu

NWG, LANES, ROUNDS = 256, 256, 1000
MTX = dict(nwg=NWG, lanes=LANES, total=1 << 14, max_delay=200)
SEM = dict(nwg=NWG, lanes=LANES, total=1 << 14, max_hold=200)


def _expect(seed):
    return (oracle.barrier_closed(seed, NWG, ROUNDS),
            oracle.mutex_closed(seed, NWG, MTX["total"], 4, 16),
            oracle.sem_closed(seed, NWG, SEM["total"]))


def _check(bar, mtx, sem, exp, K):
    assert (bar.checksums() == exp[0]).all()
    assert (mtx.words() == exp[1]).all()
    r = sem.result()
    assert (r["chk"] == exp[2]).all()
    assert 1 <= r["maxocc"] <= K and r["state"][3] == SEM["total"]


@pytest.mark.parametrize("barrier", ["xcd", "central", "flag", "tree"])
def test_recorded_step_replays_match_oracle(ctx, barrier):
    import paper_1110_4623_amd as sp
    seed, K = 42, 4
    exp = _expect(seed)
    bar = sp.Barrier(ctx, barrier, NWG)
    mtx = sp.Mutex(ctx, "ticket", 4, 16)
    sem = sp.Semaphore(ctx, "sleep", K)
    other = sp.Barrier(ctx, "central", 64)
    try:
        announce("graph eager", barrier)
        bar.launch(LANES, ROUNDS, seed)
        mtx.launch(seed=seed, **MTX)
        sem.launch(seed=seed, **SEM)
        _check(bar, mtx, sem, exp, K)
        g = sp.Graph(ctx)
        with g:
            bar.launch(LANES, ROUNDS, seed)
            mtx.launch(seed=seed, **MTX)
            sem.launch(seed=seed, **SEM)
        for rep in range(3):
            announce("graph replay", barrier, rep)
            st = g.launch(replays=1 + rep)
            assert st["device_error"] == 0 and st["ops"] == 1 + rep
            _check(bar, mtx, sem, exp, K)
            # eager work between replays, on other state and with a host wait
            chk, _ = other.run_hash(64, 100, 7 + rep)
            assert (chk == oracle.barrier_closed(7 + rep, 64, 100)).all()
        g.close()
    finally:
        for o in (bar, mtx, sem, other):
            o.close()


def test_replay_overhead_below_call_overhead(ctx):
    """Many short runs: one graph replay per run costs less host time than one library
    call per run (which waits and reads the watchdog word every time)."""
    import time

    import paper_1110_4623_amd as sp
    bar = sp.Barrier(ctx, "xcd", 16)
    try:
        bar.launch(64, 10, 1)
        t = time.perf_counter()
        for _ in range(50):
            bar.launch(64, 10, 1)
        eager = (time.perf_counter() - t) / 50
        g = sp.Graph(ctx)
        with g:
            bar.launch(64, 10, 1)
        g.launch(1)
        t = time.perf_counter()
        g.launch(50)
        replay = (time.perf_counter() - t) / 50
        assert (bar.checksums() == oracle.barrier_closed(1, 16, 10)).all()
        print(f"[graph] per run: eager {eager * 1e6:.1f} us, replay {replay * 1e6:.1f} us",
              flush=True)
        assert replay < eager
        g.close()
    finally:
        bar.close()


@pytest.mark.parametrize("kind,params", [("grid_sync", {}), ("central", {"cooperative": 1})])
def test_cooperative_launch_cannot_be_recorded(ctx, kind, params):
    import paper_1110_4623_amd as sp
    announce("graph refuses cooperative", kind, params)
    bar = sp.Barrier(ctx, kind, 16, **params)
    try:
        g = sp.Graph(ctx)
        with pytest.raises(sp.SpError):
            with g:
                bar.launch(64, 10, 1)
    finally:
        bar.close()
    # the context still works after the refused recording
    ok = sp.Barrier(ctx, "central", 16)
    try:
        chk, _ = ok.run_hash(64, 10, 3)
        assert (chk == oracle.barrier_closed(3, 16, 10)).all()
    finally:
        ok.close()


def test_default_mutex_recorded_on_first_use(ctx):
    """A DEFAULT mutex whose kind resolves to the cohort lock (2048 contenders on one lock)
    records into a graph on its very first run: its state is allocated at creation."""
    import paper_1110_4623_amd as sp
    seed, total = 9, 1 << 14
    m = sp.Mutex(ctx, "default", 1, 16)
    try:
        announce("graph default mutex first use")
        g = sp.Graph(ctx)
        with g:
            m.launch(2048, 256, total, 200, seed)
        for rep in range(2):
            st = g.launch(replays=1)
            assert st["device_error"] == 0
            assert (m.words() == total).all()
        g.close()
    finally:
        m.close()


def test_calls_that_cannot_be_recorded_are_refused(ctx):
    """Inside a recording, calls that wait for a host result or allocate raise at once and
    leave the recording usable: what was recorded before and after still replays."""
    import paper_1110_4623_amd as sp
    bar = sp.Barrier(ctx, "central", 64)
    try:
        announce("graph refusals")
        g = sp.Graph(ctx)
        with g:
            bar.launch(64, 50, 3)
            with pytest.raises(sp.SpError):
                sp.shader_clock_mhz(ctx)
            with pytest.raises(sp.SpError):
                sp.bench_fence(ctx, "release", 8)
            bar.launch(64, 50, 4)
        st = g.launch(replays=2)
        assert st["device_error"] == 0
        assert (bar.checksums() == oracle.barrier_closed(4, 64, 50)).all()
        g.close()
    finally:
        bar.close()
