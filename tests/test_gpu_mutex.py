"""GPU parity of the mutexes: the final critical-section words must equal the exact
acquisition counts of the oracle's closed form."""

import numpy as np
import pytest

import oracle
from conftest import announce

pytestmark = pytest.mark.gpu

KINDS = ["spin_cas", "spin_exch", "spin_backoff", "ticket", "sleep", "ring", "array", "adaptive",
         "cohort", "mcs", "cu_cohort"]


def _run(ctx, kind, nwg, lanes, total, L, W, delay, seed, **params):
    import paper_1110_4623_amd as sp
    announce("mutex", kind, f"nwg={nwg} lanes={lanes} total={total} L={L} W={W} delay={delay}",
             params)
    m = sp.Mutex(ctx, kind, L, W, **params)
    try:
        words, st, fin = m.run(nwg=nwg, lanes=lanes, total=total, max_delay=delay, seed=seed,
                               finish=True)
    finally:
        m.close()
    return words, st, fin


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("L,W", [(1, 1), (1, 256), (16, 16), (256, 1), (3, 100)])
def test_small(ctx, kind, L, W):
    total, nwg, seed = 1 << 13, 64, 42
    words, st, _ = _run(ctx, kind, nwg, 256, total, L, W, 200, seed)
    assert (words == oracle.mutex_closed(seed, nwg, total, L, W)).all()


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("nwg", [1, 5, 2048])
def test_workgroup_counts(ctx, kind, nwg):
    total, seed = 3000, 7
    words, _, _ = _run(ctx, kind, nwg, 64, total, 4, 3, 0, seed)
    assert (words == oracle.mutex_closed(seed, nwg, total, 4, 3)).all()


@pytest.mark.parametrize("kind", KINDS)
def test_full_size_single_lock(ctx, kind):
    # 2048 workgroups x 256 lanes contend for one lock with 16 words.  The queue locks
    # (ticket, ring, array) run all 2^20 acquisitions; the spin and polling locks hand the
    # lock over far more slowly with 2048 contenders (every waiter hammers the lock word),
    # so they run 2^14 acquisitions at the same contention.
    total = 1 << 20 if kind in ("ticket", "ring", "array", "adaptive", "cohort", "mcs",
                                "cu_cohort") else 1 << 14
    words, st, fin = _run(ctx, kind, 2048, 256, total, 1, 16, 1000, 0xC0FFEE)
    assert (words == total).all()


@pytest.mark.parametrize("kind", ["spin_cas", "spin_backoff", "sleep", "ticket", "array", "ring",
                                  "cohort", "mcs", "cu_cohort"])
@pytest.mark.parametrize("L,W", [(16, 256), (256, 16)])
def test_full_size_many_locks(ctx, kind, L, W):
    total, seed = 1 << 20, 42
    words, _, _ = _run(ctx, kind, 2048, 256, total, L, W, 1000, seed, timeout_ms=60000)
    assert (words == oracle.mutex_closed(seed, 2048, total, L, W)).all()


@pytest.mark.parametrize("params", [dict(backoff="paper", backoff_min=1, backoff_max=32),
                                    dict(backoff="exp", backoff_unit="load"),
                                    dict(pad_bytes=4), dict(pad_bytes=4096)])
def test_backoff_and_padding(ctx, params):
    total, seed = 1 << 14, 3
    for kind in ("spin_exch", "ticket"):
        words, _, _ = _run(ctx, kind, 512, 128, total, 8, 8, 100, seed, **params)
        assert (words == oracle.mutex_closed(seed, 512, total, 8, 8)).all()


def test_watchdog_timeout_path(ctx):
    # A 1 ms watchdog on a run that needs far longer: every wait gives up, the kernel
    # drains and the call reports a timeout; the library keeps working afterwards.
    import paper_1110_4623_amd as sp
    announce("mutex watchdog")
    m = sp.Mutex(ctx, "spin_cas", 1, 1, timeout_ms=1)
    with pytest.raises(sp.SpTimeout):
        m.run(nwg=1024, lanes=64, total=1 << 20, max_delay=1000, seed=1)
    m.close()
    words, _, _ = _run(ctx, "ticket", 64, 64, 1000, 1, 1, 0, 1)
    assert (words == 1000).all()


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("L,W", [(1, 16), (16, 16), (256, 1)])
def test_coherent_critical_sections(ctx, kind, L, W):
    """coherent_cs: critical sections with agent-scope accesses and no fences around them
    give the same exact counts (owner word checked on every entry)."""
    total, seed = 1 << 13, 42
    nwg = 64 if kind.startswith("spin") else 256
    words, st, _ = _run(ctx, kind, nwg, 256, total, L, W, 200, seed, coherent_cs=1, verify=1)
    assert st["device_error"] == 0
    assert (words == oracle.mutex_closed(seed, nwg, total, L, W)).all()


def test_coherent_critical_sections_full_size_ticket(ctx):
    total, seed, nwg = 1 << 20, 7, 2048
    fenced, st_f, _ = _run(ctx, "ticket", nwg, 256, total, 1, 16, 1000, seed)
    coh, st_c, _ = _run(ctx, "ticket", nwg, 256, total, 1, 16, 1000, seed, coherent_cs=1)
    expect = oracle.mutex_closed(seed, nwg, total, 1, 16)
    assert (fenced == expect).all() and (coh == expect).all()
    print(f"[mutex] ticket 2048 WG one lock: fenced {total / st_f['kernel_ms'] * 1e3:.3e} acq/s, "
          f"coherent {total / st_c['kernel_ms'] * 1e3:.3e} acq/s", flush=True)


@pytest.mark.parametrize("kind", ["cohort", "cu_cohort"])
@pytest.mark.parametrize("passes", [1, 2, 64, 255])
@pytest.mark.parametrize("L,W,delay", [(1, 16, 1000), (1, 256, 0), (16, 256, 100)])
def test_cohort_local_hand_overs(ctx, kind, passes, L, W, delay):
    """The cohort lock hands the lock to a holder of the same XCD without the L2
    writeback, the CU-cohort lock also to a holder of the same CU without any cache
    maintenance: at 2048 contenders most hand-overs are local, and the counts (W words
    spread over eight lines at W = 256) and the owner check stay exact for any bound."""
    total, seed = 1 << 18, 5
    words, st, _ = _run(ctx, kind, 2048, 256, total, L, W, delay, seed,
                        cohort_passes=passes, verify=1)
    assert st["device_error"] == 0
    assert (words == oracle.mutex_closed(seed, 2048, total, L, W)).all()


@pytest.mark.parametrize("kind", ["cohort", "cu_cohort"])
@pytest.mark.parametrize("pad", [4, 4096])
def test_cohort_padding_and_coherent(ctx, kind, pad):
    total, seed = 1 << 16, 9
    for coherent in (0, 1):
        words, st, _ = _run(ctx, kind, 1024, 128, total, 4, 32, 100, seed, pad_bytes=pad,
                            coherent_cs=coherent, verify=1)
        assert st["device_error"] == 0
        assert (words == oracle.mutex_closed(seed, 1024, total, 4, 32)).all()
