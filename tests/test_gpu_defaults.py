"""The *_DEFAULT kinds resolve, per contention bucket, to the library's built-in choices
(the winners of a tuning pass) and reproduce the oracle at both buckets."""

import pytest

import oracle
from conftest import announce

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nwg", [16, 512])
def test_default_barrier(ctx, nwg):
    import paper_1110_4623_amd as sp
    announce("default barrier", nwg)
    b = sp.Barrier(ctx, "default", nwg)
    try:
        chk, _ = b.run_hash(256, 500, 9)
    finally:
        b.close()
    assert (chk == oracle.barrier_closed(9, nwg, 500)).all()


@pytest.mark.parametrize("nwg", [16, 256, 1024, 2048])
def test_default_mutex(ctx, nwg):
    """The default mutex at low contention (spin lock with backoff), at one contender per
    CU (the XCD-cohort lock) and at four and eight (the CU-cohort lock): exact counts, no
    two holders at once."""
    import paper_1110_4623_amd as sp
    announce("default mutex", nwg)
    m = sp.Mutex(ctx, "default", 1, 16, verify=1)
    try:
        words, st, _ = m.run(nwg, 256, 4096, 500, 9)
    finally:
        m.close()
    assert st["device_error"] == 0
    assert (words == oracle.mutex_closed(9, nwg, 4096, 1, 16)).all()


@pytest.mark.parametrize("nwg", [64, 2048])
def test_default_semaphore(ctx, nwg):
    import paper_1110_4623_amd as sp
    announce("default semaphore", nwg)
    s = sp.Semaphore(ctx, "default", 32)
    try:
        r = s.run(nwg, 256, 8192, 500, 9)
    finally:
        s.close()
    assert (r["chk"] == oracle.sem_closed(9, nwg, 8192)).all()
    assert 1 <= r["maxocc"] <= 32 and r["state"][3] == 8192
