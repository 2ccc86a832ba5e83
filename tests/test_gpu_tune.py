"""Autotuner on the GPU: a reduced tuning pass picks consistent winners, installs them as
the library's defaults, and the *_DEFAULT primitives then reproduce the oracle."""

import pytest

import oracle
from conftest import announce

pytestmark = pytest.mark.gpu


def test_tune_install_and_default_parity(ctx, tmp_path):
    import paper_1110_4623_amd as sp
    from paper_1110_4623_amd import tune
    announce("tune barrier")
    res = {"device": tune.device_key(ctx), "barrier": {}, "mutex": {}, "semaphore": {}}
    bc = [("central", {"poll_sleep": 1}), ("xcd", {"poll_sleep": 1}),
          ("tree", {"fan_in": 8, "poll_sleep": 0}), ("flag", {"flags_packed": 1})]
    res["barrier"]["0"] = tune.tune_barrier(ctx, 16, rounds=200, candidates=bc)
    res["barrier"]["1"] = tune.tune_barrier(ctx, 512, rounds=200, candidates=bc)
    announce("tune mutex")
    mc = [("ticket", {"poll_sleep": 0}), ("sleep", {"poll_sleep": 4}),
          ("spin_backoff", {"backoff": "exp", "backoff_max": 32})]
    res["mutex"]["0"] = tune.tune_mutex(ctx, 16, total=512, candidates=mc)
    res["mutex"]["1"] = tune.tune_mutex(ctx, 256, total=512, candidates=mc)
    announce("tune semaphore")
    sc = [("ticket", {"poll_sleep": 0}), ("sleep", {"poll_sleep": 4})]
    res["semaphore"]["0"] = tune.tune_semaphore(ctx, 64, 32, total=1024, candidates=sc)
    res["semaphore"]["1"] = tune.tune_semaphore(ctx, 2048, 32, total=4096, candidates=sc)
    for prim in ("barrier", "mutex", "semaphore"):
        for b in ("0", "1"):
            best = res[prim][b]["best"]
            assert best["consistent"], (prim, b, best)
    path = str(tmp_path / "tuner.json")
    tune.save(res, path)
    tune.apply(ctx, tune.load(path))
    announce("defaults after tuning")
    for nwg in (16, 512):
        bar = sp.Barrier(ctx, "default", nwg)
        try:
            chk, _ = bar.run_hash(256, 300, 42)
        finally:
            bar.close()
        assert (chk == oracle.barrier_closed(42, nwg, 300)).all()
    m = sp.Mutex(ctx, "default", 1, 16)
    try:
        for nwg in (16, 256):
            words, _, _ = m.run(nwg, 256, 2048, 100, 7)
            assert (words == oracle.mutex_closed(7, nwg, 2048, 1, 16)).all()
    finally:
        m.close()
    s = sp.Semaphore(ctx, "default", 32)
    try:
        for nwg in (64, 2048):
            r = s.run(nwg, 256, 4096, 100, 7)
            assert (r["chk"] == oracle.sem_closed(7, nwg, 4096)).all()
            assert r["maxocc"] <= 32
    finally:
        s.close()


def test_tune_rejects_a_candidate_that_times_out(ctx):
    from paper_1110_4623_amd import tune
    # spin semaphores hand over a few hundred pairs per second at 2048 workgroups: with a
    # 300 ms limit the spin candidate times out and the sleeping one wins
    announce("tune semaphore timeout")
    r = tune.tune_semaphore(ctx, 2048, 4, total=8192, limit_ms=300,
                            candidates=[("spin", {}), ("sleep", {"poll_sleep": 4})])
    rows = {c["kind"]: c for c in r["candidates"]}
    assert "error" in rows["spin"] and not rows["spin"]["consistent"]
    assert r["best"]["kind"] == "sleep"


def test_tune_serve_picks_a_consistent_config(ctx):
    import sp_inputs
    from paper_1110_4623_amd import tune
    reqs = sp_inputs.request_table(3000, 1e5, 42)
    announce("tune serve")
    r = tune.tune_serve(ctx, reqs, candidates=[dict(nwg=256, poll_sleep=0, far_sleep=4),
                                               dict(nwg=1024, poll_sleep=2, far_sleep=1)])
    assert all(c["consistent"] for c in r["candidates"])
    assert r["best"]["p99_us"] == min(c["p99_us"] for c in r["candidates"])


def test_tune_mutex_times_queue_locks(ctx):
    """Queue mutexes allocate their slots on first use; the tuner warms every candidate up
    before recording it, so they are timed rather than rejected."""
    from paper_1110_4623_amd import tune
    announce("tune queue mutexes")
    r = tune.tune_mutex(ctx, 256, total=1024, candidates=[("array", {"poll_sleep": 0}),
                                                           ("ring", {"poll_sleep": 0})])
    for c in r["candidates"]:
        assert c["consistent"] and "error" not in c, c
