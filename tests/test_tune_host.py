"""Host logic of the autotuner (no GPU): installation of the winners and the cache."""

import pytest


class FakeCtx:
    info = {"arch": "gfx950:sramecc+:xnack-", "cu_count": 256, "xcd_count": 8}

    def __init__(self):
        self.calls = []

    def set_default(self, prim, bucket, kind, **params):
        self.calls.append((prim, bucket, kind, params))


def _tuned(device):
    best = lambda k, p: {"best": {"kind": k, "params": p, "consistent": True}}  # noqa: E731
    return {"device": device,
            "barrier": {"0": best("central_split", {"poll_sleep": 1}), "1": best("xcd", {})},
            "mutex": {"0": best("ticket", {}), "1": best("sleep", {"poll_sleep": 4})},
            "semaphore": {"1": best("sleep", {"poll_sleep": 16})}}


def test_apply_installs_every_bucket(tmp_path):
    from paper_1110_4623_amd import tune
    ctx = FakeCtx()
    path = str(tmp_path / "sub" / "t.json")
    tune.save(_tuned(tune.device_key(ctx)), path)
    tune.apply(ctx, tune.load(path))
    assert ("barrier", 1, "xcd", {}) in ctx.calls
    assert ("mutex", 1, "sleep", {"poll_sleep": 4}) in ctx.calls
    assert ("semaphore", 1, "sleep", {"poll_sleep": 16}) in ctx.calls
    assert len(ctx.calls) == 5


def test_apply_refuses_another_device():
    from paper_1110_4623_amd import tune
    with pytest.raises(ValueError):
        tune.apply(FakeCtx(), _tuned("gfx942/304cu/8xcd"))


def test_candidate_lists_cover_every_kind():
    from paper_1110_4623_amd import tune
    assert {k for k, _ in tune.barrier_candidates()} == {"central", "central_split", "xcd",
                                                          "flag", "tree"}
    assert {k for k, _ in tune.mutex_candidates()} == {"spin_cas", "spin_exch", "spin_backoff",
                                                        "ticket", "sleep", "ring", "array",
                                                        "adaptive", "cohort", "mcs",
                                                        "cu_cohort"}
    assert {k for k, _ in tune.semaphore_candidates()} == {"spin", "spin_backoff", "ticket",
                                                            "sleep", "counters", "adaptive",
                                                            "cohort", "array", "chain",
                                                            "xcd_chain"}
    # Algorithm 4's post backoff is searched both ways
    assert {p.get("post_backoff") for k, p in tune.semaphore_candidates()
            if k == "spin_backoff"} == {0, 1}


def test_semaphore_points_rank_by_geometric_mean(monkeypatch):
    """A candidate must be correct at every point; the best geometric mean wins, so a
    candidate fast at one K and slow at the other loses to a steady one."""
    import math
    from paper_1110_4623_amd import tune
    rates = {(2048, 32): {"a": 10.0, "b": 6.0, "c": 9.0},
             (2048, 4): {"a": 1.0, "b": 2.0, "c": 3.0}}

    def fake(ctx, nwg, K, total, **kw):
        rows = [{"kind": k, "params": {"poll_sleep": 1}, "pairs_per_s": v,
                 "consistent": not (k == "c" and K == 4)}
                for k, v in rates[(nwg, K)].items()]
        return {"nwg": nwg, "K": K, "total": total, "candidates": rows}

    monkeypatch.setattr(tune, "tune_semaphore", fake)
    r = tune.tune_semaphore_points(None, [(2048, 32), (2048, 4)], 1024)
    by_kind = {row["kind"]: row for row in r["candidates"]}
    assert not by_kind["c"]["consistent"] and "pairs_per_s" not in by_kind["c"]
    assert by_kind["a"]["pairs_per_s"] == pytest.approx(math.sqrt(10.0))
    assert by_kind["b"]["pairs_per_s"] == pytest.approx(math.sqrt(12.0))
    assert r["best"]["kind"] == "b" and r["points"] == [[2048, 32], [2048, 4]]
