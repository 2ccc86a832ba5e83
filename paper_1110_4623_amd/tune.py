"""Autotuner: picks each primitive's algorithm and parameters per contention level.

Section 7 proposes tuning the backoff parameters for each GPU under differing levels of
contention.  This tuner widens that to every choice the library exposes: for barriers the
algorithm, the tree's fan-in, flag packing, the per-XCD barrier's stamp copies and the
polling sleep; for mutexes and semaphores the algorithm, the backoff policy and bounds,
and the polling sleep; for the serving queue the polling sleeps and the number of
persistent workgroups.  Each candidate runs a short representative workload through libsp
(barrier, mutex and semaphore candidates are recorded into a HIP graph once and timed over
replays); the fastest candidate whose results pass the workload's own consistency checks
wins (semaphores: the best geometric mean over two K of the bucket).  The winners
are installed with sp_set_default, so that the *_DEFAULT kinds resolve to them, and can
be saved to and loaded from a JSON cache keyed by the device.

Contention buckets follow the library: bucket 0 has fewer than 64 workgroups per
resource (per barrier, per lock, per K semaphore units), bucket 1 has 64 or more.
"""

from __future__ import annotations

import json
import math
import os

import numpy as np

from . import api

BUCKET_SPLIT = 64
LIMIT_MS = 3000  # watchdog of every tuning run: a slower candidate is rejected


def _median(xs):
    return float(np.median(np.asarray(xs, dtype=np.float64)))


def _graph_time(ctx, record, replays: int) -> float:
    """Records `record()` into a graph and returns ms per replay (median of 3 launches)."""
    g = api.Graph(ctx)
    with g:
        record()
    try:
        g.launch(1)  # warm-up
        ms = [g.launch(replays)["kernel_ms"] / replays for _ in range(3)]
    finally:
        g.close()
    return _median(ms)


# ---- barriers ---------------------------------------------------------------------------

def barrier_candidates():
    out = [("central", {}), ("central_split", {}),
           ("flag", {"flags_packed": 0}), ("flag", {"flags_packed": 1})]
    out += [("xcd", {"xcd_copies": c}) for c in (0, 8, 64, 256)]
    out += [("tree", {"fan_in": f}) for f in (4, 8, 16, 32)]
    return [(k, dict(p, poll_sleep=ps)) for k, p in out for ps in (0, 1, 4)]


def tune_barrier(ctx, nwg: int, lanes: int = 256, rounds: int = 1000, seed: int = 42,
                 candidates=None, limit_ms: int = LIMIT_MS) -> dict:
    """Times every candidate barrier on the hash exchange among nwg workgroups.  The
    checksums are deterministic, so every correct candidate returns the same ones; a
    candidate that disagrees with the majority is rejected."""
    rows = []
    for kind, params in candidates or barrier_candidates():
        b = api.Barrier(ctx, kind, nwg, timeout_ms=limit_ms, **params)
        try:
            ms = _graph_time(ctx, lambda: b.launch(lanes, rounds, seed), 2)
            chk = b.checksums()
        except api.N.SpError as e:  # not co-resident, or slower than the limit
            rows.append({"kind": kind, "params": params, "error": str(e)})
            continue
        finally:
            b.close()
        rows.append({"kind": kind, "params": params, "us_per_round": ms * 1e3 / rounds,
                     "chk": chk.tobytes()})
    ok = [r for r in rows if "chk" in r]
    if not ok:
        raise RuntimeError("no barrier candidate ran")
    votes: dict[bytes, int] = {}
    for r in ok:
        votes[r["chk"]] = votes.get(r["chk"], 0) + 1
    majority = max(votes, key=votes.get)
    for r in ok:
        r["consistent"] = r["chk"] == majority
        del r["chk"]
    best = min((r for r in ok if r["consistent"]), key=lambda r: r["us_per_round"])
    return {"nwg": nwg, "lanes": lanes, "rounds": rounds, "best": best, "candidates": rows}


# ---- mutexes ------------------------------------------------------------------------------

def mutex_candidates():
    out = [("spin_cas", {}), ("spin_exch", {})]
    for policy in ("exp", "paper"):
        for imax in (8, 32, 128):
            out.append(("spin_backoff", {"backoff": policy, "backoff_min": 1, "backoff_max": imax}))
    out += [("ticket", {"poll_sleep": ps}) for ps in (0, 1, 4)]
    out += [("sleep", {"poll_sleep": ps}) for ps in (1, 4, 16)]
    out += [("array", {"poll_sleep": ps}) for ps in (0, 1, 4)]
    out += [("ring", {"poll_sleep": 0}), ("adaptive", {})]
    out += [("mcs", {"poll_sleep": ps}) for ps in (0, 1)]
    out += [("cohort", {"poll_sleep": ps, "cohort_passes": cp}) for ps in (0, 4)
            for cp in (16, 64)]
    out += [("cu_cohort", {"poll_sleep": 0, "cohort_passes": cp}) for cp in (16, 64)]
    return out


def tune_mutex(ctx, nwg: int, nlocks: int = 1, words: int = 16, total: int = 4096,
               max_delay: int = 1000, lanes: int = 256, seed: int = 42, candidates=None,
               limit_ms: int = LIMIT_MS) -> dict:
    """Times every candidate mutex on the contention workload.  With one lock every
    critical-section word must end at exactly `total`; with several, every lock's words
    must agree and sum to `total`."""
    rows = []
    for kind, params in candidates or mutex_candidates():
        m = api.Mutex(ctx, kind, nlocks, words, timeout_ms=limit_ms, **params)
        try:
            # one eager run first: queue mutexes size their slots on first use, which a
            # graph recording cannot do
            m.launch(nwg, lanes, nwg, 0, seed)
            ms = _graph_time(ctx, lambda: m.launch(nwg, lanes, total, max_delay, seed), 1)
            w = m.words()
        except api.N.SpError as e:
            rows.append({"kind": kind, "params": params, "error": str(e), "consistent": False})
            continue
        finally:
            m.close()
        ok = bool((w == w[:, :1]).all() and int(w[:, 0].sum()) == total)
        rows.append({"kind": kind, "params": params, "acq_per_s": total / (ms * 1e-3),
                     "consistent": ok})
    best = max((r for r in rows if r["consistent"]), key=lambda r: r["acq_per_s"])
    return {"nwg": nwg, "nlocks": nlocks, "total": total, "best": best, "candidates": rows}


def tune_mutex_points(ctx, points, total: int, **kw) -> dict:
    """tune_mutex at several (nwg, nlocks) points of one contention bucket; the best
    geometric mean of acquisitions/s wins (the cohort lock, for one, pays a round trip
    when uncontended and gains from a few contenders on)."""
    runs = [tune_mutex(ctx, nwg, nlocks, total=total, **kw) for nwg, nlocks in points]
    best, rows = _combine_points(runs, "acq_per_s")
    return {"points": [list(p) for p in points], "total": total, "best": best,
            "candidates": rows}


# ---- semaphores ---------------------------------------------------------------------------

def semaphore_candidates():
    out = [("spin", {})]
    # Algorithm 4: the waiters' backoff cap, and whether post backs off too (the listing)
    # or retries at once (Section 5's prose); caps up to 8192 units keep 2048 waiters
    # from holding the word S busy
    for imax in (32, 1024, 8192):
        for pb in (0, 1):
            out.append(("spin_backoff", {"backoff": "exp", "backoff_min": 1, "backoff_max": imax,
                                         "post_backoff": pb}))
    out.append(("spin_backoff", {"backoff": "paper", "backoff_min": 1, "backoff_max": 32,
                                 "post_backoff": 0}))
    out += [("ticket", {"poll_sleep": 0})]
    out += [("sleep", {"poll_sleep": ps}) for ps in (1, 4, 16)]
    out += [("counters", {"poll_sleep": ps}) for ps in (0, 1, 4, 16, 64)]
    out += [("adaptive", {"poll_sleep": ps}) for ps in (0, 1, 4)]
    out += [("cohort", {"poll_sleep": ps, "cohort_passes": cp}) for ps in (0, 4)
            for cp in (16, 64)]
    out += [("array", {"poll_sleep": ps}) for ps in (0, 1, 4)]
    out += [("chain", {"poll_sleep": ps}) for ps in (0, 1, 4)]
    out += [("xcd_chain", {"poll_sleep": ps}) for ps in (0, 1, 4)]
    return out


def tune_semaphore(ctx, nwg: int, K: int, total: int = 8192, max_hold: int = 2000,
                   lanes: int = 256, seed: int = 42, candidates=None,
                   limit_ms: int = LIMIT_MS) -> dict:
    """Times every candidate semaphore on the wait/post workload; a candidate must admit
    exactly `total` times and never hold more than K."""
    rows = []
    for kind, params in candidates or semaphore_candidates():
        try:
            s = api.Semaphore(ctx, kind, K, timeout_ms=limit_ms, **params)
        except api.N.SpError:
            # outside the kind's range of K (the per-XCD chains need a unit per XCD):
            # time what a default semaphore naming it would run, the one-chain kind
            if kind != "xcd_chain":
                raise
            s = api.Semaphore(ctx, "chain", K, timeout_ms=limit_ms, **params)
        try:
            # checked with the occupancy tracked, timed without it: tracking adds three
            # contended atomics per pair, which cap the fastest kinds near A1 / 3
            s.launch(nwg, lanes, total, max_hold, seed, track=True)
            r = s.result()
            ms = _graph_time(ctx, lambda: s.launch(nwg, lanes, total, max_hold, seed,
                                                   track=False), 1)
        except api.N.SpError as e:
            rows.append({"kind": kind, "params": params, "error": str(e), "consistent": False})
            continue
        finally:
            s.close()
        ok = r["state"][3] == total and 1 <= r["maxocc"] <= K
        rows.append({"kind": kind, "params": params, "pairs_per_s": total / (ms * 1e-3),
                     "consistent": bool(ok)})
    best = max((r for r in rows if r["consistent"]), key=lambda r: r["pairs_per_s"])
    return {"nwg": nwg, "K": K, "total": total, "best": best, "candidates": rows}


def _combine_points(runs, key: str) -> tuple:
    """Candidates correct at every point, ranked by the geometric mean of `key`."""
    keyed = {}
    for run in runs:
        for r in run["candidates"]:
            keyed.setdefault((r["kind"], json.dumps(r["params"], sort_keys=True)), []).append(r)
    rows = []
    for (kind, _), rs in keyed.items():
        ok = len(rs) == len(runs) and all(r["consistent"] for r in rs)
        row = {"kind": kind, "params": rs[0]["params"], "consistent": ok}
        if ok:
            row["points_" + key] = [r[key] for r in rs]
            row[key] = math.exp(sum(math.log(v) for v in row["points_" + key]) / len(rs))
        rows.append(row)
    best = max((r for r in rows if r["consistent"]), key=lambda r: r[key])
    return best, rows


def tune_semaphore_points(ctx, points, total: int, **kw) -> dict:
    """Times every candidate at several (nwg, K) points of one contention bucket and keeps
    the best geometric mean of pairs/s among the candidates correct at every point (a
    bucket spans many K, and the best waiting policy depends on K)."""
    runs = [tune_semaphore(ctx, nwg, K, total=total, **kw) for nwg, K in points]
    best, rows = _combine_points(runs, "pairs_per_s")
    return {"points": [list(p) for p in points], "total": total, "best": best,
            "candidates": rows}


# ---- serving queue ----------------------------------------------------------------------

def tune_serve(ctx, reqs: dict, seed: int = 42, budget_units: int = 16384,
               unit_bytes: int = 65536, candidates=None) -> dict:
    """Runs the request stream with each candidate configuration of the persistent queue
    and keeps the one with the lowest p99 latency; every candidate must return the same
    per-request results."""
    cands = candidates or [dict(nwg=nwg, poll_sleep=ps, far_sleep=fs)
                           for nwg in (256, 1024) for ps in (0, 2) for fs in (1, 4, 16)]
    rows, ref = [], None
    for c in cands:
        out, _, res = api.serve(ctx, reqs, seed=seed, budget_units=budget_units,
                                unit_bytes=unit_bytes, **c)
        if ref is None:
            ref = out
        rows.append({"cfg": c, "p50_us": res["p50_us"], "p99_us": res["p99_us"],
                     "req_per_s": res["req_per_s"], "consistent": bool((out == ref).all())})
    best = min((r for r in rows if r["consistent"]), key=lambda r: r["p99_us"])
    return {"n": int(len(reqs["L"])), "best": best, "candidates": rows}


# ---- whole tuning pass, cache, installation ------------------------------------------------

def device_key(ctx) -> str:
    i = ctx.info
    return f"{i['arch']}/{i['cu_count']}cu/{i['xcd_count']}xcd"


def tune_all(ctx, quick: bool = False) -> dict:
    """Tunes barriers (16 and 1024 workgroups), mutexes (bucket 0: one lock at 4 and 32
    workgroups; bucket 1: one lock at 1024, 16 locks at 2048) and semaphores (bucket 0:
    K = 32 at 256 workgroups and K = 256 at 2048; bucket 1: K = 32 and K = 4 at 2048)."""
    rounds = 300 if quick else 1000
    mt = 1024 if quick else 4096
    res = {"device": device_key(ctx), "barrier": {}, "mutex": {}, "semaphore": {}}
    res["barrier"]["0"] = tune_barrier(ctx, 16, rounds=rounds)
    res["barrier"]["1"] = tune_barrier(ctx, 1024, rounds=rounds)
    res["mutex"]["0"] = tune_mutex_points(ctx, [(4, 1), (32, 1)], mt)
    res["mutex"]["1"] = tune_mutex_points(ctx, [(1024, 1), (2048, 16)], mt)
    # 128 waits per workgroup at 2048: the queues reach their steady state (with 32 the
    # cohort semaphore measured 9.6 M pairs/s at K = 256 and 2048 workgroups, with 128
    # 4.8) and the adaptive kind has learned its interval
    res["semaphore"]["0"] = tune_semaphore_points(ctx, [(256, 32), (2048, 256)], 64 * mt)
    res["semaphore"]["1"] = tune_semaphore_points(ctx, [(2048, 32), (2048, 4)], 64 * mt)
    return res


def apply(ctx, tuned: dict) -> None:
    """Installs the winners as the library's defaults for this context."""
    if tuned.get("device") not in (None, device_key(ctx)):
        raise ValueError(f"tuning for {tuned['device']} does not match {device_key(ctx)}")
    for prim in ("barrier", "mutex", "semaphore"):
        for bucket, r in tuned.get(prim, {}).items():
            best = r["best"]
            ctx.set_default(prim, int(bucket), best["kind"], **best["params"])


def save(tuned: dict, path: str) -> None:
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "w") as f:
        json.dump(tuned, f, indent=1)


def load(path: str) -> dict:
    with open(path) as f:
        return json.load(f)


def default_cache_path() -> str:
    return os.environ.get("SP_TUNER_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "paper_1110_4623_amd",
                                       "tuner.json"))


def main(argv=None) -> int:
    """python -m paper_1110_4623_amd.tune [--out PATH] [--quick] [--serve-rate R]:
    tunes every primitive on this GPU, prints the winners, saves the cache."""
    import argparse
    import sys
    ap = argparse.ArgumentParser(description="tune the synchronization primitives")
    ap.add_argument("--out", default=None, help="cache path (default: SP_TUNER_CACHE or "
                                                "~/.cache/paper_1110_4623_amd/tuner.json)")
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--serve-rate", type=float, default=0.0,
                    help="also tune the serving queue at this arrival rate (req/s)")
    a = ap.parse_args(argv)
    ctx = api.Context(0)
    res = tune_all(ctx, quick=a.quick)
    if a.serve_rate > 0:
        import sp_inputs
        n = int(max(2e4, 2 * a.serve_rate)) if not a.quick else 5000
        res["serve"] = tune_serve(ctx, sp_inputs.request_table(n, a.serve_rate, 42))
    for prim in ("barrier", "mutex", "semaphore"):
        for bucket, r in res[prim].items():
            b = r["best"]
            metric = {k: v for k, v in b.items() if k.endswith("_per_s") or k.startswith("us_")}
            print(f"{prim:9s} bucket {bucket}: {b['kind']:13s} {b['params']} {metric}",
                  flush=True)
    if "serve" in res:
        b = res["serve"]["best"]
        print(f"serve: {b['cfg']} p50 {b['p50_us']:.1f} us p99 {b['p99_us']:.1f} us", flush=True)
    path = a.out or default_cache_path()
    save(res, path)
    print(f"saved {path}", flush=True)
    ctx.close()
    sys.stdout.flush()
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
