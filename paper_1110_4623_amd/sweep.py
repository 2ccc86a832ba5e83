"""Measurement sweeps over the primitives and the memory system, on one GPU.

  micro    the atomic / load / store grid of Section 3 widened to this GPU: operation x
           workgroups x targets x stride x issue mode, plus the derived ceilings (A1 the
           contended rate on one word, A_dist the best rate over a million words, the
           streaming read bandwidth and the cross-workgroup coherence latency);
  mutex    every mutex algorithm x 1..2048 workgroups x 1/16/256 locks x 1/16/256 words;
  barrier  every barrier x 256/1024/2048 co-resident workgroups x 10^4 rounds;
  sem      every semaphore x K in {1, 4, 32, 256} x 2048 workgroups;
  card     the machine abstraction of Section 4 from the twelve tests of Table 1.

Every point runs a short pilot, then the full operation count of the workload unless
that would take longer than the time budget, in which case the count is scaled down
(and recorded): spin locks under heavy contention hand over a few thousand times per
second, so their full counts would take minutes per point.  Each point also checks the
workload's own invariants (exact count sums, equal checksums across barriers, occupancy
at most K); the element-by-element parity against the CPU oracle is the test-suite's.

Usage: python -m paper_1110_4623_amd.sweep {micro,mutex,barrier,sem,card,all}
       [--out DIR] [--budget SECONDS] [--quick]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import abstraction, api

OPS = ["add", "cas", "exch", "ld", "st"]
NWGS = [1, 8, 64, 256, 1024, 2048]
TARGETS = [1, 32, 1024, 1 << 20]
STRIDES = [4, 64, 128]
MODES = ["per_lane", "wave_leader"]


def _log(*a):
    print(*a, flush=True)


def _scaled(full: int, pilot: int, pilot_ms: float, budget_s: float, floor: int) -> int:
    """Operation count that fits the budget, from a pilot of `pilot` operations."""
    per_op = max(pilot_ms, 1e-3) * 1e-3 / pilot
    return int(max(floor, min(full, budget_s / per_op * (1 + 1e-9))))


# ---- memory-system grid -------------------------------------------------------------------

def micro(ctx, budget_s: float = 0.15, lanes: int = 256, seed: int = 42, quick: bool = False):
    import sp_inputs
    rows = []
    nwgs = [1, 64, 2048] if quick else NWGS
    targets = [1, 1 << 20] if quick else TARGETS
    strides = [128] if quick else STRIDES
    buf = ctx.zeros((1 << 20) * 128 // 4)
    perms = {T: ctx.upload(sp_inputs.permutation(T, seed)) for T in targets}
    for op in OPS:
        for mode in MODES:
            per_issuer_full = 15625 if mode == "per_lane" else 10 ** 6  # 10^6 per wavefront
            for nwg in nwgs:
                issuers = nwg * lanes if mode == "per_lane" else nwg * (lanes // 64)
                for T in targets:
                    for stride in strides:
                        # c contenders on one word retry a compare-and-swap loop about
                        # c^2 / 2 times per round of successes: beyond ~4 x 10^8 attempts
                        # even one operation per issuer exceeds the watchdog
                        c = issuers / T
                        if op == "cas" and T * c * c / 2 > 4e8:
                            rows.append({"op": op, "mode": mode, "nwg": nwg, "T": T,
                                         "stride": stride, "skipped": "quadratic retries"})
                            continue
                        # pilot: one operation per lane, or 16 per wavefront leader
                        pilot = 1 if mode == "per_lane" else 16
                        try:
                            _, _, st = api.bench_atomic(ctx, op, nwg, lanes, T, stride, mode,
                                                        pilot, seed, perms[T], buf)
                        except api.N.SpTimeout:
                            rows.append({"op": op, "mode": mode, "nwg": nwg, "T": T,
                                         "stride": stride, "skipped": "pilot timed out"})
                            _log(f"micro {op} {mode} nwg={nwg} T={T} stride={stride}: timeout")
                            continue
                        n = _scaled(per_issuer_full, pilot, st["kernel_ms"], budget_s, 1)
                        fin, _, st = api.bench_atomic(ctx, op, nwg, lanes, T, stride, mode, n,
                                                      seed, perms[T], buf)
                        ops = issuers * n
                        secs = st["kernel_ms"] * 1e-3
                        ok = None
                        if op in ("add", "cas"):  # every increment lands exactly once
                            ok = int(fin.astype(np.uint64).sum() % (1 << 32)) == ops % (1 << 32)
                        payload = 4 if op in ("ld", "st") else 8
                        r = {"op": op, "mode": mode, "nwg": nwg, "T": T, "stride": stride,
                             "n_per_issuer": n, "ops": ops, "ms": st["kernel_ms"],
                             "ops_per_s": ops / secs, "GB_per_s": ops * payload / secs / 1e9,
                             "count_exact": ok}
                        rows.append(r)
                        _log(f"micro {op:4s} {mode:11s} nwg={nwg:5d} T={T:8d} stride={stride:3d} "
                             f"n={n:8d} {r['ops_per_s']:.3e} ops/s ok={ok}")
    return {"rows": rows, "ceilings": ceilings(ctx, rows)}


def fence_costs(ctx) -> dict:
    """Agent-scope fences alone (eight workgroups, one per XCD, one fence each after one
    dirty line; median of five runs) and when 2048 workgroups issue one each at once (span
    from the first start to the last end, and the slowest workgroup's fence)."""
    out = {}
    for kind in ("release", "acquire"):
        alone = [api.bench_fence(ctx, kind, 8, 64, reps=1, lines=1)["clk_per_fence_mean"]
                 for _ in range(5)]
        together = api.bench_fence(ctx, kind, 2048, 64, reps=1, lines=1)
        out[f"{kind}_alone_clk"] = float(np.median(alone))
        out[f"{kind}_2048_span_us"] = together["span_us"]
        out[f"{kind}_2048_max_clk"] = together["clk_per_fence_max"]
    return out


def signal_latencies(ctx, rounds: int = 20000) -> dict:
    """One-way latency of a signal between two workgroups (ns, token ping-pong): across
    XCDs and within one, relaxed agent-scope accesses only and with a release store and
    acquire fence per hand-over; plus where the two workgroups ran."""
    out = {}
    for fenced in (False, True):
        for same in (False, True):
            api.pingpong(ctx, 100, fenced=fenced, same_xcd=same)
            xcc, st = api.pingpong(ctx, rounds, fenced=fenced, same_xcd=same)
            key = ("fenced" if fenced else "relaxed") + ("_same_xcd" if same else "_cross_xcd")
            out[key + "_ns"] = st["kernel_ms"] * 1e6 / (2 * rounds)
            out[key + "_xcc"] = xcc[2:4]
    return out


def ceilings(ctx, rows) -> dict:
    """A1, A_dist, streaming read bandwidth, signal latencies and fence costs."""
    rows = [r for r in rows if "ops_per_s" in r]
    a1 = max((r for r in rows if r["T"] == 1 and r["op"] in ("add", "exch")),
             key=lambda r: r["ops_per_s"], default=None)
    ad = max((r for r in rows if r["T"] == 1 << 20 and r["stride"] == 128 and r["op"] in
              ("add", "exch")), key=lambda r: r["ops_per_s"], default=None)
    nbytes = 4 << 30
    buf = ctx.zeros(nbytes // 4)
    api.stream_read(ctx, buf, nbytes, 1)
    _, st = api.stream_read(ctx, buf, nbytes, 3)
    stream = 3 * nbytes / (st["kernel_ms"] * 1e-3) / 1e9
    # L2-resident: 16 MiB read by 2048 workgroups is 2 MiB per XCD (inside its 4 MB L2) and
    # 64 KiB per CU (beyond its 32 KiB L1)
    small = 16 << 20
    api.stream_read(ctx, buf, small, 5, nwg=2048)
    _, st = api.stream_read(ctx, buf, small, 200, nwg=2048)
    l2 = 200 * small / (st["kernel_ms"] * 1e-3) / 1e9
    del buf
    sig = signal_latencies(ctx)
    return {"A1_ops_per_s": a1 and a1["ops_per_s"], "A1_setting": a1 and
            {k: a1[k] for k in ("op", "mode", "nwg")},
            "A_dist_ops_per_s": ad and ad["ops_per_s"], "A_dist_setting": ad and
            {k: ad[k] for k in ("op", "mode", "nwg")},
            "stream_read_GB_per_s": stream, "l2_read_GB_per_s": l2,
            "coherence_latency_ns": sig["fenced_cross_xcd_ns"],
            "shader_clock_mhz": api.shader_clock_mhz(ctx), "signal_latency": sig,
            "fences": fence_costs(ctx)}


# ---- mutexes ------------------------------------------------------------------------------

MUTEX_VARIANTS = [("spin_cas", {}), ("spin_backoff", {"backoff": "exp"}),
                  ("spin_backoff", {"backoff": "paper"}), ("ticket", {}), ("sleep", {}),
                  ("ring", {}), ("array", {}), ("adaptive", {}), ("cohort", {}), ("mcs", {}),
                  ("cu_cohort", {})]


def mutex(ctx, budget_s: float = 0.3, lanes: int = 256, seed: int = 42, quick: bool = False,
          limit_ms: int = 8000):
    rows = []
    nwgs = [1 << i for i in range(12)]
    if quick:
        nwgs = [1, 64, 2048]
    full = 1 << 20
    for kind, params in MUTEX_VARIANTS:
        for L in (1, 16, 256):
            for W in (1, 16, 256):
                if quick and (L, W) not in ((1, 16), (256, 1)):
                    continue
                m = api.Mutex(ctx, kind, L, W, timeout_ms=limit_ms, **params)
                try:
                    for nwg in nwgs:
                        pilot = max(nwg, 256)
                        try:
                            _, st, _ = m.run(nwg, lanes, pilot, 1000, seed)
                        except api.N.SpTimeout:
                            rows.append({"kind": kind, "params": params, "L": L, "W": W,
                                         "nwg": nwg, "total": pilot, "timeout_ms": limit_ms,
                                         "acq_per_s_below": pilot / (limit_ms * 1e-3)})
                            _log(f"mutex {kind} {params} L={L} W={W} nwg={nwg}: pilot of "
                                 f"{pilot} exceeded {limit_ms} ms")
                            continue
                        total = _scaled(full, pilot, st["kernel_ms"], budget_s, nwg)
                        words, st, fin = m.run(nwg, lanes, total, 1000, seed, finish=True)
                        ok = bool((words == words[:, :1]).all() and int(words[:, 0].sum()) == total)
                        # fairness: spread of the workgroups' finishing times relative to the
                        # run (0 = all finish together)
                        span = float(fin.max() - fin.min())
                        dur = st["kernel_ms"] * ctx.info["wall_clock_khz"]
                        r = {"kind": kind, "params": params, "L": L, "W": W, "nwg": nwg,
                             "total": total, "ms": st["kernel_ms"],
                             "acq_per_s": total / (st["kernel_ms"] * 1e-3), "count_exact": ok,
                             "finish_spread": span / dur if dur else 0.0}
                        rows.append(r)
                        _log(f"mutex {kind:12s} {params} L={L:3d} W={W:3d} nwg={nwg:5d} "
                             f"total={total:8d} {r['acq_per_s']:.3e} acq/s ok={ok}")
                finally:
                    m.close()
    return {"rows": rows}


# ---- barriers -----------------------------------------------------------------------------

BARRIERS = ["central", "central_split", "tree", "flag", "xcd", "grid_sync"]


def barrier(ctx, rounds: int = 10_000, lanes: int = 256, seed: int = 42, quick: bool = False):
    rows = []
    for N in ((256, 2048) if quick else (256, 1024, 2048)):
        chks = {}
        for kind in BARRIERS:
            b = api.Barrier(ctx, kind, N)
            try:
                b.run_hash(lanes, 100, seed)
                chk, st = b.run_hash(lanes, rounds, seed)
                # the same kernel and grid with zero rounds: what the launch itself costs
                empty_ms = b.launch(lanes, 0, seed)["kernel_ms"]
            finally:
                b.close()
            chks[kind] = chk.tobytes()
            us = st["kernel_ms"] * 1e3 / rounds
            rows.append({"kind": kind, "nwg": N, "rounds": rounds, "us_per_round": us,
                         "empty_launch_us": empty_ms * 1e3,
                         "us_per_round_minus_empty_launch":
                             (st["kernel_ms"] - empty_ms) * 1e3 / rounds,
                         "arrivals_per_s": N * rounds / (st["kernel_ms"] * 1e-3)})
            _log(f"barrier {kind:13s} N={N:5d} {us:8.2f} us/round (empty launch "
                 f"{empty_ms * 1e3:.1f} us)")
        for kind in ("launch", "graph"):
            chk, st = api.barrier_hash_launches(ctx, N, lanes, rounds, seed, graph=kind == "graph")
            chks[kind] = chk.tobytes()
            us = st["kernel_ms"] * 1e3 / rounds
            rows.append({"kind": f"kernel_boundary_{kind}", "nwg": N, "rounds": rounds,
                         "us_per_round": us,
                         "arrivals_per_s": N * rounds / (st["kernel_ms"] * 1e-3)})
            _log(f"barrier boundary-{kind:6s} N={N:5d} {us:8.2f} us/round")
        agree = len(set(chks.values())) == 1
        for r in rows:
            if r["nwg"] == N:
                r["checksums_agree"] = agree
    return {"rows": rows}


# ---- semaphores ---------------------------------------------------------------------------

# Algorithm 4 with backoff: waiters back off exponentially up to 8192 s_sleep units and
# posts retry at once, the form that runs the full configuration
SEMS = [("spin", {}), ("spin_backoff", {"backoff": "exp", "backoff_max": 8192, "post_backoff": 0}),
        ("ticket", {}), ("sleep", {}),
        ("counters", {}), ("adaptive", {}), ("cohort", {}), ("array", {}),
        ("chain", {}), ("xcd_chain", {}), ("cu_lock", {})]


def sem(ctx, budget_s: float = 0.3, nwg: int = 2048, lanes: int = 256, seed: int = 42,
        quick: bool = False, limit_ms: int = 8000):
    rows = []
    full = 1 << 20
    for kind, params in SEMS:
        for K in ((4, 256) if quick else (1, 4, 32, 256)):
            try:
                s = api.Semaphore(ctx, kind, K, timeout_ms=limit_ms, **params)
            except api.N.SpError as e:  # K outside the kind's range
                rows.append({"kind": kind, "params": params, "K": K, "nwg": nwg,
                             "refused": str(e)})
                continue
            try:
                pilot = nwg
                try:
                    r0 = s.run(nwg, lanes, pilot, 2000, seed, track=True)
                except api.N.SpTimeout:
                    rows.append({"kind": kind, "params": params, "K": K, "nwg": nwg,
                                 "total": pilot, "timeout_ms": limit_ms,
                                 "pairs_per_s_below": pilot / (limit_ms * 1e-3)})
                    _log(f"sem {kind} K={K}: pilot of {pilot} pairs exceeded {limit_ms} ms")
                    continue
                total = _scaled(full, pilot, r0["stats"]["kernel_ms"], budget_s, nwg)
                try:
                    checked = s.run(nwg, lanes, total, 2000, seed, track=True)
                    timed = s.run(nwg, lanes, total, 2000, seed, track=False)
                except api.N.SpTimeout:  # slower at the full count than the pilot said
                    total, checked = pilot, r0
                    try:
                        timed = s.run(nwg, lanes, total, 2000, seed, track=False)
                    except api.N.SpTimeout:  # the pilot's count too, this time
                        rows.append({"kind": kind, "params": params, "K": K, "nwg": nwg,
                                     "total": pilot, "timeout_ms": limit_ms,
                                     "pairs_per_s_below": pilot / (limit_ms * 1e-3)})
                        _log(f"sem {kind} K={K}: {pilot} pairs exceeded {limit_ms} ms")
                        continue
            finally:
                s.close()
            ok = checked["state"][3] == total and 1 <= checked["maxocc"] <= K
            r = {"kind": kind, "params": params, "K": K, "nwg": nwg, "total": total,
                 "pairs_per_s": total / (timed["stats"]["kernel_ms"] * 1e-3),
                 "pairs_per_s_tracked": total / (checked["stats"]["kernel_ms"] * 1e-3),
                 "maxocc": checked["maxocc"], "invariants_ok": bool(ok)}
            rows.append(r)
            _log(f"sem {kind:12s} K={K:4d} total={total:8d} {r['pairs_per_s']:.3e} pairs/s "
                 f"maxocc={r['maxocc']} ok={ok}")
    return {"rows": rows}


# ---- machine card ---------------------------------------------------------------------------

def card(ctx, quick: bool = False):
    out = {}
    for nwg in ((256,) if quick else (256, 2048)):
        times = abstraction.measure(ctx, nwg)
        out[str(nwg)] = {"times_ms": times, "card": abstraction.card(times)}
        c = out[str(nwg)]["card"]
        _log(f"card nwg={nwg}: atomic/volatile {c['atomic_to_volatile']} "
             f"cont/noncont volatile {c['contentious_to_noncontentious_volatile']} "
             f"hostage {c['volatile_after_atomic_to_volatile']}")
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("what", choices=["micro", "mutex", "barrier", "sem", "card", "all"])
    ap.add_argument("--out", default=".")
    ap.add_argument("--budget", type=float, default=None, help="seconds per point")
    ap.add_argument("--quick", action="store_true")
    a = ap.parse_args(argv)
    ctx = api.Context(0)
    todo = ["card", "barrier", "sem", "mutex", "micro"] if a.what == "all" else [a.what]
    os.makedirs(a.out, exist_ok=True)
    for w in todo:
        t = time.time()
        kw = {"quick": a.quick}
        if a.budget is not None and w in ("micro", "mutex", "sem"):
            kw["budget_s"] = a.budget
        res = {"micro": micro, "mutex": mutex, "barrier": barrier, "sem": sem,
               "card": card}[w](ctx, **kw)
        res["device"] = ctx.info
        path = os.path.join(a.out, f"sweep_{w}.json")
        with open(path, "w") as f:
            json.dump(res, f, indent=1, default=str)
        _log(f"== {w} done in {time.time() - t:.1f} s -> {path}")
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
