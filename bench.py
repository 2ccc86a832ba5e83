"""Benchmark of the synchronization hot path on one MI355X.

One step runs the whole path once over the full-size synthetic workloads:

  1. contended-atomic ceiling: 2048 workgroups x 4 wavefront leaders add 1 to one word
     (the A1 ceiling the barrier and lock figures are compared with);
  2. barrier: the per-XCD barrier, 2048 co-resident workgroups x 256 lanes x 10^4
     rounds of the hash exchange (the headline: microseconds per barrier round);
  3. mutex: ticket lock (Algorithm 3), 2048 workgroups x 256 lanes, one lock guarding 16
     words, 2^20 acquisitions with non-critical delays uniform in [0, 1000] cycles, then
     the same workload on the library's default mutex for this contention (the CU-cohort
     lock);
  4. semaphore: fetch-and-add semaphore (Algorithm 5 with s_sleep polling) with K = 32,
     2048 workgroups, 2^20 wait/post pairs holding uniform [0, 2000] cycles, then the
     same workload on the library's default semaphore for this contention (per-XCD
     chains: the units split over the XCDs, each holder granting the ticket K_x after its
     own on its XCD without an L2 writeback);
  5. serving: 2 x 10^5 requests arriving as a Poisson stream at 10^5 req/s (lognormal
     hash-chain lengths, 1 GiB workspace budget in 64 KiB units), drained by 1024
     persistent workgroups, then the same stream served with one kernel launch per
     request over four streams (the comparator); p50/p99 latency of both.

Every step also times the kernel-boundary comparator: one launch per round of the same
hash exchange, 10^4 + 1 launches replayed from one HIP graph.

Prints one JSON line.  `value` is microseconds per barrier round (lower is better), the
mean over the timed steps (the figure a kernel trace's average duration gives); the
median and minimum ride along with the other primitives' throughputs in `metrics`, and
`env` records the device, its clock, the occupancy and the build.

The process does not import PyTorch: the library binds to the system ROCm runtime and
allocates its buffers itself (SP_NO_TORCH), which is also what rocprofv3 profiles.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
os.environ.setdefault("SP_NO_TORCH", "1")

METRIC = "µs/barrier round, mutex & semaphore ops/s vs #WGs; persistent-queue p99 latency"
NWG, LANES, ROUNDS = 2048, 256, 10_000
C1_NWG, C1_LANES, C1_ROUNDS = 16, 64, 1000
AB_ROUNDS = 2000  # the split central barrier against A1 (outside the timed region)
MUTEX_TOTAL, SEM_TOTAL, SEM_K = 1 << 20, 1 << 20, 32
CURVE_NWG, CURVE_OPS = (64, 256, 1024), 1 << 18
SEM_KS = (1, 4, 32, 256)
# read-modify-writes per wait/post pair on each semaphore kind's busiest contended word
SEM_RMW_PER_PAIR = {"spin": 4, "spin_backoff": 4, "ticket": 2, "sleep": 2, "cohort": 2,
                    "counters": 1, "adaptive": 1, "array": 1, "chain": 1, "xcd_chain": 1,
                    "cu_lock": 1}
SERVE_RATE, SERVE_N, SERVE_NWG = 1e5, 200_000, 1024


def measured_traffic(kernel_sources_dir: str) -> float | None:
    """HBM bytes per launch of the barrier kernel from the committed rocprofv3 counter
    runs, if the kernel's sources are unchanged since those counters were taken."""
    import hashlib
    path = os.path.join(kernel_sources_dir, "profiles", "hbm_bytes_barrier_xcd_2048wg.json")
    try:
        rec = json.load(open(path))
        h = hashlib.sha256()
        for src in rec["sources"]:
            with open(os.path.join(kernel_sources_dir, src), "rb") as f:
                h.update(f.read())
        if h.hexdigest() != rec["sources_sha256"]:
            return None
        return rec["read_bytes_per_launch"] + rec["write_bytes_per_launch"]
    except (OSError, KeyError, ValueError):
        return None


def cpu_baseline(headline_chk, config1_chk, curve_out=None, budget_s: float = 20.0,
                 atomic_chk=None, sem_k_chk=None) -> dict:
    """The CPU oracle on this host, and the check of this run's barrier checksums against
    it (both outside the timed region).

    Timing: the threaded oracle (one std::thread per workgroup) running the per-XCD flag
    protocol with 2048 agents in 8 groups on the same hash exchange -- all the rounds of
    the workload when they fit the time budget, else the number that does.  Check: the
    closed form of the hash exchange for the headline configuration (2048 x 10^4, seed 42)
    and for the 16-workgroup, 1000-round configuration, element by element; and every
    result of the curves against #WGs (barrier checksums, mutex words, semaphore
    admission checksums) against its closed form."""
    import oracle
    oracle.lib()
    probe_rounds = 256
    _, rc, secs = oracle.barrier_threaded("xcd", 42, NWG, probe_rounds, groups=8)
    rounds = max(probe_rounds, min(ROUNDS, int(budget_s / max(secs, 1e-6) * probe_rounds)))
    _, rc2, secs2 = oracle.barrier_threaded("xcd", 42, NWG, rounds, groups=8)
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    t_closed = time.perf_counter()
    ref = oracle.barrier_closed(42, NWG, ROUNDS)
    t_closed = time.perf_counter() - t_closed  # the closed form: ground truth, not a baseline
    ref1 = oracle.barrier_closed(42, C1_NWG, C1_ROUNDS)
    atomic_ok = None
    if atomic_chk is not None:
        atomic_ok = bool((atomic_chk == oracle.barrier_closed(42, NWG, AB_ROUNDS)).all())
    sem_k_ok = None
    if sem_k_chk is not None:
        want = oracle.sem_closed(42, NWG, CURVE_OPS)
        sem_k_ok = all(bool((c == want).all()) for c in sem_k_chk.values())
    curves_ok = None
    if curve_out is not None:
        curves_ok = True
        for nwg, (bchk, words, schk) in curve_out.items():
            curves_ok &= bool((bchk == oracle.barrier_closed(42, nwg, ROUNDS)).all())
            curves_ok &= bool((words == oracle.mutex_closed(42, nwg, CURVE_OPS, 1, 16)).all())
            curves_ok &= bool((schk == oracle.sem_closed(42, nwg, CURVE_OPS)).all())
    return {"value": secs2 * 1e6 / rounds, "unit": "µs/round", "cores": cores,
            "kind": "oracle", "threads": NWG,
            "sample": f"per-XCD flag protocol, {NWG} std::thread agents (8 groups of 4 CUs), "
                      f"{rounds} of the {ROUNDS} rounds of the hash exchange; {secs2:.1f} s",
            "ok": rc == 0 and rc2 == 0,
            "closed_form_seconds": round(t_closed, 4),
            "headline_checksums_match_oracle": bool((headline_chk == ref).all()),
            "config1_checksums_match_oracle": bool((config1_chk == ref1).all()),
            "curves_match_oracle": curves_ok,
            "atomic_barrier_checksums_match_oracle": atomic_ok,
            "semaphore_vs_K_checksums_match_oracle": sem_k_ok}


def environment(ctx, resident_per_cu: int) -> dict:
    """Device, runtime and build the figures were taken with."""
    from paper_1110_4623_amd import build
    try:
        rocm = open("/opt/rocm/.info/version").read().strip()
    except OSError:
        rocm = None
    return {"device": ctx.info["name"] or None, "arch": ctx.info["arch"], "cus": ctx.info["cu_count"],
            "xcds": ctx.info["xcd_count"], "peak_shader_clock_mhz": ctx.info["clock_khz"] / 1e3,
            "barrier_resident_workgroups_per_cu": int(resident_per_cu), "rocm": rocm,
            "hipcc_flags": " ".join(os.path.relpath(f, ROOT) if os.path.isabs(f) else f
                                    for f in build.CFLAGS)}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--barrier", default="xcd")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the primitives synchronize workgroups of a single "
              f"device and there is no multi-GPU path (--gpus {args.gpus} requested)",
              file=sys.stderr)
        return 2

    import numpy as np

    import paper_1110_4623_amd as sp
    import sp_inputs
    from paper_1110_4623_amd import abstraction

    ctx = sp.Context(0)
    bar = sp.Barrier(ctx, args.barrier, NWG)
    # the same barrier for data exchanged with agent-scope accesses: no cache maintenance
    bar_coh = sp.Barrier(ctx, args.barrier, NWG, coherent_cs=1)
    mtx = sp.Mutex(ctx, "ticket", 1, 16)
    mtx_def = sp.Mutex(ctx, "default", 1, 16)
    sem = sp.Semaphore(ctx, "sleep", SEM_K)
    sem_def = sp.Semaphore(ctx, "default", SEM_K)
    perm1 = ctx.zeros(1)
    abuf = ctx.zeros(64)
    reqs = sp_inputs.request_table(SERVE_N, SERVE_RATE, 42)

    def step():
        r = {}
        _, _, st = sp.bench_atomic(ctx, "add", NWG, LANES, 1, 4, "wave_leader", 100, 42, perm1, abuf)
        r["a1_ms"], r["a1_ops"] = st["kernel_ms"], st["ops"]
        chk, st = bar.run_hash(LANES, ROUNDS, 42)
        r["bar_ms"], r["bar_chk"], r["bar_occ"] = st["kernel_ms"], chk, st["resident_per_cu"]
        chk_k, st_k = sp.barrier_hash_launches(ctx, NWG, LANES, ROUNDS, 42, graph=True)
        r["bar_kb_ms"], r["bar_kb_same"] = st_k["kernel_ms"], bool((chk_k == chk).all())
        chk_c, st_c = bar_coh.run_hash(LANES, ROUNDS, 42)
        r["bar_coh_ms"], r["bar_coh_same"] = st_c["kernel_ms"], bool((chk_c == chk).all())
        words, st, _ = mtx.run(NWG, LANES, MUTEX_TOTAL, 1000, 42)
        r["mtx_ms"], r["mtx_ok"] = st["kernel_ms"], bool((words == MUTEX_TOTAL).all())
        words_d, st_d, _ = mtx_def.run(NWG, LANES, MUTEX_TOTAL, 1000, 42)
        r["mtx_def_ms"] = st_d["kernel_ms"]
        r["mtx_ok"] = r["mtx_ok"] and bool((words_d == MUTEX_TOTAL).all())
        res = sem.run(NWG, LANES, SEM_TOTAL, 2000, 42, track=False)
        r["sem_ms"] = res["stats"]["kernel_ms"]
        r["sem_ok"] = res["state"][3] == SEM_TOTAL and res["state"][0] == 0
        res_d = sem_def.run(NWG, LANES, SEM_TOTAL, 2000, 42, track=False)
        r["sem_def_ms"] = res_d["stats"]["kernel_ms"]
        r["sem_def_ok"] = res_d["state"][3] == SEM_TOTAL and bool(
            (res_d["chk"] == res["chk"]).all())
        out_p, _, rp = sp.serve(ctx, reqs, nwg=SERVE_NWG, seed=42)
        out_l, _, rl = sp.serve_launch_per_request(ctx, reqs, seed=42, streams=4)
        r["serve"], r["serve_launch"] = rp, rl
        r["serve_same"] = bool((out_p == out_l).all())
        return r

    for _ in range(args.warmup):
        step()
    ctx.synchronize()  # every library call returns after its kernels finished
    clock_before = sp.shader_clock_mhz(ctx)
    t0 = time.perf_counter()
    results = [step() for _ in range(args.steps)]
    ctx.synchronize()
    wall = time.perf_counter() - t0
    clock_after = sp.shader_clock_mhz(ctx)
    # ---- outside the timed region ------------------------------------------------------
    # Cache maintenance the plain-data barrier adds to the coherent-data one: one L2
    # writeback per XCD (8 workgroups, one per XCD) and the invalidations of 32 CUs per XCD
    # at once (256 workgroups); the slowest of each.
    rel_us = sp.bench_fence(ctx, "release", 8, 64)["clk_per_fence_max"] / clock_after
    inv_us = sp.bench_fence(ctx, "acquire", 256, 64)["clk_per_fence_max"] / clock_after
    # L_coh: one-way latency of a signal between workgroups on different XCDs, relaxed
    # agent-scope store and polling (token ping-pong, 2 x 10^4 hand-overs per run).  It
    # depends on which XCDs the pair runs on and on where the two words live: eight runs
    # with the words 4 KiB further on each time, the fastest is the hop.
    sp.pingpong(ctx, 100, fenced=False)
    sig_runs = []
    for i in range(8):
        pp_xcc, pp_st = sp.pingpong(ctx, 10000, fenced=False, offset_bytes=4096 * i)
        sig_runs.append([round(pp_st["kernel_ms"] * 1e3 / (2 * 10000), 4), pp_xcc[2:4]])
    sig_us = min(v for v, _ in sig_runs)
    # The small barrier configuration: central counter, 16 workgroups x 64 lanes x 1000
    # rounds (median of five runs).
    bar1 = sp.Barrier(ctx, "central", C1_NWG)
    c1 = [bar1.run_hash(C1_LANES, C1_ROUNDS, 42) for _ in range(5)]
    c1_us = float(np.median([st["kernel_ms"] for _, st in c1])) * 1e3 / C1_ROUNDS
    c1_chk = c1[0][0]
    c1_same = all((chk == c1_chk).all() for chk, _ in c1)
    # The contended-atomic barrier against A1: the split central counter (every workgroup
    # adds one to one word, the last one stores the release word the others poll) with
    # coherently accessed data, so that no fence separates the atomics, 2048 workgroups x
    # AB_ROUNDS rounds (best of two).
    bar_ab = sp.Barrier(ctx, "central_split", NWG, coherent_cs=1)
    ab = [bar_ab.run_hash(LANES, AB_ROUNDS, 42) for _ in range(2)]
    bar_ab.close()
    ab_us = min(st["kernel_ms"] for _, st in ab) * 1e3 / AB_ROUNDS
    ab_chk = ab[0][0]
    # Section 4's machine card on this GPU: the twelve tests of Section 3 at 2048
    # workgroups (leader per workgroup, 1000 accesses, noncontentious words 256 B apart),
    # and the ceilings: A1 (timed steps), A_dist (adds spread over 2^20 words 128 B apart),
    # B_stream (1 GiB read with 16-byte loads), L_coh (above).
    times = abstraction.measure(ctx, NWG, reps=1)
    mcard = abstraction.card(times)
    permd = sp_inputs.permutation(1 << 20, 42)
    _, _, st_d = sp.bench_atomic(ctx, "add", NWG, LANES, 1 << 20, 128, "per_lane", 64, 42, permd)
    a_dist = st_d["ops"] / (st_d["kernel_ms"] * 1e-3)
    sbuf = ctx.zeros((1 << 30) // 4)
    sp.stream_read(ctx, sbuf, 1 << 30)
    _, st_s = sp.stream_read(ctx, sbuf, 1 << 30, reps=3)
    b_stream = 3 * (1 << 30) / (st_s["kernel_ms"] * 1e-3)
    sbuf.close()
    # The metric's "vs #WGs": the library's default barrier, mutex and semaphore at fewer
    # workgroups (the barrier's 10^4 rounds of the hash exchange; one lock x 16 words and
    # K = 32 with 2^18 operations), each result kept for the check against the oracle.
    curves = {"barrier_default_us_per_round": {}, "mutex_default_acq_per_s": {},
              "semaphore_k32_default_pairs_per_s": {}}
    curve_out = {}
    for n in CURVE_NWG:
        b = sp.Barrier(ctx, "default", n)
        bchk, bst = b.run_hash(LANES, ROUNDS, 42)
        b.close()
        m = sp.Mutex(ctx, "default", 1, 16)
        words, mst, _ = m.run(n, LANES, CURVE_OPS, 1000, 42)
        m.close()
        s = sp.Semaphore(ctx, "default", SEM_K)
        sres = s.run(n, LANES, CURVE_OPS, 2000, 42, track=False)
        s.close()
        curves["barrier_default_us_per_round"][n] = round(bst["kernel_ms"] * 1e3 / ROUNDS, 4)
        curves["mutex_default_acq_per_s"][n] = round(CURVE_OPS / (mst["kernel_ms"] * 1e-3), 1)
        curves["semaphore_k32_default_pairs_per_s"][n] = round(
            CURVE_OPS / (sres["stats"]["kernel_ms"] * 1e-3), 1)
        curve_out[n] = (bchk, words, sres["chk"])
    # Config 4's semaphore range at 2048 workgroups: the default kind at every K (2^18
    # pairs each; checked against the closed form like the curves)
    sem_vs_k, sem_k_chk = {}, {}
    for K in SEM_KS:
        s = sp.Semaphore(ctx, "default", K)
        sres = s.run(NWG, LANES, CURVE_OPS, 2000, 42, track=False)
        s.close()
        sem_vs_k[K] = round(CURVE_OPS / (sres["stats"]["kernel_ms"] * 1e-3), 1)
        sem_k_chk[K] = sres["chk"]

    bar_ms = float(np.mean([r["bar_ms"] for r in results]))
    us_round = bar_ms * 1e3 / ROUNDS
    per_round = np.array([r["bar_ms"] for r in results]) * 1e3 / ROUNDS
    kb_us = float(np.median([r["bar_kb_ms"] for r in results])) * 1e3 / ROUNDS
    a1 = float(np.mean([r["a1_ops"] / (r["a1_ms"] * 1e-3) for r in results]))
    arrivals = NWG * ROUNDS / (bar_ms * 1e-3)
    deterministic = all((r["bar_chk"] == results[0]["bar_chk"]).all() for r in results)
    mtx_rate = float(np.mean([MUTEX_TOTAL / (r["mtx_ms"] * 1e-3) for r in results]))
    mtx_def_rate = float(np.mean([MUTEX_TOTAL / (r["mtx_def_ms"] * 1e-3) for r in results]))
    sem_rate = float(np.mean([SEM_TOTAL / (r["sem_ms"] * 1e-3) for r in results]))
    sem_def_rate = float(np.mean([SEM_TOTAL / (r["sem_def_ms"] * 1e-3) for r in results]))
    # the kind the default semaphore ran (bucket 1: at least 64 workgroups per unit) and
    # the read-modify-writes per pair on its busiest contended word
    sem_def_kind = ctx.get_default("semaphore", 1 if NWG // SEM_K >= 64 else 0)
    sem_def_rmw = SEM_RMW_PER_PAIR[sem_def_kind]
    coh_us = float(np.mean([r["bar_coh_ms"] for r in results])) * 1e3 / ROUNDS

    def med(key, field):
        return round(float(np.median([r[key][field] for r in results])), 2)

    traffic = measured_traffic(ROOT) if args.barrier == "xcd" else None
    # Algorithmic bytes per workgroup per round: the exchanged slot's store and load (4 + 4)
    # and the barrier's arrival and release flags (4 + 4).  The round is latency-bound
    # (flag hops and cache maintenance), so this view is context, not the bound.
    alg_bytes = 16 * NWG * ROUNDS
    gbps = alg_bytes / (bar_ms * 1e-3) / 1e9
    # The bound of a hierarchical round (no read-modify-write in this barrier, so the
    # atomic term is zero): an arrival reaches its XCD's master, the master's stamp
    # reaches the other XCDs, and the release reaches each CU's workgroups -- three
    # one-way hops of L_coh, measured above.  The kernel boundary replayed from a graph
    # does the same exchange in kb_us: the demonstrated alternative.
    hops = 3
    floor_us = hops * sig_us

    line = {
        "metric": METRIC,
        "value": round(us_round, 4),
        "unit": "µs/round",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic (seeded hash-exchange, lock and semaphore schedules, Poisson request stream)",
        "config": {"workload": f"{args.barrier} barrier, {NWG} co-resident workgroups x {LANES} "
                               f"lanes x {ROUNDS} rounds (hash exchange); ticket mutex and "
                               f"K={SEM_K} semaphore at {NWG} workgroups, 2^20 operations each; "
                               f"serving queue, {SERVE_NWG} persistent workgroups, {SERVE_N} "
                               f"requests at {SERVE_RATE:g} req/s",
                   "nwg": NWG, "lanes": LANES, "rounds": ROUNDS},
        "metrics": {
            "barrier_us_per_round": round(us_round, 4),
            "barrier_us_per_round_median": round(float(np.median(per_round)), 4),
            "barrier_us_per_round_min": round(float(per_round.min()), 4),
            "kernel_boundary_graph_us_per_round": round(kb_us, 4),
            "kernel_boundary_checksums_identical": all(r["bar_kb_same"] for r in results),
            "barrier_coherent_data_us_per_round": round(coh_us, 4),
            "barrier_coherent_checksums_identical": all(r["bar_coh_same"] for r in results),
            "barrier_plain_minus_coherent_us": round(us_round - coh_us, 4),
            "central_barrier_16wg_x64_1000_rounds_us_per_round": round(c1_us, 4),
            "central_barrier_16wg_checksums_deterministic": bool(c1_same),
            "fence_writeback_per_xcd_us": round(rel_us, 4),
            "fence_invalidate_32_cus_per_xcd_us": round(inv_us, 4),
            "signal_one_way_cross_xcd_us": round(sig_us, 4),
            "signal_one_way_runs_us_xcc": sig_runs,
            "barrier_arrivals_per_s": round(arrivals, 1),
            "mutex_ticket_acq_per_s": round(mtx_rate, 1),
            "mutex_default_kind_acq_per_s": round(mtx_def_rate, 1),
            "semaphore_k32_pairs_per_s": round(sem_rate, 1),
            "semaphore_k32_default_kind_pairs_per_s": round(sem_def_rate, 1),
            "barrier_checksums_deterministic": bool(deterministic),
            "mutex_counts_exact": all(r["mtx_ok"] for r in results),
            "semaphore_state_exact": all(r["sem_ok"] and r["sem_def_ok"] for r in results),
            "serve_persistent_p50_us": med("serve", "p50_us"),
            "serve_persistent_p99_us": med("serve", "p99_us"),
            "serve_persistent_req_per_s": med("serve", "req_per_s"),
            "serve_launch_per_request_p50_us": med("serve_launch", "p50_us"),
            "serve_launch_per_request_p99_us": med("serve_launch", "p99_us"),
            "serve_launch_per_request_req_per_s": med("serve_launch", "req_per_s"),
            "serve_results_identical": all(r["serve_same"] for r in results),
            "shader_clock_mhz_before_after": [round(clock_before, 1), round(clock_after, 1)],
            "curves_vs_nwg": curves,
            "semaphore_default_2048wg_pairs_per_s_vs_K": sem_vs_k,
            # Section 4's card and the ceilings the primitives are compared with
            "machine_card_2048wg": {
                "atomic_to_volatile_contentious": mcard["atomic_to_volatile"],
                "contentious_to_noncontentious_volatile":
                    mcard["contentious_to_noncontentious_volatile"],
                "volatile_after_atomic_to_volatile": mcard["volatile_after_atomic_to_volatile"],
                "times_ms": {k: round(v, 4) for k, v in times.items()}},
            "ceilings": {"A1_contended_atomics_per_s": round(a1, 1),
                         "A_dist_atomics_per_s_2p20_words": round(a_dist, 1),
                         "B_stream_read_GB_per_s": round(b_stream / 1e9, 1),
                         "L_coh_one_way_us": round(sig_us, 4)},
            # The mutex and semaphore against their own bounds.  A contended word takes
            # at most A1 read-modify-writes per second, so a semaphore kind that makes r
            # of them per pair on its busiest word admits at most A1 / r pairs per second:
            # Algorithm 5 r = 2 (count, up in the wait and down in the post), the ticket
            # kinds r = 1 (the tickets word in the wait, the posts word in the post).  A
            # lock hand-over through memory moves ownership at least one one-way hop, so at
            # most 1 / L_coh acquisitions per second (the critical section's own time left
            # out); the CU-cohort lock's hand-overs within a CU stay in the CU's L1, so for
            # it the figure is a reference, not a bound.
            "bounds": {
                "semaphore_k32_alg5_bound_per_s": round(a1 / 2, 1),
                "semaphore_k32_alg5_frac": round(sem_rate / (a1 / 2), 4),
                "semaphore_k32_default_kind": sem_def_kind,
                "semaphore_k32_default_kind_bound_per_s": round(a1 / sem_def_rmw, 1),
                "semaphore_k32_default_kind_frac": round(sem_def_rate / (a1 / sem_def_rmw), 4),
                "mutex_acq_bound_per_s": round(1e6 / sig_us, 1),
                "mutex_default_kind_frac": round(mtx_def_rate * sig_us * 1e-6, 4),
                "mutex_ticket_frac": round(mtx_rate * sig_us * 1e-6, 4),
                # one read-modify-write per workgroup per round on one word: at most A1
                # arrivals per second
                "atomic_barrier_split_central_coherent_2048wg": {
                    "us_per_round": round(ab_us, 4),
                    "arrivals_per_s": round(NWG / (ab_us * 1e-6), 1),
                    "frac_of_A1": round(NWG / (ab_us * 1e-6) / a1, 4)}},
            # other views of the headline kernel (not bounds)
            "barrier_arrivals_vs_A1": round(arrivals / a1, 4),
            "barrier_hbm_view": {"algorithmic_bytes_per_launch": alg_bytes,
                                 "algorithmic_GB_per_s": round(gbps, 3),
                                 "frac_of_8_TB_per_s": round(gbps / 8000.0, 6)},
        },
        "roofline": {
            "bound": "latency",
            "kernel": f"k_barrier_hash<{args.barrier}, plain data>",
            "achieved": round(1.0 / us_round, 6),
            "peak": round(1.0 / floor_us, 6),
            "unit": "M barrier rounds/s (peak: 1 / three one-way hops of L_coh)",
            "frac": round(floor_us / us_round, 4),
            "traffic": traffic,
            "traffic_unit": "bytes per launch moved between the L2s and memory (rocprofv3 "
                            "FETCH_SIZE + WRITE_SIZE, calibrated)",
            "bound_terms": {"hops": hops, "L_coh_us": round(sig_us, 4),
                            "floor_us": round(floor_us, 4),
                            "source": "sp_bench_pingpong in this run"},
            "kernel_boundary_us_per_round": round(kb_us, 4),
            "coherent_data_round_us": round(coh_us, 4),
            "coherent_data_frac": round(floor_us / coh_us, 4),
        },
        "env": environment(ctx, results[0]["bar_occ"]),
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(results[0]["bar_chk"], c1_chk, curve_out,
                                            atomic_chk=ab_chk, sem_k_chk=sem_k_chk)
    print(json.dumps(line), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
