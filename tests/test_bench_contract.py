"""bench.py's output contract: one JSON line with the fields the measurement needs."""

import json
import os
import subprocess
import sys

import pytest

from conftest import ROOT, announce


def _bench(*args, timeout=300):
    env = dict(os.environ, SP_NO_TORCH="1")
    return subprocess.run([sys.executable, "-u", os.path.join(ROOT, "bench.py"), *args],
                          cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)


def test_more_than_one_gpu_is_refused_with_a_message():
    p = _bench("--gpus", "2", timeout=60)
    assert p.returncode == 2
    assert "one GPU" in p.stderr and p.stdout == ""


@pytest.mark.gpu
def test_one_step_prints_the_contract_line():
    announce("bench.py", "--steps 1 --warmup 0 --no-cpu-baseline")
    p = _bench("--steps", "1", "--warmup", "0", "--no-cpu-baseline")
    assert p.returncode == 0, p.stderr[-2000:]
    lines = [l for l in p.stdout.splitlines() if l.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
              "metrics", "roofline", "env"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 1 and d["warmup"] == 0
    assert d["value"] > 0 and d["higher_is_better"] is False and d["dtype"] == "u32"
    assert "workload" in d["config"]
    m = d["metrics"]
    for flag in ("barrier_checksums_deterministic", "barrier_coherent_checksums_identical",
                 "kernel_boundary_checksums_identical", "mutex_counts_exact",
                 "semaphore_state_exact", "serve_results_identical"):
        assert m[flag] is True, flag
    assert m["barrier_us_per_round_min"] <= m["barrier_us_per_round_median"]
    r = d["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in r, k
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"], rel=1e-2)
    assert r["bound"] == "latency" and r["bound_terms"]["hops"] == 3
    assert r["peak"] == pytest.approx(1.0 / r["bound_terms"]["floor_us"], rel=1e-3)
    assert r["kernel_boundary_us_per_round"] > 0
    card = m["machine_card_2048wg"]
    for name in ("atomic_to_volatile_contentious", "contentious_to_noncontentious_volatile",
                 "volatile_after_atomic_to_volatile"):
        assert card[name]["read"] > 0 and card[name]["write"] > 0, name
    for k in ("A1_contended_atomics_per_s", "A_dist_atomics_per_s_2p20_words",
              "B_stream_read_GB_per_s", "L_coh_one_way_us"):
        assert m["ceilings"][k] > 0, k
    assert m["central_barrier_16wg_x64_1000_rounds_us_per_round"] > 0
    for k in ("semaphore_k32_default_kind_frac", "semaphore_k32_alg5_frac",
              "mutex_default_kind_frac", "mutex_ticket_frac"):
        assert 0 < m["bounds"][k] < 1, k
    assert sorted(int(k) for k in m["semaphore_default_2048wg_pairs_per_s_vs_K"]) == [1, 4, 32, 256]
    assert min(m["semaphore_default_2048wg_pairs_per_s_vs_K"].values()) > 0
    ab = m["bounds"]["atomic_barrier_split_central_coherent_2048wg"]
    assert 0 < ab["frac_of_A1"] < 1.5 and ab["us_per_round"] > 0
    import bench
    kind = m["bounds"]["semaphore_k32_default_kind"]
    assert m["bounds"]["semaphore_k32_default_kind_bound_per_s"] == round(
        m["ceilings"]["A1_contended_atomics_per_s"] / bench.SEM_RMW_PER_PAIR[kind], 1)
    assert m["central_barrier_16wg_checksums_deterministic"] is True
    for name in ("barrier_default_us_per_round", "mutex_default_acq_per_s",
                 "semaphore_k32_default_pairs_per_s"):
        assert len(m["curves_vs_nwg"][name]) == 3 and min(m["curves_vs_nwg"][name].values()) > 0
    assert d["env"]["arch"].startswith("gfx950")
    assert "packed-fp32-ops" in d["env"]["hipcc_flags"]


def test_cpu_baseline_leg_checks_checksums_against_the_oracle():
    """The oracle leg of bench.py (CPU only): it times the threaded per-XCD protocol and
    compares the run's checksums with the closed form, element by element."""
    import importlib.util
    import numpy as np
    import oracle
    spec = importlib.util.spec_from_file_location("_bench", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    ref = oracle.barrier_closed(42, bench.NWG, bench.ROUNDS)
    ref1 = oracle.barrier_closed(42, bench.C1_NWG, bench.C1_ROUNDS)
    d = bench.cpu_baseline(ref, ref1, budget_s=0.5)
    assert d["ok"] and d["kind"] == "oracle" and d["cores"] >= 1 and d["value"] > 0
    assert d["headline_checksums_match_oracle"] and d["config1_checksums_match_oracle"]
    bad = ref.copy()
    bad[7] ^= 1
    d = bench.cpu_baseline(bad, ref1, budget_s=0.5)
    assert not d["headline_checksums_match_oracle"]
    # the curves against #WGs: every result checked, one wrong word is caught
    n = 64
    good = {n: (oracle.barrier_closed(42, n, bench.ROUNDS),
                oracle.mutex_closed(42, n, bench.CURVE_OPS, 1, 16),
                oracle.sem_closed(42, n, bench.CURVE_OPS))}
    assert bench.cpu_baseline(ref, ref1, good, budget_s=0.5)["curves_match_oracle"] is True
    words = good[n][1].copy()
    words[0, 3] += 1
    bad_curve = {n: (good[n][0], words, good[n][2])}
    assert bench.cpu_baseline(ref, ref1, bad_curve, budget_s=0.5)["curves_match_oracle"] is False
    # the atomic barrier's checksums (2048 x AB_ROUNDS), one planted wrong word
    refab = oracle.barrier_closed(42, bench.NWG, bench.AB_ROUNDS)
    assert bench.cpu_baseline(ref, ref1, budget_s=0.5,
                              atomic_chk=refab)["atomic_barrier_checksums_match_oracle"] is True
    want = oracle.sem_closed(42, bench.NWG, bench.CURVE_OPS)
    ok = bench.cpu_baseline(ref, ref1, budget_s=0.5, sem_k_chk={1: want, 32: want})
    assert ok["semaphore_vs_K_checksums_match_oracle"] is True
    wrong = want.copy()
    wrong[5] ^= 1
    ok = bench.cpu_baseline(ref, ref1, budget_s=0.5, sem_k_chk={1: want, 32: wrong})
    assert ok["semaphore_vs_K_checksums_match_oracle"] is False
    refab[100] ^= 4
    assert bench.cpu_baseline(ref, ref1, budget_s=0.5,
                              atomic_chk=refab)["atomic_barrier_checksums_match_oracle"] is False


def test_semaphore_bound_covers_every_kind():
    """Every semaphore kind has a read-modify-write count for its busiest word."""
    import bench
    from paper_1110_4623_amd import _native as N
    assert set(bench.SEM_RMW_PER_PAIR) == set(N.SEM_KINDS) - {"default"}
