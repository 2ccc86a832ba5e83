"""GPU parity of the serving queue: every request's hash chain equals the oracle's, bit
for bit, in the persistent kernel and in the launch-per-request comparator; the budget's
weighted semaphore never lets the admitted requests hold more than its units and ends
with every unit returned."""

import numpy as np
import pytest

import oracle
import sp_inputs
from conftest import announce

pytestmark = pytest.mark.gpu

UNIT = 65536


def _units(reqs, unit=UNIT):
    nb = reqs["nbytes"].astype(np.uint64)
    return (nb + np.uint64(unit - 1)) // np.uint64(unit)


def _check(reqs, out, lat, res, seed, budget, unit=UNIT, tracked=True):
    n = len(reqs["L"])
    expect = oracle.chain_batch(seed, reqs["L"])
    bad = np.nonzero(out != expect)[0]
    assert bad.size == 0, f"{bad.size} wrong results, first at request {bad[:5]}"
    assert res["completed"] == n and res["device_error"] == 0
    assert np.isfinite(lat).all() and (lat > 0).all()
    assert res["p50_us"] <= res["p99_us"] <= res["max_us"]
    total = int(_units(reqs, unit).sum())
    assert res["units_issued"] == total and res["units_released"] == total
    if tracked:
        assert int(_units(reqs, unit).max()) <= res["max_units_in_use"] <= budget


def _persistent(ctx, reqs, seed, nwg=1024, budget=16384, unit=UNIT, **cfg):
    import paper_1110_4623_amd as sp
    announce("serve persistent", f"n={len(reqs['L'])} nwg={nwg} budget={budget}", cfg)
    return sp.serve(ctx, reqs, nwg=nwg, budget_units=budget, unit_bytes=unit, seed=seed, **cfg)


def _launch(ctx, reqs, seed, budget=16384, unit=UNIT, **cfg):
    import paper_1110_4623_amd as sp
    announce("serve launch", f"n={len(reqs['L'])} budget={budget}", cfg)
    return sp.serve_launch_per_request(ctx, reqs, budget_units=budget, unit_bytes=unit,
                                       seed=seed, **cfg)


@pytest.mark.parametrize("seed", sp_inputs.SEEDS)
def test_persistent_small(ctx, seed):
    reqs = sp_inputs.request_table(3000, 1e5, seed)
    out, lat, res = _persistent(ctx, reqs, seed, track=1)
    _check(reqs, out, lat, res, seed, 16384)
    assert res["launches"] == 1


def test_persistent_tight_budget_queues(ctx):
    # chains clipped to 1024 steps need at most 64 units; a 64-unit budget admits large
    # requests one at a time, so most requests wait in the semaphore's FIFO
    seed = 7
    reqs = sp_inputs.request_table(2000, 1e6, seed, lmax=1024)
    out, lat, res = _persistent(ctx, reqs, seed, budget=64, track=1)
    _check(reqs, out, lat, res, seed, 64)
    assert res["max_units_in_use"] > 32


@pytest.mark.parametrize("n,nwg", [(1, 16), (3, 16), (17, 16), (100, 1), (64, 64)])
def test_persistent_ragged(ctx, n, nwg):
    seed = 42
    reqs = sp_inputs.request_table(n, 1e5, seed, lmax=4096)
    out, lat, res = _persistent(ctx, reqs, seed, nwg=nwg, track=1, ring_slots=64)
    _check(reqs, out, lat, res, seed, 16384)


def test_persistent_zero_length_chains_and_simultaneous_arrivals(ctx):
    seed = 0xC0FFEE
    n = 500
    reqs = {"L": np.arange(n, dtype=np.uint32) % 3, "t_arr": np.zeros(n),
            "nbytes": np.zeros(n, dtype=np.uint64)}
    out, lat, res = _persistent(ctx, reqs, seed, nwg=256, track=1, ring_slots=128)
    assert (out[reqs["L"] == 0] == (seed ^ np.arange(n, dtype=np.uint32))[reqs["L"] == 0]).all()
    _check(reqs, out, lat, res, seed, 16384, tracked=False)


def test_persistent_lanes_above_one_wave(ctx):
    seed = 42
    reqs = sp_inputs.request_table(1000, 1e5, seed)
    out, lat, res = _persistent(ctx, reqs, seed, nwg=512, lanes=256, track=1)
    _check(reqs, out, lat, res, seed, 16384)


@pytest.mark.parametrize("streams,batch", [(1, 1), (4, 1), (1, 32), (4, 32)])
def test_launch_per_request(ctx, streams, batch):
    seed = 42
    reqs = sp_inputs.request_table(1500, 1e5, seed)
    out, lat, res = _launch(ctx, reqs, seed, streams=streams, batch=batch)
    _check(reqs, out, lat, res, seed, 16384, tracked=False)
    assert res["launches"] >= (1500 if batch == 1 else 1500 // batch)


def test_launch_tight_budget(ctx):
    seed = 7
    reqs = sp_inputs.request_table(800, 1e6, seed, lmax=1024)
    out, lat, res = _launch(ctx, reqs, seed, budget=64, streams=4, batch=8)
    _check(reqs, out, lat, res, seed, 64, tracked=False)


@pytest.mark.parametrize("streams,graph", [(1, 1), (1, 8), (4, 8), (4, 64)])
def test_launch_graph_batched(ctx, streams, graph):
    """graph_batch: a recorded graph of G one-workgroup nodes is replayed per G arrivals;
    the partial last batch is flushed; results are the oracle's for every request."""
    seed = 11
    reqs = sp_inputs.request_table(1500, 1e5, seed)
    out, lat, res = _launch(ctx, reqs, seed, streams=streams, graph_batch=graph)
    _check(reqs, out, lat, res, seed, 16384, tracked=False)
    assert res["launches"] >= -(-1500 // graph)


@pytest.mark.parametrize("budget,ring,graph", [(64, 65536, 16), (16384, 64, 128)])
def test_launch_graph_batched_flushes_on_stalls(ctx, budget, ring, graph):
    """A tight budget, or a ring smaller than a batch, stops publishing before a batch is
    full: the waiting requests are launched as a partial batch instead of deadlocking."""
    seed = 3
    reqs = sp_inputs.request_table(700, 1e6, seed, lmax=1024)
    out, lat, res = _launch(ctx, reqs, seed, budget=budget, streams=2, graph_batch=graph,
                            ring_slots=ring)
    _check(reqs, out, lat, res, seed, budget, tracked=False)


def test_launch_graph_batched_bad_arguments(ctx):
    import paper_1110_4623_amd as sp
    reqs = sp_inputs.request_table(10, 1e5, 1)
    for kw in (dict(graph_batch=4097), dict(graph_batch=8, batch=4)):
        with pytest.raises(sp.SpError):
            _launch(ctx, reqs, 1, **kw)


def test_bad_tables_rejected(ctx):
    import paper_1110_4623_amd as sp
    reqs = sp_inputs.request_table(10, 1e5, 42)
    with pytest.raises(sp.SpError):  # a request needing more units than the budget
        sp.serve(ctx, reqs, nwg=16, budget_units=1, unit_bytes=64)
    bad = dict(reqs, t_arr=reqs["t_arr"][::-1].copy())
    with pytest.raises(sp.SpError):  # arrivals out of order
        sp.serve(ctx, bad, nwg=16)
    with pytest.raises(sp.SpError):
        sp.serve(ctx, reqs, nwg=16, ring_slots=100)  # not a power of two
    with pytest.raises(sp.SpNotResident):
        sp.serve(ctx, reqs, nwg=1 << 16, lanes=1024)


@pytest.mark.parametrize("rate", [1e4, 1e5, 1e6])
def test_persistent_full_size(ctx, rate):
    """1024 persistent workgroups, a 1 GiB budget in 64 KiB units, Poisson arrivals for
    2 s at the given rate (at least 2 x 10^4 requests), lognormal(5, 1.5) chain lengths:
    every result checked."""
    seed = 42
    n = int(max(2e4, 2 * rate))
    reqs = sp_inputs.request_table(n, rate, seed)
    out, lat, res = _persistent(ctx, reqs, seed, track=1)
    _check(reqs, out, lat, res, seed, 16384)
    print(f"[serve] rate={rate:g} n={n} p50={res['p50_us']:.1f}us p99={res['p99_us']:.1f}us "
          f"req/s={res['req_per_s']:.0f} lag={res['publish_lag_max_us']:.1f}us", flush=True)


def test_launch_per_request_full_size_low_rate(ctx):
    seed = 42
    reqs = sp_inputs.request_table(20000, 1e4, seed)
    out, lat, res = _launch(ctx, reqs, seed)
    _check(reqs, out, lat, res, seed, 16384, tracked=False)
    print(f"[serve-launch] p50={res['p50_us']:.1f}us p99={res['p99_us']:.1f}us", flush=True)
