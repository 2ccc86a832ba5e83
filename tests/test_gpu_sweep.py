"""The measurement sweeps on the GPU: short runs whose results must agree across kinds."""

import pytest

from conftest import announce

pytestmark = pytest.mark.gpu


def test_barrier_sweep_kinds_agree_and_report_the_launch(ctx):
    from paper_1110_4623_amd import sweep
    announce("sweep barrier", "rounds=100 quick (N = 256, 2048)")
    rows = sweep.barrier(ctx, rounds=100, quick=True)["rows"]
    kinds = {r["kind"] for r in rows}
    assert set(sweep.BARRIERS) | {"kernel_boundary_launch", "kernel_boundary_graph"} == kinds
    assert all(r["checksums_agree"] for r in rows)
    for r in rows:
        if r["kind"] in sweep.BARRIERS:
            assert 0 < r["empty_launch_us"] < 1e3 * r["us_per_round"] * r["rounds"]
            assert r["us_per_round_minus_empty_launch"] < r["us_per_round"]
