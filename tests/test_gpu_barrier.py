"""GPU parity of the global barriers on the hash-exchange workload: element-by-element
equality of every workgroup's checksum with the oracle's closed form."""

import numpy as np
import pytest

import oracle
import sp_inputs
from conftest import announce

pytestmark = pytest.mark.gpu

KINDS = ["central", "central_split", "tree", "flag", "xcd", "grid_sync"]
OURS = ["central", "central_split", "tree", "flag", "xcd"]


def _run(ctx, kind, nwg, lanes, rounds, seed, **params):
    import paper_1110_4623_amd as sp
    announce("barrier", kind, f"nwg={nwg} lanes={lanes} rounds={rounds} seed={seed}", params)
    bar = sp.Barrier(ctx, kind, nwg, **params)
    try:
        chk, st = bar.run_hash(lanes=lanes, rounds=rounds, seed=seed)
    finally:
        bar.close()
    return chk, st


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("seed", sp_inputs.SEEDS)
def test_small_config(ctx, kind, seed):
    # 16 workgroups x 64 lanes x 1000 rounds
    chk, st = _run(ctx, kind, 16, 64, 1000, seed)
    assert (chk == oracle.barrier_closed(seed, 16, 1000)).all()
    assert st["device_error"] == 0


@pytest.mark.parametrize("kind", OURS)
@pytest.mark.parametrize("nwg,lanes,rounds", [(1, 64, 10), (2, 128, 50), (7, 256, 300),
                                               (9, 64, 300), (100, 192, 200), (257, 256, 100),
                                               (500, 1024, 20)])
def test_ragged_shapes(ctx, kind, nwg, lanes, rounds):
    chk, _ = _run(ctx, kind, nwg, lanes, rounds, 0xC0FFEE)
    assert (chk == oracle.barrier_closed(0xC0FFEE, nwg, rounds)).all()


@pytest.mark.parametrize("kind", OURS)
@pytest.mark.parametrize("nwg", [256, 1024, 2048])
def test_at_scale(ctx, kind, nwg):
    # co-resident workgroups x 256 lanes x 10^4 rounds
    chk, st = _run(ctx, kind, nwg, 256, 10_000, 42)
    assert (chk == oracle.barrier_closed(42, nwg, 10_000)).all()


@pytest.mark.parametrize("params", [dict(fan_in=2), dict(fan_in=16), dict(fan_in=64),
                                    dict(pad_bytes=4), dict(pad_bytes=4096), dict(poll_sleep=0),
                                    dict(poll_sleep=8)])
def test_tree_parameters(ctx, params):
    chk, _ = _run(ctx, "tree", 512, 256, 500, 7, **params)
    assert (chk == oracle.barrier_closed(7, 512, 500)).all()


@pytest.mark.parametrize("params", [dict(flags_packed=1), dict(pad_bytes=64), dict(poll_sleep=0)])
def test_flag_parameters(ctx, params):
    chk, _ = _run(ctx, "flag", 1024, 256, 500, 7, **params)
    assert (chk == oracle.barrier_closed(7, 1024, 500)).all()


@pytest.mark.parametrize("params", [dict(pad_bytes=64), dict(pad_bytes=4096), dict(poll_sleep=0),
                                    dict(poll_sleep=16)])
def test_xcd_parameters(ctx, params):
    chk, _ = _run(ctx, "xcd", 2048, 256, 500, 7, **params)
    assert (chk == oracle.barrier_closed(7, 2048, 500)).all()


@pytest.mark.parametrize("kind", ["central", "xcd"])
def test_cooperative_launch(ctx, kind):
    chk, _ = _run(ctx, kind, 2048, 256, 300, 5, cooperative=1)
    assert (chk == oracle.barrier_closed(5, 2048, 300)).all()


@pytest.mark.parametrize("graph", [False, True])
def test_kernel_boundary_comparator(ctx, graph):
    import paper_1110_4623_amd as sp
    announce("barrier launches", f"graph={graph}")
    chk, st = sp.barrier_hash_launches(ctx, 64, 64, 200, 42, graph=graph)
    assert (chk == oracle.barrier_closed(42, 64, 200)).all()


def test_not_resident_is_refused(ctx):
    import paper_1110_4623_amd as sp
    nwg = ctx.info["cu_count"] * 64  # far more 1024-lane workgroups than can be resident
    announce("barrier not-resident", nwg)
    bar = sp.Barrier(ctx, "central", nwg)
    with pytest.raises(sp.SpNotResident):
        bar.run_hash(lanes=1024, rounds=1, seed=1)
    bar.close()


@pytest.mark.parametrize("nwg,lanes", [(3, 64), (13, 128), (1024, 256), (2048, 256)])
def test_xcd_barrier_reads_placement_after_cooperative_launch(ctx, nwg, lanes):
    """After a cooperative launch the dispatcher has been seen to start later launches one
    XCD further on (workgroup w on XCD (w - 1) mod 8).  The per-XCD barrier registers
    every workgroup under the XCD it actually runs on, so it keeps its fast path and its
    exact results whatever the rotation."""
    import paper_1110_4623_amd as sp
    announce("grid_sync then xcd", f"nwg={nwg} lanes={lanes}")
    g = sp.Barrier(ctx, "grid_sync", 256)
    try:
        g.run_hash(256, 10, 1)
    finally:
        g.close()
    b = sp.Barrier(ctx, "xcd", nwg)
    try:
        for seed in (42, 7):
            chk, _ = b.run_hash(lanes, 300, seed)
            assert (chk == oracle.barrier_closed(seed, nwg, 300)).all()
            info = b.info()
            assert info["xcd_path"] and info["cu_overflow"] == 0, info
    finally:
        b.close()


def test_xcd_barrier_info_fresh_placement(ctx):
    import paper_1110_4623_amd as sp
    b = sp.Barrier(ctx, "xcd", 512)
    try:
        chk, _ = b.run_hash(256, 100, 3)
        assert (chk == oracle.barrier_closed(3, 512, 100)).all()
        assert b.info()["xcd_path"]
    finally:
        b.close()


@pytest.mark.parametrize("kind", ["central", "central_split", "tree", "flag", "xcd"])
@pytest.mark.parametrize("nwg,lanes", [(16, 64), (257, 128), (2048, 256)])
def test_coherent_data_barriers(ctx, kind, nwg, lanes):
    """coherent_cs: the exchanged slots are written and read with agent-scope accesses
    and the barrier does no cache maintenance; the checksums are the oracle's."""
    import paper_1110_4623_amd as sp
    if kind in ("central", "central_split", "tree", "flag") and nwg == 2048:
        rounds = 200
    else:
        rounds = 1000
    announce("coherent barrier", kind, f"nwg={nwg} lanes={lanes} rounds={rounds}")
    b = sp.Barrier(ctx, kind, nwg, coherent_cs=1)
    try:
        for seed in (42, 0xC0FFEE):
            chk, _ = b.run_hash(lanes, rounds, seed)
            assert (chk == oracle.barrier_closed(seed, nwg, rounds)).all()
        if kind == "xcd":
            assert b.info()["xcd_path"]
    finally:
        b.close()


@pytest.mark.parametrize("copies", [1, 8, 64, 256])
@pytest.mark.parametrize("coherent", [0, 1])
@pytest.mark.parametrize("nwg,lanes", [(5, 64), (300, 128), (2048, 256)])
def test_xcd_stamp_copies(ctx, copies, coherent, nwg, lanes):
    """xcd_copies: the XCD masters publish into several packed copies of the stamps and
    the CUs poll different copies; the checksums stay the oracle's."""
    import paper_1110_4623_amd as sp
    announce("xcd copies", f"copies={copies} coherent={coherent} nwg={nwg} lanes={lanes}")
    b = sp.Barrier(ctx, "xcd", nwg, xcd_copies=copies, coherent_cs=coherent)
    try:
        for seed in (42, 7):
            chk, _ = b.run_hash(lanes, 400, seed)
            assert (chk == oracle.barrier_closed(seed, nwg, 400)).all()
        assert b.info()["xcd_path"]
    finally:
        b.close()


def _near_expected(ctx, nwg, copies, placement, pad=128):
    """Bits of what the measured placement covers: 1 arrival blocks, 2 stamp copies,
    4 per-CU release lines (each where it fits an 8 KiB chunk)."""
    n = ctx.info["xcd_count"]
    xblock = ((nwg + n - 1) // n + 31) // 32 * 32
    if placement == 1 or n < 2 or xblock * 4 > 2048:
        return 0
    sw = max(1, pad // 4)
    mstride = (max(sw, n) + sw - 1) // sw * sw
    bits = 1
    if copies >= n and copies % n == 0 and copies // n * mstride <= 2048:
        bits |= 2
    if 64 * sw <= 2048:
        bits |= 4
    return bits


@pytest.mark.parametrize("placement", [0, 1])
@pytest.mark.parametrize("copies", [0, 4, 8, 64, 256])
@pytest.mark.parametrize("coherent", [0, 1])
def test_xcd_flag_placement(ctx, placement, copies, coherent):
    """flag_placement 0 measures at creation which 8 KiB chunks are close to each XCD and
    puts the XCD's arrival flags there, and the stamp copies it polls when every copy is
    polled by one XCD; 1 keeps the fixed layout.  The checksums are the oracle's either
    way, run after run."""
    import paper_1110_4623_amd as sp
    nwg = 2048
    announce("xcd placement", f"placement={placement} copies={copies} coherent={coherent}")
    b = sp.Barrier(ctx, "xcd", nwg, xcd_copies=copies, coherent_cs=coherent,
                   flag_placement=placement)
    try:
        assert b.info()["near_placed"] == _near_expected(ctx, nwg, copies, placement)
        for seed in (42, 7, 42):
            chk, _ = b.run_hash(256, 500, seed)
            assert (chk == oracle.barrier_closed(seed, nwg, 500)).all()
        assert b.info()["xcd_path"]
    finally:
        b.close()


@pytest.mark.parametrize("nwg,lanes,pad", [(5, 64, 128), (300, 128, 4), (1000, 256, 4096),
                                           (4096, 64, 128)])
def test_xcd_flag_placement_shapes(ctx, nwg, lanes, pad):
    """Ragged grids, tiny and page-sized padding: the measured layout where the blocks
    fit a chunk, the fixed one where they do not."""
    import paper_1110_4623_amd as sp
    announce("xcd placement shapes", f"nwg={nwg} lanes={lanes} pad={pad}")
    b = sp.Barrier(ctx, "xcd", nwg, xcd_copies=64, pad_bytes=pad)
    try:
        assert b.info()["near_placed"] == _near_expected(ctx, nwg, 64, 0, pad)
        chk, _ = b.run_hash(lanes, 300, 5)
        assert (chk == oracle.barrier_closed(5, nwg, 300)).all()
    finally:
        b.close()


def test_xcd_flag_placement_invalid(ctx):
    import paper_1110_4623_amd as sp
    with pytest.raises(sp.SpError):
        sp.Barrier(ctx, "xcd", 64, flag_placement=2)


def test_xcd_stamp_copies_after_cooperative_launch(ctx):
    import paper_1110_4623_amd as sp
    announce("grid_sync then xcd copies=8")
    g = sp.Barrier(ctx, "grid_sync", 256)
    try:
        g.run_hash(256, 10, 1)
    finally:
        g.close()
    b = sp.Barrier(ctx, "xcd", 2048, xcd_copies=8)
    try:
        chk, _ = b.run_hash(256, 300, 11)
        assert (chk == oracle.barrier_closed(11, 2048, 300)).all()
        assert b.info()["xcd_path"]
    finally:
        b.close()


@pytest.mark.parametrize("params", [dict(xcd_copies=3), dict(xcd_copies=512)])
def test_xcd_stamp_copies_invalid(ctx, params):
    import paper_1110_4623_amd as sp
    with pytest.raises(sp.SpError):
        sp.Barrier(ctx, "xcd", 64, **params)


@pytest.mark.parametrize("pad", [4, 16, 4096])
def test_xcd_stamp_copies_with_small_and_large_padding(ctx, pad):
    """A copy holds every XCD's stamp even when the padding is below 8 words."""
    chk, _ = _run(ctx, "xcd", 1024, 128, 300, 42, xcd_copies=64, pad_bytes=pad)
    assert (chk == oracle.barrier_closed(42, 1024, 300)).all()


def _max_resident(ctx, lanes):
    import paper_1110_4623_amd as sp
    b = sp.Barrier(ctx, "central", 64)
    try:
        _, st = b.run_hash(lanes, 1, 1)
    finally:
        b.close()
    return st["resident_per_cu"] * ctx.info["cu_count"]


@pytest.mark.parametrize("kind", ["xcd", "central", "tree", "flag"])
def test_largest_co_resident_grid(ctx, kind):
    """The most workgroups that can be resident at once (64-lane workgroups, every wave
    slot of every CU): each XCD's master scans a full flag block, every CU releases 32
    workgroups through its line; the checksums are the oracle's."""
    import paper_1110_4623_amd as sp
    nwg = _max_resident(ctx, 64)
    assert nwg >= 4096
    announce("barrier largest grid", kind, f"nwg={nwg} lanes=64 rounds=200")
    b = sp.Barrier(ctx, kind, nwg)
    try:
        for seed in (42, 7):
            chk, _ = b.run_hash(64, 200, seed)
            assert (chk == oracle.barrier_closed(seed, nwg, 200)).all()
        if kind == "xcd":
            assert b.info()["xcd_path"]
            assert b.info()["near_placed"] == _near_expected(ctx, nwg, 64, 0)
    finally:
        b.close()


def test_one_more_than_resident_is_refused(ctx):
    import paper_1110_4623_amd as sp
    nwg = _max_resident(ctx, 64) + 1
    b = sp.Barrier(ctx, "xcd", nwg)
    try:
        with pytest.raises(sp.SpNotResident):
            b.run_hash(64, 1, 1)
    finally:
        b.close()


@pytest.mark.parametrize("nwg,xcd", [(32, False), (39, False), (40, True), (63, True)])
def test_default_barrier_split_at_40_workgroups(ctx, nwg, xcd):
    """A default barrier runs the central counter below 40 workgroups and the per-XCD
    barrier from 40 on (the measured crossover); both give the oracle's checksums."""
    import paper_1110_4623_amd as sp
    announce("default barrier", f"nwg={nwg}")
    b = sp.Barrier(ctx, "default", nwg)
    try:
        chk, _ = b.run_hash(256, 200, 5)
        assert (chk == oracle.barrier_closed(5, nwg, 200)).all()
        assert b.info()["kind"] == ("xcd" if xcd else "central")
        assert b.info()["xcd_path"] == xcd
    finally:
        b.close()
