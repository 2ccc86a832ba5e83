"""GPU parity of the memory-system microbenchmarks against the oracle's closed forms."""

import numpy as np
import pytest

import oracle
import sp_inputs
from conftest import announce

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("op", ["add", "cas", "ld", "st"])
@pytest.mark.parametrize("mode", ["per_lane", "wave_leader"])
@pytest.mark.parametrize("T,stride", [(1, 4), (32, 64), (1024, 128), (1 << 20, 128), (37, 4)])
def test_closed_forms(ctx, op, mode, T, stride):
    import paper_1110_4623_amd as sp
    nwg, lanes, n, seed = 64, 256, 40, 42
    if op == "cas" and T == 1 and mode == "per_lane":
        n = 4  # one word, 16384 lanes retrying compare-and-swap: keep the run short
    announce("bench", op, mode, f"T={T} stride={stride} nwg={nwg} n={n}")
    perm_np = sp_inputs.permutation(T, seed)
    finals, s, st = sp.bench_atomic(ctx, op, nwg, lanes, T, stride, mode, n, seed, perm_np)
    U = nwg * lanes if mode == "per_lane" else nwg * (lanes // 64)
    ef, es = oracle.bench_closed(op, seed, U, n, perm_np)
    assert (finals == ef).all()
    if op != "st":
        assert s == es


@pytest.mark.parametrize("mode", ["per_lane", "wave_leader"])
@pytest.mark.parametrize("T", [1, 32, 1024])
def test_exchange_conservation(ctx, mode, T):
    import paper_1110_4623_amd as sp
    nwg, lanes, n, seed = 32, 128, 50, 7
    announce("bench exch", mode, T)
    perm_np = sp_inputs.permutation(T, seed)
    finals, s, _ = sp.bench_atomic(ctx, "exch", nwg, lanes, T, 128, mode, n, seed, perm_np)
    U = nwg * lanes if mode == "per_lane" else nwg * (lanes // 64)
    _, conserved = oracle.bench_closed("exch", seed, U, n, perm_np)
    assert s == conserved
    # every final word is its initial value or a value written to it
    assert oracle.exch_finals_invalid(seed, U, n, perm_np, finals) == 0


def test_full_size_add_sampled(ctx):
    # 2048 workgroups x 256 lanes per-lane adds over 2^20 words: sampled words are
    # compared one by one with the oracle's per-word count, and the total is exact.
    import paper_1110_4623_amd as sp
    nwg, lanes, T, n, seed = 2048, 256, 1 << 20, 200, 42
    announce("bench add full", nwg, lanes, T, n)
    perm_np = sp_inputs.permutation(T, seed)
    finals, s, _ = sp.bench_atomic(ctx, "add", nwg, lanes, T, 128, "per_lane", n, seed, perm_np)
    U = nwg * lanes
    f = finals.astype(np.int64)
    assert int(f.sum()) == U * n
    inv = np.argsort(perm_np)
    rng = np.random.default_rng(0)
    for t in rng.choice(T, 64, replace=False):
        assert f[t] == oracle.bench_count_one(U, n, T, int(inv[t]))


@pytest.mark.parametrize("test", ["cont_vol_read", "cont_vol_write", "noncont_vol_read",
                                  "noncont_vol_write", "cont_atom_read", "cont_atom_write",
                                  "noncont_atom_read", "noncont_atom_write",
                                  "cont_vol_read_after_atom", "cont_vol_write_after_atom",
                                  "noncont_vol_read_after_atom", "noncont_vol_write_after_atom"])
def test_paper12_leaves_zeros(ctx, test):
    # add-of-zero reads and exchange-with-zero writes keep every word at 0 (Section 3)
    import paper_1110_4623_amd as sp
    announce("paper12", test)
    s, words, st = sp.paper12(ctx, test, nwg=256, lanes=64, n_ops=1000, stride=256)
    assert s == 0
    assert int(words.astype(np.int64).sum()) == 0


@pytest.mark.parametrize("n,nwg", [(1 << 24, 0), (3 * (1 << 20) + 20, 7), ((1 << 22) + 4, 64)])
def test_stream_sum(ctx, n, nwg):
    """Every word read once per repetition: the unrolled steps (four loads per lane) and
    the ragged tail, with the default grid and with small ones."""
    import paper_1110_4623_amd as sp
    announce("stream", n, nwg)
    buf = ctx.upload(np.arange(n, dtype=np.uint32))
    s, st = sp.stream_read(ctx, buf, 4 * n, reps=2, nwg=nwg)
    assert s == 2 * (n * (n - 1) // 2)
    if nwg:
        return
    dst = ctx.zeros(n)
    sp.copy(ctx, dst, buf, 4 * n)
    assert (ctx.read(dst, "u32", n) == np.arange(n, dtype=np.uint32)).all()


@pytest.mark.parametrize("fenced", [True, False])
@pytest.mark.parametrize("same_xcd", [False, True])
def test_pingpong(ctx, fenced, same_xcd):
    import paper_1110_4623_amd as sp
    announce("pingpong", f"fenced={fenced} same_xcd={same_xcd}")
    out, st = sp.pingpong(ctx, 1000, fenced=fenced, same_xcd=same_xcd)
    assert out[0] == 2000 and out[1] == 1999
    assert out[2] < 16 and out[3] < 16 and st["kernel_ms"] > 0
    print(f"[pingpong] xcc {out[2]} / {out[3]}, one way {st['kernel_ms'] * 1e6 / 2000:.0f} ns",
          flush=True)


@pytest.mark.parametrize("nwg", [1, 8, 2048])
@pytest.mark.parametrize("mode", ["per_lane", "wave_leader"])
@pytest.mark.parametrize("op", ["add", "cas", "exch", "ld", "st"])
def test_config_grid_at_full_width(ctx, op, mode, nwg):
    """The memory-system grid at its own workgroup counts (up to 2048 x 256 lanes): every
    target count and two strides, every final word (and returned-value sum) against the
    oracle's closed form, with a few operations per issuer.  Compare-and-swap with every
    lane on 1 or 32 words is left out at 2048 workgroups: its retries grow with the square
    of the contenders."""
    import paper_1110_4623_amd as sp
    lanes, seed = 256, 0xC0FFEE
    n = 2 if mode == "per_lane" else 16
    U = nwg * lanes if mode == "per_lane" else nwg * (lanes // 64)
    buf = ctx.zeros((1 << 20) * 128 // 4)
    for T in (1, 32, 1024, 1 << 20):
        if op == "cas" and mode == "per_lane" and nwg == 2048 and T <= 32:
            continue
        perm_np = sp_inputs.permutation(T, seed)
        perm = ctx.upload(perm_np)
        ef, es = oracle.bench_closed(op, seed, U, n, perm_np)
        for stride in (4, 128):
            announce("bench grid", op, mode, f"nwg={nwg} T={T} stride={stride} n={n}")
            finals, s, _ = sp.bench_atomic(ctx, op, nwg, lanes, T, stride, mode, n, seed, perm,
                                           buf)
            if op == "exch":
                assert s == es  # conservation: returned + final = initial + written
                assert oracle.exch_finals_invalid(seed, U, n, perm_np, finals) == 0
            else:
                assert (finals == ef).all(), (T, stride)
                if op != "st":
                    assert s == es


def test_shader_clock_probe(ctx):
    import paper_1110_4623_amd as sp
    mhz = sp.shader_clock_mhz(ctx, 10)
    print(f"[clock] shader clock {mhz:.0f} MHz", flush=True)
    assert 300 < mhz < 4000


@pytest.mark.parametrize("kind", ["release", "acquire"])
def test_fence_cost_alone_and_together(ctx, kind):
    """sp_bench_fence: per-fence clocks are positive and bounded; when 2048 workgroups
    fence at once the span covers at least the slowest workgroup's fence."""
    import paper_1110_4623_amd as sp
    announce("bench fence", kind)
    alone = sp.bench_fence(ctx, kind, 1, 64, reps=50, lines=1)
    assert 0 < alone["clk_per_fence_mean"] < 1e6
    together = sp.bench_fence(ctx, kind, 2048, 64, reps=1, lines=4)
    assert together["clk_per_fence_max"] >= together["clk_per_fence_mean"] > 0
    mhz = sp.shader_clock_mhz(ctx)
    assert together["span_us"] * mhz >= 0.5 * together["clk_per_fence_max"]
    assert together["stats"]["device_error"] == 0


def test_fence_bad_arguments(ctx):
    import ctypes
    import paper_1110_4623_amd as sp
    from paper_1110_4623_amd import _native as N
    out = ctx.zeros(8, "u64")
    st = N.Stats()
    for kind, nwg, reps, lines in ((3, 1, 1, 1), (0, 0, 1, 1), (0, 1, 0, 1), (1, 1, 1, 2000)):
        rc = N.lib.sp_bench_fence(ctx.h, kind, nwg, 64, reps, lines, ctx.ptr(out),
                                  ctypes.byref(st), ctx.stream())
        assert rc == N.SP_E_INVAL
    with pytest.raises(sp.SpError):
        sp.bench_fence(ctx, "acquire", 1 << 17, 64)


def test_pingpong_words_at_an_offset(ctx):
    import paper_1110_4623_amd as sp
    announce("pingpong offset 12288")
    out, _ = sp.pingpong(ctx, 500, fenced=False, offset_bytes=3 * 4096)
    assert out[0] == 1000 and out[1] == 999
    with pytest.raises(ValueError):
        sp.pingpong(ctx, 10, offset_bytes=100)
