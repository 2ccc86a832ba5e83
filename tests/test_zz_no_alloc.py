"""The allocation-free bounded buffer (sp_cond_run_bounded_buffer_noalloc) against the
allocating entry point: the same unique outputs on two calls in a row, the second on a
smaller input, and a clear refusal of inputs beyond its fixed workspace."""

import ctypes

import numpy as np
import pytest

from conftest import announce

pytestmark = pytest.mark.gpu


def _both(ctx, kind, nwg, producers, cap, items, seed, lanes=64):
    import paper_1110_4623_amd as sp
    announce("bounded buffer noalloc vs alloc", kind, nwg, producers, cap, items)
    ref = sp.bounded_buffer(ctx, kind, nwg, producers, cap, items, seed, lanes=lanes,
                            values=True)
    got = sp.bounded_buffer(ctx, kind, nwg, producers, cap, items, seed, lanes=lanes,
                            values=True, noalloc=True)
    return ref, got


def test_noalloc_matches_the_allocating_call_twice_second_smaller(ctx):
    seed = 0xC0FFEE
    for kind, nwg, producers, cap, items, lanes in (("array", 2048, 1024, 64, 1 << 14, 256),
                                                   ("ticket", 9, 4, 4, 1000, 64)):
        ref, got = _both(ctx, kind, nwg, producers, cap, items, seed, lanes)
        # unique outputs: what was taken and put, element by element as multisets
        for k in ("xor", "sum", "taken", "put", "left"):
            assert got[k] == ref[k], k
        assert got["taken"] == items and got["left"] == 0
        assert (np.sort(got["values"]) == np.sort(ref["values"])).all()
        # not unique: the ring's peak fill depends on timing; both stay within the capacity
        assert 1 <= got["max_count"] <= cap and 1 <= ref["max_count"] <= cap


def test_noalloc_refuses_what_does_not_fit(ctx):
    import paper_1110_4623_amd as sp
    from paper_1110_4623_amd import _native as N
    p = sp.make_params()
    out = ctx.zeros(6, "u64")
    st = N.Stats()
    rc = N.lib.sp_cond_run_bounded_buffer_noalloc(ctx.h, N.MUTEX_KINDS["ticket"], 16, 8, 64,
                                                  1 << 20, 1000, 1, ctypes.byref(p),
                                                  ctx.ptr(out), None, ctypes.byref(st),
                                                  ctx.stream())
    assert rc == N.SP_E_RANGE
    assert "fixed workspace" in N.lib.sp_strerror(rc).decode()
