"""Condition variables on the GPU: the bounded buffer's consumers take exactly what its
producers put (xor and sum against the oracle's closed form), the ring never holds more
than its capacity, and it ends empty."""

import numpy as np
import pytest

import oracle
from conftest import announce

pytestmark = pytest.mark.gpu


def _run(ctx, kind, nwg, producers, cap, items, seed, lanes=64, **params):
    import paper_1110_4623_amd as sp
    announce("bounded buffer", kind, f"nwg={nwg} producers={producers} cap={cap} items={items}",
             params)
    return sp.bounded_buffer(ctx, kind, nwg, producers, cap, items, seed, lanes=lanes,
                             values=True, **params)


def _check(r, producers, cap, items, seed):
    assert (r["xor"], r["sum"]) == oracle.bb_closed(seed, producers, items)
    assert r["taken"] == r["put"] == items and r["left"] == 0
    assert 1 <= r["max_count"] <= cap
    # value by value: the multiset taken is exactly the multiset put (which consumer took
    # which value is not unique, so both sides are compared sorted)
    assert (np.sort(r["values"]) == np.sort(oracle.bb_values(seed, producers, items))).all()


@pytest.mark.parametrize("kind", ["ticket", "array", "sleep", "spin_cas", "cohort"])
@pytest.mark.parametrize("cap", [1, 16, 1024])
@pytest.mark.parametrize("nwg,producers", [(2, 1), (9, 4), (64, 32)])
def test_small(ctx, kind, cap, nwg, producers):
    seed, items = 42, 3000
    r = _run(ctx, kind, nwg, producers, cap, items, seed)
    _check(r, producers, cap, items, seed)


@pytest.mark.parametrize("kind", ["ticket", "array", "cohort"])
@pytest.mark.parametrize("cap", [1, 64])
def test_full_width(ctx, kind, cap):
    # 2048 workgroups of 256 lanes: 1024 producers, 1024 consumers
    seed, items, nwg = 0xC0FFEE, 1 << 15, 2048
    r = _run(ctx, kind, nwg, 1024, cap, items, seed, lanes=256)
    _check(r, 1024, cap, items, seed)


def test_uneven_roles(ctx):
    seed, items = 7, 5000
    for producers, nwg in ((1, 64), (63, 64)):
        r = _run(ctx, "ticket", nwg, producers, 8, items, seed, poll_sleep=2)
        _check(r, producers, 8, items, seed)


def test_bad_arguments(ctx):
    import paper_1110_4623_amd as sp
    with pytest.raises(sp.SpError):
        sp.bounded_buffer(ctx, "ticket", 4, 4, 8, 100, 1)  # no consumers
    with pytest.raises(sp.SpError):
        sp.bounded_buffer(ctx, "ring", 4, 2, 8, 100, 1)  # not a supported mutex
    with pytest.raises(sp.SpNotResident):
        sp.bounded_buffer(ctx, "ticket", 1 << 16, 8, 8, 100, 1, lanes=1024)
