"""Section 4's machine card measured on the GPU: the twelve tests of Section 3 (Table 1)
at a saturating grid, their data path checked exactly, and the three parameters of the
abstraction derived from their times."""

import math

import pytest

from conftest import announce

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nwg", [256, 2048])
def test_machine_card_on_this_gpu(ctx, nwg):
    import paper_1110_4623_amd as sp
    from paper_1110_4623_amd import abstraction
    times = {}
    for key, test in abstraction._TEST_OF_KEY.items():
        announce("paper12", test, nwg)
        s, words, st = sp.paper12(ctx, test, nwg=nwg, lanes=64, n_ops=1000, stride=256)
        # every access reads or writes 0 (atomic read = add of 0, atomic write = exchange
        # with 0, volatile write stores 0): the loaded sum and every word stay 0
        assert s == 0, test
        assert not words.any(), test
        assert st["ops"] == nwg * 1000
        times[key] = st["kernel_ms"]
    card = abstraction.card(times)
    for name in ("atomic_to_volatile", "contentious_to_noncontentious_volatile",
                 "volatile_after_atomic_to_volatile"):
        for col in ("read", "write"):
            v = card[name][col]
            assert math.isfinite(v) and v > 0, (name, col, v)
    # contended atomics on one word cost more than contended loads of it: the property
    # that rules out spinning with atomics (Section 4)
    assert card["atomic_to_volatile"]["read"] > 1.0
    assert set(card["atomic_unit_holds_line_hostage"]) == {"read", "write"}
