"""Memory-model litmus tests across XCDs: with the fences the primitives use, the
forbidden outcomes never occur (over 4 x 10^6 trials each); without them, how often they
do is reported."""

import pytest

from conftest import announce

pytestmark = pytest.mark.gpu

PAIRS, ITERS = 1024, 4000


@pytest.mark.parametrize("test", ["mp", "sb"])
def test_fenced_never_forbidden(ctx, test):
    import paper_1110_4623_amd as sp
    announce("litmus", test, "fenced", PAIRS, ITERS)
    r = sp.litmus(ctx, test, "fenced", PAIRS, ITERS)
    assert r["stats"]["device_error"] == 0
    print(f"[litmus] {test} fenced: {r['forbidden']} forbidden in {r['trials']} trials", flush=True)
    assert r["forbidden"] == 0


@pytest.mark.parametrize("test,variant", [("mp", "no_acquire"), ("mp", "no_release"),
                                          ("mp", "none"), ("sb", "none")])
def test_unfenced_variants_run(ctx, test, variant):
    import paper_1110_4623_amd as sp
    announce("litmus", test, variant, PAIRS, ITERS)
    r = sp.litmus(ctx, test, variant, PAIRS, ITERS)
    assert r["stats"]["device_error"] == 0
    assert 0 <= r["forbidden"] <= r["trials"]
    print(f"[litmus] {test} {variant}: {r['forbidden']} forbidden in {r['trials']} trials",
          flush=True)


def test_bad_arguments(ctx):
    import paper_1110_4623_amd as sp
    with pytest.raises(sp.SpError):
        sp.litmus(ctx, "mp", "fenced", 2048, 10)  # more pairs than allowed
