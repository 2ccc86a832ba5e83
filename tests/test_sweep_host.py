"""Host logic of the measurement sweeps (no GPU): operation-count scaling."""


def test_scaled_counts_fit_the_budget():
    from paper_1110_4623_amd.sweep import _scaled
    # 1000 operations took 10 ms: 0.15 s fits 15000
    assert _scaled(10 ** 6, 1000, 10.0, 0.15, 1) == 15000
    # never more than the workload's full count, never fewer than the floor
    assert _scaled(5000, 1000, 1.0, 10.0, 1) == 5000
    assert _scaled(10 ** 6, 1000, 1e4, 0.01, 64) == 64
    # a zero-time pilot does not divide by zero
    assert _scaled(100, 10, 0.0, 1.0, 1) == 100
