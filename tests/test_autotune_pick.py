"""Host-side choice of the number of G-block copies (no GPU)."""
from paper_2511_21535_amd import autotune


def _t(shape, ms_by_copies):
    return {str(list(shape) + [c]): ms for c, ms in ms_by_copies.items()}


def test_fewest_copies_within_margin():
    shape = (4, 1, 64)
    # timing noise between copy counts: one copy is kept
    assert autotune.pick_copies(_t(shape, {1: 32.23, 2: 32.24, 4: 32.26, 8: 32.15}), shape) == (4, 1, 64, 1)
    # a clear gain for two copies
    assert autotune.pick_copies(_t(shape, {1: 40.0, 2: 36.0, 4: 35.9, 8: 36.5}), shape) == (4, 1, 64, 2)
    # the fastest time may belong to another launch shape with one copy
    t = _t(shape, {1: 40.0, 2: 39.5, 4: 39.0, 8: 38.0})
    t[str([2, 2, 32, 1])] = 30.0
    assert autotune.pick_copies(t, shape) == (2, 2, 32, 1)
