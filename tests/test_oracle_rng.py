"""Pins of the oracle's counter-based RNG: SplitMix64 published outputs, and
the properties the env layer relies on (counter-based, uniform enough for
the reset pick and the sticky draw)."""
import os

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_seed0.txt")


def test_splitmix64_published_outputs():
    want = [int(l, 16) for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert oracle.splitmix64_stream(0, len(want)) == want


def test_counter_based_draws_are_order_free_and_uniform():
    a = [oracle.rng(7, e, 1, n) for e in range(20) for n in range(50)]
    b = [oracle.rng(7, e, 1, n) for e in reversed(range(20)) for n in range(50)]
    assert sorted(a) == sorted(b)
    assert oracle.rng(7, 3, 1, 5) != oracle.rng(7, 3, 2, 5) != oracle.rng(8, 3, 1, 5)
    picks = np.array([(oracle.rng(1, e, 2, 0) >> 32) % 30 for e in range(30000)])
    counts = np.bincount(picks, minlength=30)
    assert counts.min() > 850 and counts.max() < 1150
    sticky = np.array([(oracle.rng(1, 0, 1, n) >> 32) < 0x40000000 for n in range(40000)])
    assert abs(sticky.mean() - 0.25) < 0.01
