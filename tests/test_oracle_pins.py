"""The oracle against its pins (CPU only)."""
import numpy as np
import pytest

import oracle
from tests.oracle_pins import ALL_PINS


@pytest.mark.parametrize("pin", ALL_PINS, ids=[p.__name__ for p in ALL_PINS])
def test_pin(pin, orc):
    pin(orc)


def test_get_tile_hand_example():
    # Sec. 5.2.3: a group's tiles with 2, 0, 3, 1 atoms own atoms
    # [0, 2), [2, 2), [2, 5), [5, 6): the empty tile owns none.
    assert list(oracle.get_tile_brute([2, 0, 3, 1])) == [0, 0, 2, 2, 2, 3]


def test_get_tile_matches_upper_bound():
    # The owner of atom a is the last tile whose exclusive prefix sum is <= a,
    # i.e. upper_bound(scan, a) - 1 (library search on the scan).
    rng = np.random.default_rng(0)
    for _ in range(50):
        sizes = rng.integers(0, 6, rng.integers(1, 40)) * (rng.random(1) < 0.9)
        scan = np.concatenate([[0], np.cumsum(sizes)])
        atoms = np.arange(scan[-1])
        ub = np.searchsorted(scan, atoms, side="right") - 1
        assert np.array_equal(oracle.get_tile_brute(sizes), ub)
