"""Host-side input generators and schedules (no GPU): the seeded generators
both sides share, and the fixed centre-outwards LED order of the sequential
loop (Sec. 3.1, Eq. 7)."""
import numpy as np
import pytest

from oracle import fpm_oracle as fo
from paper_2408_13782_amd import inputs

from cases import optics_of


@pytest.mark.parametrize("name", ["small", "paper", "large"])
def test_centre_out_order_is_a_ring_order_of_every_led(name):
    """A permutation of the LEDs that starts at the centre LED (k = 0) and never
    moves inwards: |k| is non-decreasing along the order, and equal radii
    (the LEDs of one ring of the square grid) come in increasing angle."""
    w = inputs.workload(name)
    k = fo.led_wavevectors(optics_of(w), w.n_side, w.pitch_mm, w.height_mm)
    order = inputs.centre_out_order(k)
    assert order.dtype == np.int32
    assert sorted(order.tolist()) == list(range(w.n_led))
    centre = (w.n_side // 2) * w.n_side + w.n_side // 2
    assert order[0] == centre
    r = np.round(np.hypot(k[order, 0], k[order, 1]), 9)
    assert np.all(np.diff(r) >= 0)
    ang = np.arctan2(k[order, 0], k[order, 1])
    same = np.diff(r) == 0
    assert np.all(np.diff(ang)[same] > 0)


def test_seeded_generators_are_deterministic_and_seed_dependent():
    """The same seed gives the same arrays, another seed different ones (both
    sides of every parity test build their inputs from these)."""
    a = inputs.random_complex((8, 8), seed=3)
    assert np.array_equal(a, inputs.random_complex((8, 8), seed=3))
    assert not np.array_equal(a, inputs.random_complex((8, 8), seed=4))
    p = inputs.led_permutations(49, 3, seed=1)
    assert p.shape == (3, 49)
    assert all(sorted(row.tolist()) == list(range(49)) for row in p)
    assert np.array_equal(p, inputs.led_permutations(49, 3, seed=1))
    assert not np.array_equal(p[0], p[1])
    idx = inputs.random_indices(225, 16, seed=2)
    assert len(set(idx.tolist())) == 16 and idx.min() >= 0 and idx.max() < 225
