"""The seeded input generators (workloads/): SplitMix64 against its published output
sequence, the uniforms it feeds, and strips of a noise field generated on their own."""
import numpy as np

import workloads as W


def test_splitmix64_reference_sequence():
    # SplitMix64 (Steele, Lea, Flood 2014) as a generator: the state advances by the
    # golden-ratio increment and each output is the mix of the new state. From state
    # 1234567 the reference implementation's first five outputs are these.
    golden = np.uint64(0x9E3779B97F4A7C15)
    with np.errstate(over="ignore"):
        states = np.uint64(1234567) + np.arange(5, dtype=np.uint64) * golden
    got = [int(v) for v in W.splitmix64(states)]
    assert got == [6457827717110365317, 3203168211198807973, 9817491932198370423,
                   4593380528125082431, 16408922859458223821]


def test_uniforms_in_unit_interval():
    u = W.uniform01(3, 200000)
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 5e-3
    assert abs(u.var() - 1.0 / 12.0) < 2e-3


def test_noise_rows_are_strips_of_the_field():
    full = W.noise_field(11, 37, 29, 0.25)
    assert full.shape == (29, 37) and np.abs(full).max() <= 0.25
    for y0, y1 in ((0, 29), (0, 1), (5, 17), (28, 29)):
        assert np.array_equal(W.noise_rows(11, 37, y0, y1, 0.25), full[y0:y1])
    # a strip does not depend on how many rows follow it
    assert np.array_equal(W.noise_field(11, 37, 40, 0.25)[:29], full)
