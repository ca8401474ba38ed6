"""Pins for the oracle's A1 generator (SplitMix64 + Box-Muller)."""
import numpy as np

from oracle import rng_ref


def test_splitmix64_published_vectors():
    # First five outputs of SplitMix64 seeded with 1234567, as published with
    # the reference implementation (Steele, Lea, Flood 2014 / Vigna's splitmix64.c).
    expect = [6457827717110365317, 3203168211198807973, 9817491932198370423,
              4593380528125082431, 16408922859458223821]
    assert [rng_ref.splitmix64(1234567, i) for i in range(5)] == expect


def test_uniform_open_interval_and_gaussian_moments():
    u = np.array([rng_ref.uniform53(7, i) for i in range(20000)])
    assert u.min() > 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 0.01
    a = rng_ref.a1_gaussian(42, 2000, 10)
    assert a.shape == (2000, 10)
    assert abs(a.mean()) < 0.02
    assert abs(a.var() - 1.0) < 0.03
    # fourth moment of a standard Gaussian is 3
    assert abs(np.mean(a ** 4) - 3.0) < 0.15


def test_a1_is_counter_based_and_seeded():
    a = rng_ref.a1_gaussian(99, 30, 4)
    b = rng_ref.a1_gaussian(99, 60, 2)     # same stream, other shape
    assert np.array_equal(a.ravel(), b.ravel()[:120])
    c = rng_ref.a1_gaussian(100, 30, 4)
    assert not np.allclose(a, c)
