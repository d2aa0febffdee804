"""Pins for the oracle's input generator (counter-based SplitMix64)."""
import numpy as np
import pytest

import oracle
from golden.load import hex_values


def test_splitmix64_published_sequence():
    # Published reference sequence from state 0 (tests/golden/splitmix64_published.txt).
    want = hex_values("splitmix64_published.txt")
    got = [oracle.splitmix64_at(0, i) for i in range(len(want))]
    assert got == want


def test_counter_form_matches_sequential_stepping():
    # The idx-th output must equal the output after idx+1 sequential steps of the
    # same generator started from another state: shifting the state by k*GAMMA
    # shifts the sequence by k (the defining property of a Weyl-sequence counter).
    gamma = 0x9E3779B97F4A7C15
    s0 = 123456789
    for k in (1, 2, 7, 1000):
        for idx in (0, 5, 99):
            assert oracle.splitmix64_at(s0, idx + k) == oracle.splitmix64_at(
                (s0 + k * gamma) % 2**64, idx)


def test_uniform_values_exact_grid_and_range():
    M = oracle.gen(2304, 0, 257, 31)
    assert M.min() >= -0.5 and M.max() < 0.5
    scaled = (M + 0.5) * 2.0**53
    assert np.all(scaled == np.floor(scaled))  # exactly 53-bit grid, no rounding


def test_uniform_statistics():
    M = oracle.gen(7, 0, 2000, 100).ravel(order="F")
    n = M.size
    assert abs(M.mean()) < 4 * np.sqrt(1 / 12 / n)
    assert abs(M.var() - 1 / 12) < 4 * np.sqrt(1 / 180 / n)
    counts, _ = np.histogram(M, bins=20, range=(-0.5, 0.5))
    chi2 = ((counts - n / 20) ** 2 / (n / 20)).sum()
    assert chi2 < 45.3  # chi-square 19 dof, p = 0.001


def test_layout_and_leading_dimension():
    a = oracle.gen(11, 1, 40, 9)
    b = oracle.gen(11, 1, 40, 9, ld=47)
    assert np.array_equal(a, b)
    flat = oracle.gen(11, 1, 40 * 9, 1)[:, 0]
    assert np.array_equal(a.ravel(order="F"), flat)  # index i + j*rows


def test_streams_and_seeds_differ():
    a = oracle.gen(5, 0, 64, 64)
    assert not np.array_equal(a, oracle.gen(5, 1, 64, 64))
    assert not np.array_equal(a, oracle.gen(6, 0, 64, 64))
    c = np.corrcoef(a.ravel(), oracle.gen(5, 1, 64, 64).ravel())[0, 1]
    assert abs(c) < 0.1


def test_conversion_of_published_outputs():
    # value = (top 53 bits of the 64-bit output) * 2^-53 - 1/2, evaluated exactly
    from fractions import Fraction
    for idx, h in enumerate(hex_values("splitmix64_published.txt")):
        want = Fraction(h >> 11, 2**53) - Fraction(1, 2)
        assert Fraction(oracle.uniform(0, idx)) == want
