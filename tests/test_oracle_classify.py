"""Pins of the oracle's critical point detection (CD, Section IV-A (1))."""
import numpy as np
import pytest

from np_ref import MAX, MIN, R, SAD, classify_np


@pytest.mark.parametrize("shape", [(1, 1), (1, 7), (7, 1), (2, 2), (3, 3), (5, 9), (64, 65),
                                   (33, 70), (1, 1, 5), (2, 3, 4), (5, 6, 7), (1, 9, 9),
                                   (17, 1, 13), (12, 12, 12)])
def test_classifier_matches_numpy_restatement(ora, shape):
    rng = np.random.default_rng(hash(shape) % 2 ** 32)
    for trial in range(3):
        if trial == 0:
            f = rng.standard_normal(shape).astype(np.float32)
        elif trial == 1:  # many ties
            f = rng.integers(0, 3, shape).astype(np.float32)
        else:  # signed zeros and denormals
            f = rng.choice(np.array([0.0, -0.0, 1e-45, -1e-45, 1.0], np.float32), shape)
        assert np.array_equal(ora.classify(f), classify_np(f))


def test_label_codes_and_boundary_counts(ora):
    """Codes r=0, m=1, s=2, M=3 (Section IV-A (1)); corners use two
    neighbours and edges three."""
    assert (R, MIN, SAD, MAX) == (ora.R, ora.MIN, ora.SAD, ora.MAX) == (0, 1, 2, 3)
    f = np.array([[0, 5, 0], [5, 2, 5], [0, 5, 0]], np.float32)
    c = ora.classify(f)
    assert c[0, 0] == MIN and c[0, 2] == MIN and c[2, 0] == MIN and c[2, 2] == MIN
    assert c[0, 1] == MAX and c[1, 0] == MAX  # edge points: 3 lower neighbours
    assert c[1, 1] == MIN  # all four higher
    g = np.array([[0, 9, 0], [1, 5, 1], [0, 9, 0]], np.float32)
    assert ora.classify(g)[1, 1] == SAD  # t, d higher; l, r lower
    h = np.array([[0, 1, 0], [9, 5, 9], [0, 1, 0]], np.float32)
    assert ora.classify(h)[1, 1] == SAD  # the "vice versa" pattern
    k = np.array([[0, 9, 0], [1, 5, 6], [0, 9, 0]], np.float32)
    assert ora.classify(k)[1, 1] == R  # mixed pair -> regular
    # ties are never critical (strict comparisons)
    assert ora.classify(np.array([[1, 1], [1, 1]], np.float32)).max() == R


def test_iid_noise_densities_2d(ora):
    """For i.i.d. continuous values the interior probabilities are
    P(m) = P(M) = 1/5 and P(s) = 2 * 2!2!/5! = 1/15."""
    f = np.random.default_rng(0).standard_normal((700, 700)).astype(np.float32)
    c = ora.classify(f)[1:-1, 1:-1]
    n = c.size
    for cls, p in [(MIN, 1 / 5), (MAX, 1 / 5), (SAD, 1 / 15)]:
        got = np.mean(c == cls)
        assert abs(got - p) < 6 * np.sqrt(p * (1 - p) / n) + 1e-3, (cls, got, p)


def test_iid_noise_densities_3d(ora):
    """3D, six face neighbours: P(m) = P(M) = 1/7; saddles need each axis pair
    uniform and both kinds present: 6 * 2!4!/7! = 2/35."""
    f = np.random.default_rng(1).standard_normal((72, 72, 72)).astype(np.float32)
    c = ora.classify(f)[1:-1, 1:-1, 1:-1]
    n = c.size
    for cls, p in [(MIN, 1 / 7), (MAX, 1 / 7), (SAD, 2 / 35)]:
        got = np.mean(c == cls)
        assert abs(got - p) < 6 * np.sqrt(p * (1 - p) / n) + 1e-3, (cls, got, p)


def test_signed_zero_equal(ora):
    f = np.array([[0.0, -0.0, 0.0]], np.float32)
    assert ora.classify(f).max() == R
