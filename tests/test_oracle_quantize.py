"""Pins of the oracle's quantizer (QZ, Section II-C) and bound rounding."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from np_ref import q_exact

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _edges_cases():
    rng = np.random.default_rng(11)
    cases = []
    for e in [0.01, 2.0 ** -10, 1.0, 0.1, 3e-7, 123.456, 2.0 ** -100, 2.0 ** 20]:
        ef = float(np.float32(e))
        for k in [-5, -1, 0, 1, 2, 7, 1000, 4194302]:
            edge = (2 * k + 1) * ef  # bin edge, exact in float64
            for v in [edge, np.nextafter(np.float32(edge), np.float32(np.inf)),
                      np.nextafter(np.float32(edge), np.float32(-np.inf))]:
                if abs(float(v)) < 3e38:
                    cases.append((float(np.float32(v)), ef))
        for a in rng.normal(0, 50 * ef, 20):
            cases.append((float(np.float32(a)), ef))
    # signed zeros, denormals, values just below a power-of-two bound
    for e in [2.0 ** -10, 2.0 ** -90, 0.25]:
        ef = float(np.float32(e))
        for a in [0.0, -0.0, 1e-45, -1e-45, 1e-39, ef, -ef,
                  float(np.nextafter(np.float32(ef), np.float32(0))),
                  float(np.nextafter(np.float32(-ef), np.float32(0)))]:
            cases.append((float(np.float32(a)), ef))
    return cases


def test_quantize_matches_exact_definition(ora):
    """q is floor((a+e)/(2e)) in exact rational arithmetic, i.e. the unique
    integer with (2q-1)e <= a < (2q+1)e."""
    for a, e in _edges_cases():
        rc, q = ora.quantize(a, e)
        qe = q_exact(a, e)
        if abs(qe) > 2 ** 22 - 1:
            assert rc == ora.E_RANGE
            continue
        assert rc == ora.OK, (a, e)
        assert q == qe, (a, e, q, qe)
        A, E = Fraction(a), Fraction(e)
        assert (2 * q - 1) * E <= A < (2 * q + 1) * E


def test_quantize_random_exact(ora):
    rng = np.random.default_rng(5)
    for _ in range(3000):
        e = float(np.float32(10.0 ** rng.uniform(-6, 2)))
        a = float(np.float32(rng.normal(0, 1) * e * 10.0 ** rng.uniform(0, 5)))
        rc, q = ora.quantize(a, e)
        qe = q_exact(a, e)
        if abs(qe) > 2 ** 22 - 1:
            assert rc == ora.E_RANGE
        else:
            assert rc == ora.OK and q == qe


def test_reconstruction_is_bin_centre_within_bound(ora):
    """|a - R(q)| <= e + half an ulp of R(q): the SZp guarantee (Section II-C)
    with R(q) = float(2q e) rounded once."""
    rng = np.random.default_rng(7)
    for _ in range(2000):
        e = float(np.float32(10.0 ** rng.uniform(-5, 1)))
        a = float(np.float32(rng.uniform(-1e3, 1e3) * e))
        rc, q = ora.quantize(a, e)
        assert rc == ora.OK
        r = ora.recon(q, e)
        assert r == np.float32(Fraction(2 * q) * Fraction(e))  # correctly rounded product
        half_ulp = float(np.spacing(np.float32(abs(r)))) / 2
        assert abs(Fraction(a) - Fraction(float(r))) <= Fraction(e) + Fraction(half_ulp)


def test_quantizer_and_reconstruction_monotone(ora):
    """a1 < a2 implies q1 <= q2 and R(q1) <= R(q2) (Section III-B premise)."""
    e = float(np.float32(0.003))
    xs = np.sort(np.random.default_rng(3).uniform(-2, 2, 4000).astype(np.float32))
    qs = [ora.quantize(float(x), e)[1] for x in xs]
    rs = [float(ora.recon(q, e)) for q in qs]
    assert all(a <= b for a, b in zip(qs, qs[1:]))
    assert all(a <= b for a, b in zip(rs, rs[1:]))
    # strictly increasing bin centres
    assert all(float(ora.recon(k, e)) < float(ora.recon(k + 1, e)) for k in range(-700, 700))


def test_eps_float_is_largest_float_not_above(ora):
    rng = np.random.default_rng(9)
    for x in list(10.0 ** rng.uniform(-30, 30, 500)) + [0.1, 1e-3, 0.01, 1.0, 2.0 ** -10]:
        ef = ora.eps_float(x)
        assert Fraction(ef) <= Fraction(x)
        nxt = float(np.nextafter(np.float32(ef), np.float32(np.inf)))
        assert Fraction(nxt) > Fraction(x)


def test_range_limits(ora):
    e = 1.0
    assert ora.quantize(float(2 ** 23), e)[0] == ora.E_RANGE
    assert ora.quantize(float((2 * (2 ** 22 - 1)) * 1.0), e)[0] == ora.OK
    assert ora.quantize(float("nan"), e)[0] == ora.E_NONFINITE
    assert ora.quantize(float("inf"), e)[0] == ora.E_NONFINITE


def test_fig2_worked_example(ora):
    """Section III-A, Fig. 2: peak 0.012 with four 0.01 neighbours, eps = 0.01:
    every value maps to bin 1 and the maximum is flattened."""
    g = json.load(open(os.path.join(GOLDEN, "fig2_flattened_max.json")))
    f = np.array(g["field"], dtype=np.float32)
    e = ora.eps_float(g["eps"])
    rc, q = ora.quantize_field(f, e)
    assert rc == ora.OK
    assert q.tolist() == g["expected_q"]
    r = (2 * q).astype(np.float32) * np.float32(e)
    # bin-centre reconstruction: all five points collapse to 2e
    assert all(r[i][j] == np.float32(g["expected_recon_centre_bin"])
               for i, j in [(1, 1), (0, 1), (1, 0), (1, 2), (2, 1)])
    cls_orig = ora.classify(f)
    cls_rec = ora.classify(r)
    assert cls_orig[1, 1] == ora.MAX and cls_rec[1, 1] == ora.R
