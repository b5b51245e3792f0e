"""Pins for the oracle's cubic B-spline basis (the B_l of Eq. 1, Sec. 2.1).

Each check is fixed by the mathematics of the uniform cubic B-spline, not by
re-typing the oracle's formula: exact rational values, partition of unity, moment
identities, symmetry, C2 joins, and scipy's independent de Boor evaluation.
"""
from fractions import Fraction

import numpy as np
import pytest
from scipy.interpolate import BSpline

import oracle
from oracle import brute

US = np.concatenate([np.linspace(0.0, 1.0, 41), np.random.default_rng(7).uniform(0, 1, 200)])


def test_node_weights():
    # At a control-point position (u = 0) the cubic B-spline weights are 1/6, 4/6, 1/6.
    np.testing.assert_allclose(oracle.basis(0.0), [1 / 6, 4 / 6, 1 / 6, 0.0], rtol=0, atol=1e-16)


@pytest.mark.parametrize("u,expect", [
    (Fraction(1, 2), [Fraction(1, 48), Fraction(23, 48), Fraction(23, 48), Fraction(1, 48)]),
    (Fraction(1, 4), [Fraction(27, 384), Fraction(235, 384), Fraction(121, 384), Fraction(1, 384)]),
    (Fraction(1, 3), [Fraction(8, 162), Fraction(93, 162), Fraction(60, 162), Fraction(1, 162)]),
])
def test_exact_rational_values(u, expect):
    # Values of the centred kernel beta3 at the four integer-shifted distances,
    # evaluated in exact rational arithmetic, must match.
    exact = [brute.beta3(u + 1), brute.beta3(u), brute.beta3(1 - u), brute.beta3(2 - u)]
    assert exact == expect
    np.testing.assert_allclose(oracle.basis(float(u)), [float(e) for e in expect], rtol=0, atol=1e-16)


def test_partition_of_unity():
    for u in US:
        assert abs(oracle.basis(u).sum() - 1.0) < 1e-15


def test_moments_reproduce_polynomials():
    # sum_l (l-1)^k B_l(u) equals the k-th moment identity of the cubic B-spline:
    # u (linear reproduction), u^2 + 1/3 (variance 1/3), u^3 + u.
    for u in US:
        B = oracle.basis(u)
        a = np.arange(4) - 1.0
        assert abs((a * B).sum() - u) < 1e-15
        assert abs((a ** 2 * B).sum() - (u * u + 1 / 3)) < 1e-14
        assert abs((a ** 3 * B).sum() - (u ** 3 + u)) < 1e-14


def test_symmetry():
    for u in US:
        np.testing.assert_allclose(oracle.basis(u), oracle.basis(1.0 - u)[::-1], rtol=0, atol=1e-15)


def test_scipy_de_boor():
    # Cardinal cubic B-spline on knots 0..4 (scipy, de Boor recursion): B_l(u) = N(u + 3 - l).
    N = BSpline.basis_element(np.arange(5.0), extrapolate=False)
    for u in US[US < 1.0]:
        ref = [N(u + 3 - l) for l in range(4)]
        np.testing.assert_allclose(oracle.basis(u), ref, rtol=0, atol=1e-15)
        # the brute-force kernel is the same function, centred
        for l in range(4):
            assert abs(brute.beta3(u + 1 - l) - N(u + 3 - l)) < 1e-15


def test_c2_join_between_tiles():
    # Tile t at u -> 1 and tile t+1 at u = 0 see the same four control points
    # shifted by one: value, first and second derivative must agree (C2, Sec. 1).
    def deriv(u, k, h=0.05):
        # five-point stencils, exact for polynomials of degree <= 4 (each piece is cubic)
        f = {j: oracle.basis(u + j * h) for j in (-2, -1, 0, 1, 2)}
        if k == 1:
            return (8 * (f[1] - f[-1]) - (f[2] - f[-2])) / (12 * h)
        return (-f[2] + 16 * f[1] - 30 * f[0] + 16 * f[-1] - f[-2]) / (12 * h * h)

    left, right = oracle.basis(1.0), oracle.basis(0.0)
    np.testing.assert_allclose(left[1:], right[:3], atol=1e-15)
    assert abs(left[0]) < 1e-16 and abs(right[3]) < 1e-16
    for k in (1, 2):
        dl, dr = deriv(1.0, k), deriv(0.0, k)
        np.testing.assert_allclose(dl[1:], dr[:3], atol=1e-11)
