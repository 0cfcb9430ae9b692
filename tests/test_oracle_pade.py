"""Pins of the oracle's Pade coefficients (Sec. 2; Algorithm 1, first step).

Each check compares against something other than the oracle's own construction:
a closed form, the target function evaluated directly, or an invariant of the
approximant.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle.pade import pade, taylor_coefficients


def f_direct(x, sigma):
    return np.exp(1j * sigma * (np.sqrt(1.0 + np.asarray(x, dtype=np.complex128)) - 1.0))


@pytest.mark.parametrize("sigma", [0.3, 2.094395102393196, 16.755160819145562])
def test_order1_closed_form(sigma):
    # The [1/1] approximant of exp(i s (sqrt(1+x)-1)) is (1 + (1+is)x/4)/(1 + (1-is)x/4):
    # from f1 = is/2, f2 = -is/8 - s^2/8, q1 = -f2/f1, p1 = f1 + q1.
    c = pade(sigma, 1)
    assert abs(c.b[0] - (1 - 1j * sigma) / 4) < 1e-14 * (1 + sigma)
    assert abs(c.a[0] - (1 + 1j * sigma) / 4) < 1e-14 * (1 + sigma)
    x = np.linspace(-3, 0.5, 7)
    R = (1 + (1 + 1j * sigma) * x / 4) / (1 + (1 - 1j * sigma) * x / 4)
    assert np.max(np.abs(c.R(x) - R)) < 1e-13


def test_taylor_coefficients_match_numerical_series():
    # independent route to the Taylor coefficients: mpmath's high-precision numerical
    # differentiation of the function itself
    sigma = 5.235987755982989
    f = taylor_coefficients(sigma, 10)
    with mp.workdps(40):
        ref = mp.taylor(lambda x: mp.exp(1j * sigma * (mp.sqrt(1 + x) - 1)), 0, 10)
    for a, b in zip(f, ref):
        assert abs(complex(a) - complex(b)) <= 1e-20 + 1e-12 * abs(complex(b))


def _series_about(c, x0, n):
    """Taylor coefficients of R = d0 + sum d_j/(1 + b_j x) about x0, from the sum form."""
    out = [complex(c.d0)] + [0j] * n
    for dj, bj in zip(c.d, c.b):
        den = 1 + bj * x0
        beta = bj / den
        for k in range(n + 1):
            out[k] += dj / den * (-beta) ** k
    return out


def _f_series(sigma, x0, n):
    with mp.workdps(40):
        return [complex(v) for v in mp.taylor(
            lambda x: mp.exp(1j * sigma * (mp.sqrt(1 + x) - 1)), x0, n)]


@pytest.mark.parametrize("sigma,p", [(2.094395102393196, 4), (5.235987755982989, 6),
                                     (16.755160819145562, 8)])
def test_matching_order(sigma, p):
    # R agrees with f through x^(2p) and not at x^(2p+1); f's coefficients come from
    # numerical differentiation of the function itself
    c = pade(sigma, p)
    R = _series_about(c, 0.0, 2 * p + 1)
    f = _f_series(sigma, 0.0, 2 * p + 1)
    scale = float(np.sum(np.abs(c.d)) + 1)
    for k in range(2 * p + 1):
        assert abs(R[k] - f[k]) < 1e-13 * scale * max(1.0, abs(f[k]))
    assert abs(R[2 * p + 1] - f[2 * p + 1]) > 1e-6 * abs(f[2 * p + 1])


def test_matching_order_rotated():
    # the rotated approximant matches f through order 2p about Z = 0, i.e. about
    # x* = e^{i alpha} - 1, where sqrt(1+x) = e^{i alpha/2} sqrt(1+Z)
    sigma, p, alpha = 2.094395102393196, 4, math.pi / 16
    c = pade(sigma, p, alpha)
    x0 = complex(np.exp(1j * alpha) - 1.0)
    R = _series_about(c, x0, 2 * p + 1)
    f = _f_series(sigma, x0, 2 * p + 1)
    scale = float(np.sum(np.abs(c.d)) + 1)
    for k in range(2 * p + 1):
        assert abs(R[k] - f[k]) < 1e-12 * scale * max(1.0, abs(f[k]))
    assert abs(R[2 * p + 1] - f[2 * p + 1]) > 1e-6 * abs(f[2 * p + 1])


@pytest.mark.parametrize("sigma,p", [(2.094395102393196, 4), (5.235987755982989, 6),
                                     (16.755160819145562, 8), (41.8879, 4)])
def test_standard_is_unitary_on_real_axis(sigma, p):
    # f has unit modulus for real x > -1 and its Taylor coefficients satisfy
    # P = conj(Q) structure, so the approximant is unitary on the real axis and its
    # numerator coefficients are the conjugates of the denominator ones.
    c = pade(sigma, p)
    x = np.concatenate([np.linspace(-200, -1, 400), np.linspace(-1, 5, 400)])
    assert np.max(np.abs(np.abs(c.R(x)) - 1.0)) < 1e-12
    assert np.max(np.abs(c.a - np.conj(c.b))) < 1e-12 * np.max(np.abs(c.b))
    assert abs(c.C - 1) < 1e-14


@pytest.mark.parametrize("alpha", [0.0, math.pi / 16])
def test_sum_equals_product(alpha):
    c = pade(5.235987755982989, 6, alpha)
    rng = np.random.default_rng(3)
    x = rng.uniform(-60, 1, 50) + 1j * rng.uniform(-1, 1, 50)
    assert np.max(np.abs(c.R(x) - c.R_product(x))) < 1e-11


def test_rotated_damps_evanescent_and_is_stable():
    # homogeneous-waveguide settings: sigma = k0 dr with k0 = 2 pi 100/1500, dr = 5 m
    k0 = 2 * math.pi * 100 / 1500
    c = pade(k0 * 5.0, 4, math.pi / 16)
    ell = np.arange(1, 257)
    x = -(ell * math.pi / (200.0 * k0)) ** 2
    G = np.exp(1j * k0 * 5.0) * c.R(x)
    assert np.max(np.abs(G)) < 1 + 1e-7
    assert np.max(np.abs(G[x < -1.5])) < 0.97          # evanescent modes decay every step


def test_factor_order_rule():
    c = pade(5.235987755982989, 6)
    args = np.angle(c.b)
    assert np.all(np.diff(args) >= 0)
