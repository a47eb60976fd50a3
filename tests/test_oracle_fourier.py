"""Pins for the closed-form Fourier coefficients (Remark anal_Fourier) against quadrature.

The coefficient int_Y f(x) exp(-2 pi i k.x) dx of each indicator is computed by
adaptive numerical integration over the shape itself, independently of the
sinc / Bessel closed forms.
"""

import math

import numpy as np
import pytest
from scipy import integrate

from oracle import fourier

KS = [(0, 0), (1, 0), (0, 3), (2, -1), (5, 7), (-11, 4)]


def _quad_rect(k, h, x0=(0.0, 0.0)):
    def f(part):
        g = (lambda y, x: math.cos(2 * math.pi * (k[0] * x + k[1] * y))) if part == 0 else \
            (lambda y, x: -math.sin(2 * math.pi * (k[0] * x + k[1] * y)))
        v, _ = integrate.dblquad(g, x0[0] - h[0] / 2, x0[0] + h[0] / 2,
                                 x0[1] - h[1] / 2, x0[1] + h[1] / 2, epsabs=1e-13, epsrel=1e-13)
        return v
    return f(0) + 1j * f(1)


def _quad_tri(k, h):
    def tent(t, w):
        return max(1.0 - abs(t / w), 0.0)
    g = lambda y, x: tent(x, h[0]) * tent(y, h[1]) * math.cos(2 * math.pi * (k[0] * x + k[1] * y))
    v, _ = integrate.dblquad(g, -h[0], h[0], -h[1], h[1], epsabs=1e-13, epsrel=1e-13)
    return v


def _quad_circ(k, r):
    g = lambda y, x: math.cos(2 * math.pi * (k[0] * x + k[1] * y))
    v, _ = integrate.dblquad(g, -r, r, lambda x: -math.sqrt(max(r * r - x * x, 0.0)),
                             lambda x: math.sqrt(max(r * r - x * x, 0.0)), epsabs=1e-13, epsrel=1e-13)
    return v


@pytest.mark.parametrize("k", KS)
def test_rect_hat(k):
    h = (0.6, 0.35)
    kk = np.array(k).reshape(2, 1)
    np.testing.assert_allclose(fourier.rect_hat(kk, h)[0], _quad_rect(k, h).real, atol=1e-11)


@pytest.mark.parametrize("k", KS)
def test_tri_hat(k):
    h = (0.3, 0.2)
    kk = np.array(k).reshape(2, 1)
    np.testing.assert_allclose(fourier.tri_hat(kk, h)[0], _quad_tri(k, h), atol=1e-11)


@pytest.mark.parametrize("k", KS)
def test_circ_hat(k):
    r = 0.3090194
    kk = np.array(k).reshape(2, 1)
    np.testing.assert_allclose(fourier.circ_hat(kk, r)[0], _quad_circ(k, r), atol=1e-10)


@pytest.mark.parametrize("k", [(1, 0), (2, -1), (3, 5)])
def test_shift_phase(k):
    h, x0 = (0.3, 0.2), (0.137, -0.271)
    kk = np.array(k).reshape(2, 1)
    val = fourier.rect_hat(kk, h)[0] * fourier.shift_phase(kk, x0)[0]
    np.testing.assert_allclose(val, _quad_rect(k, h, x0), atol=1e-11)
