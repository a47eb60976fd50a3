"""Closed-form Fourier coefficients (Sec. 2.2 convention; Remark anal_Fourier).

The Fourier coefficient of a Y-periodic f is fhat(k) = int_Y f(x) exp(-2 pi i k.x) dx,
so a translate f(x - x0) has coefficients exp(-2 pi i k.x0) fhat(k)
(the factor phi_{-k}(x0) of eq. inclcomp_formula).
"""

from __future__ import annotations

import numpy as np
from scipy.special import j1


def sinc(x):
    """sinc(x) = sin(pi x)/(pi x), sinc(0) = 1 (as defined after eq. char_func_Four)."""
    return np.sinc(x)


def rect_hat(k, h):
    """Box of side lengths h centred at 0: prod_a h_a sinc(h_a k_a) (eq. def_cube)."""
    out = np.ones(k.shape[1:])
    for a in range(k.shape[0]):
        out = out * h[a] * sinc(h[a] * k[a])
    return out


def tri_hat(k, h):
    """Tensor-product hat function: prod_a h_a sinc^2(h_a k_a) (eq. def_tri)."""
    out = np.ones(k.shape[1:])
    for a in range(k.shape[0]):
        out = out * h[a] * sinc(h[a] * k[a]) ** 2
    return out


def circ_hat(k, r):
    """Disc of radius r centred at 0 (2D): pi r^2 at k = 0, else r J_1(2 pi r |k|)/|k|."""
    kn = np.sqrt(np.sum(k.astype(float) ** 2, axis=0))
    safe = np.where(kn > 0, kn, 1.0)
    return np.where(kn > 0, r * j1(2 * np.pi * r * safe) / safe, np.pi * r * r)


def shift_phase(k, x0):
    """phi_{-k}(x0) = exp(-2 pi i k.x0), the coefficient factor of a translate."""
    arg = np.zeros(k.shape[1:])
    for a in range(k.shape[0]):
        arg = arg + k[a] * x0[a]
    return np.exp(-2j * np.pi * arg)
