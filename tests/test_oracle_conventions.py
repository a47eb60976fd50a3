"""Pins for the oracle's grid and DFT conventions (Sec. 3.1, eq. DFT)."""

import numpy as np
import pytest

from oracle import grids


@pytest.mark.parametrize("shape", [(9,), (8,), (5, 7), (4, 6), (3, 5, 7)])
def test_fft_matches_naive_dft(shape):
    rng = np.random.default_rng(1)
    u = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    size = np.prod(shape)
    # F_M = (1/|M|) omega^{-mk}; F_M^{-1} = omega^{mk}
    np.testing.assert_allclose(grids.dft(u), grids.naive_dft(u, -1) / size, atol=1e-13)
    np.testing.assert_allclose(grids.idft(u), grids.naive_dft(u, +1), atol=1e-12)
    np.testing.assert_allclose(grids.idft(grids.dft(u)), u, atol=1e-13)


def test_wrapped_freqs_is_index_set():
    # eq. index_set: -M/2 <= k < M/2, each once
    for M in (1, 2, 5, 8, 81, 250):
        k = grids.wrapped_freqs(M)
        assert sorted(k.tolist()) == list(range(-(M // 2), M - M // 2))
        assert np.all(np.mod(k, M) == np.arange(M))


def test_trig_poly_values_equal_inverse_dft():
    # eq. trig_conn_raw: values of u_N at x_M^m are the inverse DFT of its coefficients
    rng = np.random.default_rng(2)
    N, M = 5, 11
    uh = np.zeros(M, complex)
    ks = np.arange(-(N // 2), N // 2 + 1)
    c = rng.standard_normal(len(ks)) + 1j * rng.standard_normal(len(ks))
    uh[np.mod(ks, M)] = c
    x = np.arange(M) / M
    direct = np.array([np.sum(c * np.exp(2j * np.pi * ks * xi)) for xi in x])
    np.testing.assert_allclose(grids.idft(uh), direct, atol=1e-13)


def test_smooth_grid():
    assert grids.smooth_grid(81) == 81
    assert grids.smooth_grid(245) == 245
    assert grids.smooth_grid(17) == 21
    assert grids.smooth_grid(29) == 35
    for n in range(1, 400):
        m = grids.smooth_grid(n)
        assert m >= n and m % 2 == 1
