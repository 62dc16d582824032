"""Pins of the oracle's from-scratch DFT: the direct O(n^2) sum on small
sizes (including factors of 3 and a prime), numpy's FFT on large ones, and
Parseval's identity."""
import numpy as np
import pytest

import oracle


def _rand(n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 8, 9, 12, 16, 18, 24, 27, 32, 48, 7])
@pytest.mark.parametrize("sign", [-1, 1])
def test_fft_vs_direct_dft(n, sign):
    x = _rand(n, n)
    a = oracle.fft(x, sign)
    b = oracle.dft(x, sign)
    assert np.max(np.abs(a - b)) <= 1e-13 * max(1.0, np.max(np.abs(b)))


def test_direct_dft_definition():
    """The direct sum itself against the definition on a basis vector."""
    n = 6
    for j in range(n):
        e = np.zeros(n, complex)
        e[j] = 1.0
        out = oracle.dft(e, -1)
        ref = np.exp(-2j * np.pi * np.arange(n) * j / n)
        assert np.max(np.abs(out - ref)) < 1e-14


@pytest.mark.parametrize("n", [128, 256, 96, 384])
def test_fft_vs_numpy(n):
    x = _rand(n, 3)
    assert np.max(np.abs(oracle.fft(x, -1) - np.fft.fft(x))) < 1e-12
    assert np.max(np.abs(oracle.fft(x, 1) - np.fft.ifft(x) * n)) < 1e-12


@pytest.mark.parametrize("L", [4, 6, 12, 24])
def test_fft3_vs_numpy_and_parseval(L):
    rng = np.random.default_rng(L)
    x = rng.standard_normal((L, L, L)) + 1j * rng.standard_normal((L, L, L))
    X = oracle.fft3(x, -1)
    assert np.max(np.abs(X - np.fft.fftn(x))) < 1e-11
    N = L ** 3
    assert abs(np.vdot(X, X).real - N * np.vdot(x, x).real) < 1e-10 * N * np.vdot(x, x).real
    back = oracle.fft3(X, +1) / N
    assert np.max(np.abs(back - x)) < 1e-13
