"""Pins of the oracle's transforms against the DFT definition (brute force),
an independent third-party FFT (numpy.fft, test-only), Parseval and exact
spectral derivatives of trigonometric modes (pseudo-spectral discretization,
Sec. 2.3 / Sec. 3)."""
import numpy as np
import pytest

from paper_2006_04784_amd import inputs


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("N", [4, 8, 16])
def test_brute_force_dft2(orc, N):
    u = inputs.white_noise(N, seed=N)
    ref = orc.dft2_brute(u)
    assert rel(orc.r2c(u, method=0), ref) < 1e-13
    assert rel(orc.r2c(u, method=1), ref) < 1e-13


@pytest.mark.parametrize("n", [2, 8, 32, 64])
def test_fft_line_vs_naive_dft(orc, n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    for sign in (-1, 1):
        assert rel(orc.fft_1d(x, sign), orc.dft_1d(x, sign)) < 1e-13


def test_fft_rejects_non_power_of_two(orc):
    with pytest.raises(ValueError):
        orc.fft_1d(np.ones(12))


@pytest.mark.parametrize("N", [32, 64])
def test_fft2_vs_naive2(orc, N):
    u = inputs.white_noise(N, seed=1)
    assert rel(orc.r2c(u, 1), orc.r2c(u, 0)) < 1e-13
    uh = orc.r2c(u, 1)
    assert rel(orc.c2r(uh, 1), orc.c2r(uh, 0)) < 1e-13


@pytest.mark.parametrize("N", [16, 128, 256])
def test_numpy_crosscheck(orc, N):
    u = inputs.white_noise(N, seed=2)
    assert rel(orc.r2c(u), np.fft.rfft2(u)) < 1e-13
    uh = orc.r2c(u)
    # non-Hermitian input: inverse takes the real part of the inverse DFT of
    # the Hermitian extension, which is what numpy.irfft2 computes
    rng = np.random.default_rng(3)
    vh = uh + 0.1 * (rng.standard_normal(uh.shape) + 1j * rng.standard_normal(uh.shape))
    assert rel(orc.c2r(vh), np.fft.irfft2(vh, s=(N, N))) < 1e-13
    assert rel(orc.c2r(uh), u) < 1e-14


@pytest.mark.parametrize("N,L", [(32, 2 * np.pi), (64, 4 * np.pi)])
def test_spectral_laplacian_of_trig_modes(orc, N, L):
    X, Y = inputs.grid(N, L)
    m = orc.Model(N=N, L=L, eps=0.1, eta1=1.45, eta2=2.0)
    for (a, b) in [(1, 0), (0, 3), (2, 5), (N // 2 - 1, 1), (-3, 7)]:
        u = np.cos(2 * np.pi * a * X / L) * np.sin(2 * np.pi * b * Y / L)
        lap = orc.laplacian(m, u)
        exact = -(2 * np.pi / L) ** 2 * (a * a + b * b) * u
        assert np.max(np.abs(lap - exact)) <= 1e-13 * max(1.0, np.max(np.abs(exact)))


@pytest.mark.parametrize("N", [16, 64])
def test_parseval(orc, N):
    u = inputs.white_noise(N, seed=4)
    uh = orc.r2c(u)
    w = np.full(N // 2 + 1, 2.0)
    w[0] = 1.0
    w[-1] = 1.0
    lhs = np.sum(u * u)
    rhs = np.sum(w[None, :] * np.abs(uh) ** 2) / N ** 2
    assert abs(lhs - rhs) <= 1e-13 * lhs


def test_single_mode_inverse(orc):
    N = 16
    uh = np.zeros((N, N // 2 + 1), complex)
    uh[3, 2] = N * N / 2.0      # cos(2 pi (2 x + 3 y)/N) in index units
    u = orc.c2r(uh)
    i, j = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    assert np.max(np.abs(u - np.cos(2 * np.pi * (2 * j + 3 * i) / N))) < 1e-14
