"""Pins for the oracle's alternative solvers (Appendix C): the banded-Cholesky
Tikhonov solve against a dense solve of the same normal equations and
against the circulant Wiener inverse away from the ends, and the truncated
FIR decorrelation against the exact circulant inverse."""
import numpy as np
import pytest

from oracle import ipfb_oracle as O
from paper_2608_23441_amd import inputs as I


@pytest.mark.parametrize("N,p,b,phi", [(8, 4, 20, 0.1), (4, 3, 9, 0.3), (4, 5, 12, 0.05), (2, 2, 6, 1.0)])
def test_tikhonov_equals_dense_normal_equations(N, p, b, phi):
    w = O.window_sinc_hamming(p, N)
    d = I.uniform_block((b - p + 1, N), 70 + N + p)
    got = O.tikhonov_banded(d, w, N, p, phi)
    H = w.reshape(p, N)
    for n in range(N):
        W = O.linear_subproblem(H[:, n], b)
        # the linear sub-problem matrix: Toeplitz rows, the taps of path n
        assert np.array_equal(W[0, :p], H[:, n]) and np.array_equal(W[-1, -p:], H[:, n])
        ref = (1 + phi * phi) * np.linalg.solve(W.T @ W + phi * phi * np.eye(b), W.T @ d[:, n])
        assert np.abs(got[:, n] - ref).max() < 1e-12 * np.abs(ref).max()


def test_tikhonov_equals_circulant_wiener_away_from_the_ends():
    # a noise-free linear PFB: the Tikhonov solution of the linear system and
    # the circulant Wiener inverse of the zero-extended data differ only near
    # the two ends (the boundary the circulant model gets wrong); in the
    # middle they agree once the decorrelation kernels have decayed
    N, p, b, phi = 16, 4, 400, 0.1
    w = O.window_sinc_hamming(p, N)
    x = I.gaussian_timestream(N * b, 71)
    y = O.pfb_forward(x, w, N, p, circular=False)
    d = O.row_inverse(y, N)
    tik = O.tikhonov_banded(d, w, N, p, phi)
    circ = O.ipfb_linear_from_spectra(y, w, N, p, phi).reshape(b, N)
    mid = slice(150, 250)
    assert np.abs(tik[mid] - circ[mid]).max() < 1e-9 * np.abs(circ[mid]).max()
    assert np.abs(tik[:3] - circ[:3]).max() > 1e-3  # the ends do differ


def test_fir_with_the_whole_kernel_is_the_circulant_inverse():
    # b - 1 lags (b even) cover every lag but one; the missing lag (c + b/2)
    # is added back by hand, which gives the circulant inverse exactly
    N, p, b, phi = 16, 4, 64, 0.1
    w = O.window_sinc_hamming(p, N)
    d = I.uniform_block((b, N), 72)
    c = p // 2
    g = O.fir_kernels(w, N, p, b, phi, b - 1)
    got = O.fir_apply(d, g, c)
    gall = O.fir_kernels(w, N, p, b, phi, b + 1)  # lags c - b/2 .. c + b/2
    got += gall[0][None, :] * d[(np.arange(b) - (c - b // 2)) % b]
    ref = O.column_inverse(d, w, N, p, phi)
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()


def test_fir_kernels_are_the_inverse_filters_impulse_response():
    # the truncation error shrinks geometrically with the kernel length (the
    # kernels decay away from their centre), reaching the paper's regime at
    # about 50 taps (4 taps, phi = 0.1: a few per cent at the worst path)
    N, p, b, phi = 32, 4, 1024, 0.1
    w = O.window_sinc_hamming(p, N)
    d = I.uniform_block((b, N), 73)
    ref = O.column_inverse(d, w, N, p, phi)
    errs = [np.abs(O.fir_apply(d, O.fir_kernels(w, N, p, b, phi, L), p // 2) - ref).max() / np.abs(ref).max()
            for L in (11, 31, 51, 101, 151)]
    assert all(errs[i + 1] < 0.5 * errs[i] for i in range(4))
    assert errs[2] < 0.05 and errs[-1] < 1e-4
    # path 0 of the sinc-Hamming window is a pure delay of 2 frames (its other
    # taps sit on sinc zeros): its kernel is (1+phi^2) h / (h^2 + phi^2) at
    # lag 2 (the centre, index T) and rounding-level elsewhere
    g = O.fir_kernels(w, N, p, b, phi, 7)
    h = w.reshape(p, N)[2, 0]
    assert abs(g[3, 0] - (1 + phi ** 2) * h / (h * h + phi ** 2)) < 1e-12
    assert np.abs(np.delete(g[:, 0], 3)).max() < 1e-12
