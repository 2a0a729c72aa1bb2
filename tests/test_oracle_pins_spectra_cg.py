"""Pins for two oracle functions that the GPU parity tests rely on: the
autospectrum (Section 4.1, the autospectrum-error equation) and the ML-CG
preconditioner (Section 3.1 circulant eigenbasis, Section 4.2 normal
equations).

Each pin is a check function that takes an implementation. The real oracle
function must pass it; mutants with a plausible mistake planted on the CPU
(a sum for a mean, |Y| for |Y|^2, a dropped square, a transposed operand) must
fail it, which shows the pin is strong enough to catch them."""
import numpy as np
import pytest

from oracle import ipfb_oracle as O
from paper_2608_23441_amd import inputs as I


# --- autospectrum -------------------------------------------------------------
def _autospectrum_hand_case(fn):
    """Two spectra of three channels, averaged by hand:
    channel 0: |1+1j|^2 = 2 and |3|^2 = 9 -> 5.5;
    channel 1: |2|^2 = 4 and |2j|^2 = 4 -> 4;
    channel 2: |-1j|^2 = 1 and |1-2j|^2 = 5 -> 3."""
    Y = np.array([[1 + 1j, 2 + 0j, -1j], [3 + 0j, 2j, 1 - 2j]])
    A = np.asarray(fn(Y))
    return A.shape == (3,) and np.allclose(A, [5.5, 4.0, 3.0], rtol=0, atol=1e-15)


def _autospectrum_parseval(fn):
    """Parseval per fine frame, averaged over frames: with s'_j the polyphase
    sum that the fine FFT transforms (Y'_j = rfft(s'_j)),
    (1/b') sum_j sum_n s'_j[n]^2 = (1/N')(A(0) + A(N'/2) + 2 sum_{0<k<N'/2} A(k))."""
    Nf, p, bf = 64, 4, 6
    wf = O.window_sinc_hamming(p, Nf)
    x = I.gaussian_timestream(Nf * bf, 901)
    s = O.polyphase_sum(x, wf, Nf, p)
    Y = O.upchannelize(x, Nf, p, wf)
    A = np.asarray(fn(Y), dtype=np.float64)
    if A.shape != (Nf // 2 + 1,):
        return False
    lhs = np.sum(s * s) / bf
    rhs = (A[0] + A[-1] + 2.0 * np.sum(A[1:-1])) / Nf
    return abs(lhs - rhs) <= 1e-12 * lhs


def test_autospectrum_hand_case_and_parseval():
    assert _autospectrum_hand_case(O.autospectrum)
    assert _autospectrum_parseval(O.autospectrum)


@pytest.mark.parametrize("mutant", [
    lambda Y: np.sum(np.abs(Y) ** 2, axis=0),                 # sum instead of mean
    lambda Y: np.mean(np.abs(Y), axis=0),                     # |Y| instead of |Y|^2
    lambda Y: np.mean(Y.real ** 2, axis=0),                   # dropped imaginary part
    lambda Y: np.mean(np.abs(Y) ** 2, axis=1),                # averaged over channels
    lambda Y: np.abs(np.mean(Y, axis=0)) ** 2,                # power of the mean
])
def test_autospectrum_pins_reject_mutants(mutant):
    assert not (_autospectrum_hand_case(mutant) and _autospectrum_parseval(mutant))


# --- ML-CG preconditioner -----------------------------------------------------
def _precond_inverts_normal_operator(fn):
    """M^{-1} (A^T A + phi^2 I) r = r on random r, with A = S W applied by the
    direct polyphase sum and its transpose (no eigenvalues involved)."""
    N, p, b, phi = 8, 4, 12, 0.1
    w = O.window_sinc_hamming(p, N)
    r = I.uniform_block((b, N), 902)
    Hr = O.sw_adjoint(O.sw_apply(r, w, N, p), w, N, p) + phi * phi * r
    z = np.asarray(fn(Hr, w, N, p, phi))
    return z.shape == r.shape and np.abs(z - r).max() <= 1e-10 * np.abs(r).max()


def _precond_dense_inverse(fn):
    """Against the dense inverse of C_n^T C_n + phi^2 I per column, with C_n
    the circulant correlation of Section 3.1 built entry by entry."""
    N, p, b, phi = 4, 3, 7, 0.3
    w = O.window_sinc_hamming(p, N)
    r = I.uniform_block((b, N), 903)
    z = np.asarray(fn(r, w, N, p, phi))
    if z.shape != r.shape:
        return False
    for n in range(N):
        C = O.dense_circulant(w.reshape(p, N)[:, n], b)
        ref = np.linalg.inv(C.T @ C + phi * phi * np.eye(b)) @ r[:, n]
        if np.abs(z[:, n] - ref).max() > 1e-12 * np.abs(ref).max():
            return False
    return True


def test_preconditioner_inverts_the_normal_operator_and_matches_dense():
    assert _precond_inverts_normal_operator(O.ml_preconditioner)
    assert _precond_dense_inverse(O.ml_preconditioner)


def _mutant_precond(spectrum_term):
    def fn(r, window, lblock, ntap, phi):
        W = O.column_spectra(window, lblock, ntap, r.shape[0])
        return np.fft.ifft(np.fft.fft(r, axis=0) / spectrum_term(W, phi), axis=0).real
    return fn


@pytest.mark.parametrize("mutant", [
    _mutant_precond(lambda W, phi: np.abs(W) + phi * phi),        # |W| instead of |W|^2
    _mutant_precond(lambda W, phi: np.abs(W) ** 2 + phi),         # phi instead of phi^2
    _mutant_precond(lambda W, phi: np.abs(W) ** 2),               # regulariser dropped
    _mutant_precond(lambda W, phi: W * W + phi * phi),            # W^2 instead of |W|^2
    # the forward transform applied twice (no inverse)
    lambda r, w, N, p, phi: np.fft.fft(np.fft.fft(r, axis=0) / (np.abs(O.column_spectra(w, N, p, r.shape[0])) ** 2
                                                              + phi * phi), axis=0).real / r.shape[0],
    # transposed operand: the transforms taken along each frame instead of down each column
    lambda r, w, N, p, phi: np.fft.ifft(np.fft.fft(r, axis=1) / (np.abs(O.column_spectra(w, N, p, r.shape[0])) ** 2
                                                                + phi * phi), axis=1).real,
    # one scalar gain instead of the per-frequency one
    lambda r, w, N, p, phi: r / (np.abs(O.column_spectra(w, N, p, r.shape[0])) ** 2 + phi * phi).mean(),
])
def test_preconditioner_pins_reject_mutants(mutant):
    assert not (_precond_inverts_normal_operator(mutant) and _precond_dense_inverse(mutant))
