"""Pins for the CPU oracle: each test checks it against something other than
itself (a dense matrix built from the operator definition, a closed form, an
invariant, a textbook special case, or numbers the paper prints)."""
import json
import os

import numpy as np
import pytest

from oracle import ipfb_oracle as O
from paper_2608_23441_amd import inputs as I

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def _rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b))


# --- P5: forward PFB against a direct triple loop ---------------------------
def test_forward_pfb_direct_loop():
    N, p, b = 8, 4, 5
    w = O.window_sinc_hamming(p, N)
    x = I.gaussian_timestream(N * b, 11)
    y = O.pfb_forward(x, w, N, p)
    ref = np.zeros((b, N // 2 + 1), dtype=complex)
    for j in range(b):
        for k in range(N // 2 + 1):
            acc = 0j
            for n in range(N):
                for r in range(p):
                    acc += np.exp(-2j * np.pi * n * k / N) * w[r * N + n] * x[((j + r) % b) * N + n]
            ref[j, k] = acc
    assert np.abs(y - ref).max() < 1e-12


def test_forward_pfb_dense_operator_linear_and_circular():
    N, p, b = 8, 3, 6
    w = O.window_sinc_hamming(p, N)
    x = I.gaussian_timestream(N * b, 12)
    for circ in (True, False):
        P = O.dense_pfb_matrix(w, N, p, b, circular=circ)
        y = O.pfb_forward(x, w, N, p, circular=circ)
        assert y.shape[0] == (b if circ else b - p + 1)
        assert np.abs(P @ x - y.reshape(-1)).max() < 1e-12


# --- P4: one segment equals every p-th bin of the M-point DFT ---------------
@pytest.mark.parametrize("N,p", [(16, 4), (64, 4), (32, 3)])
def test_segment_identity(N, p):
    w = O.window_sinc_hamming(p, N)
    x = I.gaussian_timestream(N * p, 13)
    y = O.pfb_forward(x, w, N, p, circular=False)
    assert y.shape[0] == 1
    long = np.fft.fft(x * w)  # M-point DFT of the windowed segment
    assert np.abs(y[0] - long[::p][: N // 2 + 1]).max() < 1e-12


# --- window ------------------------------------------------------------------
def test_window_formula_and_numpy_hamming():
    N, p = 64, 4
    w = O.window_sinc_hamming(p, N)
    M = N * p
    # numpy's Hamming is exactly the taper; sinc zero crossings every N samples
    ref = np.hamming(M) * np.sinc(np.arange(M) / N - p / 2)
    assert np.abs(w - ref).max() < 1e-15
    assert w[M // 2] == pytest.approx(np.hamming(M)[M // 2])
    for r in range(1, p):
        if r * N != M // 2:
            assert abs(w[r * N]) < 1e-15


# --- P3: Parseval on the row inverse ---------------------------------------
def test_row_inverse_parseval_and_roundtrip():
    N = 128
    y = I.complex_block((7, N // 2 + 1), 14)
    d = O.row_inverse(y, N)
    yz = y.copy()
    yz[:, 0] = yz[:, 0].real
    yz[:, -1] = yz[:, -1].real
    e_freq = (np.abs(yz[:, 0]) ** 2 + np.abs(yz[:, -1]) ** 2 + 2 * np.sum(np.abs(yz[:, 1:-1]) ** 2, axis=1)) / N
    e_time = np.sum(d ** 2, axis=1)
    assert np.abs(e_time - e_freq).max() / e_freq.max() < 1e-13
    # direct definition of the N-point inverse real DFT
    n = np.arange(N)
    k = np.arange(1, N // 2)
    for j in range(3):
        ref = (yz[j, 0].real + (-1.0) ** n * yz[j, -1].real
               + 2 * np.real(np.exp(2j * np.pi * np.outer(n, k) / N) @ yz[j, 1:-1])) / N
        assert np.abs(d[j] - ref).max() < 1e-13


# --- P1: exact recovery of a circular PFB without quantisation --------------
@pytest.mark.parametrize("N,p,b", [(16, 4, 8), (64, 4, 24), (2048, 4, 128), (32, 5, 9)])
def test_exact_recovery(N, p, b):
    w = O.window_sinc_hamming(p, N)
    x = I.gaussian_timestream(N * b, 15)
    y = O.pfb_forward(x, w, N, p)
    xr = O.ipfb_wiener_from_spectra(y, w, N, p, 0.0)
    assert _rel(xr, x) < 1e-11


# --- P2: the FFT decorrelation equals the dense Tikhonov / Wiener solve -----
@pytest.mark.parametrize("N,p,b,phi,norm", [(8, 4, 6, 0.1, True), (8, 4, 12, 0.3, True),
                                            (16, 3, 7, 0.1, False), (8, 4, 3, 0.2, True)])
def test_column_wiener_dense(N, p, b, phi, norm):
    w = O.window_sinc_hamming(p, N)
    d = I.uniform_block((b, N), 16)
    xf = O.column_inverse(d, w, N, p, phi, norm)
    H = w.reshape(p, N)
    for n in range(N):
        wn = np.zeros(b)
        for r in range(p):
            wn[r % b] += H[r, n]
        ref = O.dense_column_wiener(d[:, n], wn, phi, norm)
        assert np.abs(ref - xf[:, n]).max() < 1e-12


def test_column_spectra_direct_sum():
    N, p, b = 16, 4, 10
    w = O.window_sinc_hamming(p, N)
    W = O.column_spectra(w, N, p, b)
    f = np.arange(b)
    for n in (0, 5, N // 2):
        ref = sum(w[r * N + n] * np.exp(-2j * np.pi * r * f / b) for r in range(p))
        assert np.abs(W[:, n] - ref).max() < 1e-14


def test_wiener_gain_bound_and_limits():
    W = I.complex_block((1000,), 17) * np.logspace(-4, 1, 1000)
    for phi in (0.05, 0.1, 0.5):
        G = O.wiener_gain(W, phi)
        assert np.abs(G).max() <= (1 + phi ** 2) / (2 * phi) * (1 + 1e-14)
    G0 = O.wiener_gain(W, 0.0)
    assert np.abs(G0 * np.conj(W) - 1).max() < 1e-12
    # the (1+phi^2) normalisation keeps unit gain where W = 1 (Section 4.1)
    assert np.abs(O.wiener_gain(np.array([1.0 + 0j]), 0.1)[0] - 1.0) < 1e-15


# --- P6: Appendix A, a symmetric window has a zero eigenvalue ----------------
@pytest.mark.parametrize("p", [4, 5, 2, 3])
def test_symmetric_window_zero(p):
    N, b = 32, 16
    w = O.window_symmetric_hann(p, N)
    M = N * p
    assert w[0] == 0.0
    assert np.abs(w[1:] - w[1:][::-1]).max() < 1e-15
    W = O.column_spectra(w, N, p, b)
    path = N // 2 if p % 2 == 0 else 0
    assert abs(W[b // 2, path]) < 1e-14
    # the numpy Hamming window is only nearly symmetric: no exact zero
    assert np.abs(O.column_spectra(O.window_sinc_hamming(p, N), N, p, b)).min() > 1e-6


def test_appendix_a_worked_form():
    # w_{N/2} = [a, b, b, a, 0, ...] dotted with the Nyquist phasor vanishes
    for a, bb in [(1.0, 2.0), (0.3, -0.7)]:
        wn = np.array([a, bb, bb, a, 0, 0, 0, 0])
        assert abs(np.fft.fft(wn)[4]) < 1e-15


# --- P10: shift and linearity ------------------------------------------------
def test_frame_shift_and_linearity():
    N, p, b = 32, 4, 12
    w = O.window_sinc_hamming(p, N)
    x = I.gaussian_timestream(N * b, 18)
    y = O.pfb_forward(x, w, N, p)
    y_shift = O.pfb_forward(np.roll(x, -N), w, N, p)
    assert np.abs(y_shift - np.roll(y, -1, axis=0)).max() < 1e-12
    y2 = I.complex_block(y.shape, 19)
    a, c = 0.7, -1.3
    lhs = O.ipfb_wiener_from_spectra(a * y + c * y2, w, N, p, 0.1)
    rhs = a * O.ipfb_wiener_from_spectra(y, w, N, p, 0.1) + c * O.ipfb_wiener_from_spectra(y2, w, N, p, 0.1)
    assert np.abs(lhs - rhs).max() < 1e-12


# --- P8: adjoint -------------------------------------------------------------
def test_adjoint_dense_transpose_and_dot():
    N, p, b = 8, 4, 5
    w = O.window_sinc_hamming(p, N)
    P = O.dense_pfb_matrix(w, N, p, b)
    y = I.complex_block((b, N // 2 + 1), 20)
    xa = O.pfb_adjoint(y, w, N, p, b)
    ref = np.real(P.conj().T @ y.reshape(-1))
    assert np.abs(xa - ref).max() < 1e-12
    N, p, b = 256, 4, 33
    w = O.window_sinc_hamming(p, N)
    x = I.gaussian_timestream(N * b, 21)
    y = I.complex_block((b, N // 2 + 1), 22)
    lhs = np.real(np.vdot(y, O.pfb_forward(x, w, N, p)))
    rhs = np.dot(x, O.pfb_adjoint(y, w, N, p, b))
    assert abs(lhs - rhs) / abs(lhs) < 1e-12


def test_sw_adjoint_dense():
    N, p, b = 4, 3, 5
    w = O.window_sinc_hamming(p, N)
    S = N * b
    A = np.stack([O.sw_apply(np.eye(S)[c], w, N, p).reshape(-1) for c in range(S)], axis=1)
    d = I.uniform_block((b, N), 23)
    assert np.abs(O.sw_adjoint(d, w, N, p).reshape(-1) - A.T @ d.reshape(-1)).max() < 1e-13


# --- P7: Section 4.2.2 toy model ---------------------------------------------
def test_toy_model_one_saved_sample():
    N, p, b = 8, 4, 10
    w = O.window_symmetric_hann(p, N)
    x = I.gaussian_timestream(N * b, 24)
    y = O.pfb_forward(x, w, N, p)
    d = O.row_inverse(y, N)
    xpi = O.column_inverse(d, w, N, p, 0.0).reshape(b, N)  # truncated pseudo-inverse
    X = x.reshape(b, N)
    res = xpi - X
    # only path N/2 is wrong, and only along the alternating (Nyquist) mode
    others = np.delete(res, N // 2, axis=1)
    assert np.abs(others).max() < 1e-12
    r = res[:, N // 2]
    alt = (-1.0) ** np.arange(b)
    alpha = r[0]
    assert abs(alpha) > 1e-3
    assert np.abs(r - alpha * alt).max() < 1e-12
    # one saved sample on that path pins alpha: the ML solve recovers x exactly
    mask = np.zeros(b * N)
    mask[3 * N + N // 2] = 1.0
    xml = O.ml_dense_solve(d, w, N, p, mask, x, 1.0)
    assert np.abs(xml - x).max() < 1e-10
    # and PCG converges to the same answer
    x0 = O.column_inverse(d, w, N, p, 0.1).reshape(-1)
    xcg, norms = O.ml_pcg(d, w, N, p, mask, x, 1.0, 0.1, 60, x0)
    assert np.abs(xcg - x).max() < 1e-8
    assert norms[-1] < 1e-8 * norms[0]


# --- P12: PCG converges to the dense ML solve ---------------------------------
def test_pcg_matches_dense_solve():
    N, p, b = 8, 4, 12
    w = O.window_sinc_hamming(p, N)
    x = I.gaussian_timestream(N * b, 25)
    y = O.pfb_forward(x, w, N, p)
    s = O.channel_scales(y)
    qr, qi = O.quantize(y, s)
    d = O.row_inverse(O.dequantize(qr, qi, s), N)
    mask = I.random_mask(N * b, 0.1, 26)
    ref = O.ml_dense_solve(d, w, N, p, mask, x, 1.0)
    x0 = O.column_inverse(d, w, N, p, 0.1).reshape(-1)
    xcg, norms = O.ml_pcg(d, w, N, p, mask, x, 1.0, 0.1, 200, x0)
    assert _rel(xcg, ref) < 1e-9
    # the minimiser has a smaller objective than the Wiener start
    def chi2(v):
        return np.sum((d - O.sw_apply(v, w, N, p)) ** 2) + np.sum(mask * (v - x) ** 2)
    assert chi2(xcg) <= chi2(x0)


# --- quantiser ---------------------------------------------------------------
def test_pack_unpack_all_codes():
    qr, qi = np.meshgrid(np.arange(-7, 8), np.arange(-7, 8))
    qr = qr.astype(np.int8)
    qi = qi.astype(np.int8)
    a, b = O.unpack_c4(O.pack_c4(qr, qi))
    assert (a == qr).all() and (b == qi).all()
    # Re in the high nibble
    assert O.pack_c4(np.array([1], np.int8), np.array([-1], np.int8))[0] == 0x1F


def test_ci8_pack_unpack_all_codes_and_byte_order():
    qr, qi = np.meshgrid(np.arange(-128, 128), np.arange(-128, 128))
    qr = qr.astype(np.int8)
    qi = qi.astype(np.int8)
    a, b = O.unpack_ci8(O.pack_ci8(qr, qi))
    assert (a == qr).all() and (b == qi).all()
    # the real code first, two's complement bytes
    assert O.pack_ci8(np.array([1], np.int8), np.array([-1], np.int8)).view(np.uint8).tolist() == [[1, 255]]


def test_ci8_and_c4_reconstruct_identically_on_shared_codes():
    # codes within -7..7 fit both formats; the two unpackers must agree exactly
    N, p, b = 64, 4, 16
    w = O.window_sinc_hamming(p, N)
    y = O.pfb_forward(I.gaussian_timestream(N * b, 31), w, N, p)
    s = O.channel_scales(y)
    qr, qi = O.quantize(y, s)
    x4 = O.ipfb_wiener(O.pack_c4(qr, qi), s, w, N, p, 0.1)
    x8 = O.ipfb_wiener_ci8(O.pack_ci8(qr, qi), s, w, N, p, 0.1)
    assert np.array_equal(x4, x8)


def test_ci8_quantiser_error_far_below_c4():
    # with the quantiser step 16x finer, the reconstruction error against the
    # true timestream drops by about that factor (quantisation noise is the
    # only error of the exact inverse): a swapped or mis-signed unpack fails
    N, p, b = 128, 4, 64
    w = O.window_sinc_hamming(p, N)
    x = I.gaussian_timestream(N * b, 33)
    y = O.pfb_forward(x, w, N, p)
    s4 = O.channel_scales(y, levels_rms=2.5)
    s8 = O.channel_scales(y, levels_rms=40.0)
    e4 = _rel(O.ipfb_wiener(O.pack_c4(*O.quantize(y, s4)), s4, w, N, p, 0.0), x)
    e8 = _rel(O.ipfb_wiener_ci8(O.pack_ci8(*O.quantize(y, s8, qmax=127)), s8, w, N, p, 0.0), x)
    assert e8 < e4 / 8
    # the naive inverse amplifies the quantisation noise by mean 1/|W|^2
    # (Appendix B): about 2 % at 40 levels RMS
    assert e8 < 0.03


def test_quantizer_snr_matches_paper_spacing():
    lv = GOLD["quantizer_levels"]["value"]
    N, p, b = 256, 4, 512
    w = O.window_sinc_hamming(p, N)
    x = I.gaussian_timestream(N * b, 27)
    y = O.pfb_forward(x, w, N, p)
    s = O.channel_scales(y, levels_rms=1.0 / GOLD["quantizer_spacing_over_rms"]["value"])
    qr, qi = O.quantize(y, s)
    assert qr.min() >= lv[0] and qr.max() <= lv[1]
    yh = O.dequantize(qr, qi, s)
    inner = slice(1, -1)
    snr = np.sum(np.abs(y[:, inner]) ** 2) / np.sum(np.abs(y[:, inner] - yh[:, inner]) ** 2)
    lo, hi = GOLD["quantizer_snr"]["band"]
    assert lo < snr < hi


# --- P11: Section 4.3 / Appendix B statistics --------------------------------
@pytest.mark.slow
def test_autospectrum_error_statistics():
    N, p, b, u = 256, 4, 2048, 8
    w = O.window_sinc_hamming(p, N)
    x = I.gaussian_timestream(N * b, 28)
    y = O.pfb_forward(x, w, N, p)
    s = O.channel_scales(y, levels_rms=1.0 / 0.353)
    qr, qi = O.quantize(y, s)
    yh = O.dequantize(qr, qi, s)
    snr = np.sum(np.abs(y[:, 1:-1]) ** 2) / np.sum(np.abs(y[:, 1:-1] - yh[:, 1:-1]) ** 2)
    Nf = u * N
    wf = O.window_sinc_hamming(4, Nf)
    Yt = O.upchannelize(x, Nf, 4, wf)
    phi = 1.0 / np.sqrt(snr)
    xw = O.ipfb_wiener_from_spectra(yh, w, N, p, phi, normalise=False)
    dw = O.autospectrum_error(Yt, O.upchannelize(xw, Nf, 4, wf))
    xn = O.ipfb_wiener_from_spectra(yh, w, N, p, 0.0)
    dn = O.autospectrum_error(Yt, O.upchannelize(xn, Nf, 4, wf))
    k = np.arange(Nf // 2 + 1)
    res = k % u
    # centre of every coarse channel: 1/(1+SNR) (Appendix B), about 1.1% (Section 4.3)
    centre = dw[(res == 0) & (k > u) & (k < Nf // 2 - u)].mean()
    assert centre == pytest.approx(1.0 / (1.0 + snr), rel=0.25)
    lo, hi = GOLD["centre_delta"]["band"]
    assert lo < centre < hi
    # Wiener: the Monte-Carlo delta follows 1 - (1/N) sum_n H_n per residue
    # class, the closed form averaged over each fine channel's width
    K = 16
    ana = O.analytic_delta(w, N, p, u * K, phi=phi)
    for rr in range(u):
        sel = (res == rr) & (k > u) & (k < Nf // 2 - u)
        band = (rr * K + np.arange(-K // 2, K // 2)) % (u * K)
        assert dw[sel].mean() == pytest.approx(ana[band].mean(), rel=0.3)
    worst_wiener = max(dw[(res == rr) & (k > u)].mean() for rr in range(u))
    worst_naive = max(dn[(res == rr) & (k > u)].mean() for rr in range(u))
    assert worst_naive > 3.0 * worst_wiener
    # timestream error: most samples near the 4-bit amplitude floor (Section 4.3)
    e = (xw - x).reshape(b, N)
    per_path = np.sqrt(np.mean(e ** 2, axis=0))
    lo, hi = GOLD["timestream_error_most_samples"]["band"]
    assert lo < np.median(per_path) < hi


def test_analytic_delta_at_paper_configuration():
    # N = 2048, p = 4, sinc-Hamming, 4-bit (SNR ~ 80), phi = 0.1 (Section 4.3):
    # the closed forms of Appendix B give the printed worst cases
    N, p = 2048, 4
    w = O.window_sinc_hamming(p, N)
    snr = GOLD["quantizer_snr"]["value"]
    dw = O.analytic_delta(w, N, p, 512, phi=GOLD["wiener_phi_4bit"]["value"])
    dn = O.analytic_delta(w, N, p, 512, phi=None, snr=snr)
    lo, hi = GOLD["wiener_delta_max"]["band"]
    assert lo < dw.max() < hi
    assert dn.max() > GOLD["naive_delta_max"]["band_min"]
    # both peak at the channel edge (sub-stream Nyquist) and the centre is near 1/(1+SNR)
    assert int(np.argmax(dw)) == 256 and int(np.argmax(dn)) == 256
    assert dn[0] == pytest.approx(1.0 / snr, rel=0.05)


# --- P13: injected tones land in their fine channel ---------------------------
def test_tones_peak_in_expected_channel():
    N, b, u = 128, 1024, 16
    Nf = N * u
    f, th = I.tone_parameters(3, 102)
    x = I.add_tones(I.gaussian_timestream(N * b, 29), f, th, 1.0)
    wf = O.window_sinc_hamming(4, Nf)
    A = O.autospectrum(O.upchannelize(x, Nf, 4, wf))
    for fi in f:
        k = int(round(fi * Nf))
        lo, hi = k - 3, k + 4
        assert lo + int(np.argmax(A[lo:hi])) == k


# ---- linear boundary and streaming inverse ----------------------------------

def _dominant_window(N, p):
    # first tap dominant in every column: |W_n(f)| >= 1 - 0.37 > 0, so the
    # inverse kernel is causal and decays geometrically (ratio <= 0.37)
    n = np.arange(N)
    taps = [1.0 + 0.1 * np.cos(n), 0.15 + 0.05 * np.sin(n), -0.1 + 0 * n, 0.05 + 0.02 * np.cos(3 * n)]
    return np.concatenate(taps[:p])


@pytest.mark.parametrize("nspec,p,chunk,halo", [(300, 4, 64, 8), (20, 4, 64, 8), (61, 4, 64, 8),
                                                (1000, 3, 128, 0), (5, 4, 8, 1), (4097, 4, 256, 100)])
def test_stream_geometry_partitions_the_output(nspec, p, chunk, halo):
    ch = O.stream_chunks(nspec, p, chunk, halo)
    m, L = chunk - (p - 1), chunk - (p - 1) - 2 * halo
    nframes = nspec + p - 1
    k = 0
    for s0, nvalid, k0, off, nkeep in ch:
        assert k0 == k and 1 <= nkeep <= L
        assert 0 <= s0 and 1 <= nvalid <= m and s0 + nvalid <= nspec
        assert 0 <= off and off + nkeep <= chunk
        if s0 == k0 - halo and nvalid == m:  # interior window: halo on both sides
            assert off == halo and off + nkeep <= nvalid - halo
        k += nkeep
    assert k == nframes


def test_linear_inverse_exact_except_at_the_extended_end():
    # Section 3.1: the circulant model is exact for the wrapped rows only, so a
    # noise-free linear PFB is recovered exactly away from the zero-extended end
    N, p, nspec = 16, 4, 400
    w = _dominant_window(N, p)
    x = np.random.default_rng(11).standard_normal((nspec + p - 1) * N)
    y = O.pfb_forward(x, w, N, p, circular=False)
    err = np.abs(O.ipfb_linear_from_spectra(y, w, N, p, 0.0) - x).reshape(-1, N).max(axis=1)
    assert err[:-80].max() < 1e-12
    assert err[-3:].max() > 1e-3  # the end is corrupted, as the paper says


def test_stream_recovers_noise_free_timestream():
    # the end corruption decays by about 1.7x per frame for this window, so a
    # 64-frame halo keeps every window edge below 1e-12
    N, p, nspec, chunk = 16, 4, 1000, 256
    w = _dominant_window(N, p)
    x = np.random.default_rng(12).standard_normal((nspec + p - 1) * N)
    y = O.pfb_forward(x, w, N, p, circular=False)
    good = np.abs(O.ipfb_stream_from_spectra(y, w, N, p, 0.0, chunk, 64) - x).reshape(-1, N).max(axis=1)
    assert good[:-80].max() < 1e-12
    # a halo too small leaves window-edge corruption inside the stream
    bad = np.abs(O.ipfb_stream_from_spectra(y, w, N, p, 0.0, chunk, 1) - x).reshape(-1, N).max(axis=1)
    assert bad[:-80].max() > 1e-6


def test_stream_single_window_is_the_linear_inverse():
    N, p, chunk = 32, 4, 64
    w = O.window_sinc_hamming(p, N)
    nspec = chunk - (p - 1)
    x = np.random.default_rng(13).standard_normal((nspec + p - 1) * N)
    y = O.pfb_forward(x, w, N, p, circular=False)
    ref = O.ipfb_linear_from_spectra(y, w, N, p, 0.1)
    for halo in (0, 5, 20):
        assert np.abs(O.ipfb_stream_from_spectra(y, w, N, p, 0.1, chunk, halo) - ref).max() < 1e-13


def test_stream_converges_to_linear_inverse_as_halo_grows():
    # Wiener kernels decay (the decorrelation-kernel figure), so the window
    # boundaries stop mattering once the halo exceeds their width
    N, p, nspec = 16, 4, 1000
    w = O.window_sinc_hamming(p, N)
    x = np.random.default_rng(14).standard_normal((nspec + p - 1) * N)
    y = O.pfb_forward(x, w, N, p, circular=False)
    ref = O.ipfb_linear_from_spectra(y, w, N, p, 0.1).reshape(-1, N)
    diffs = []
    for halo in (8, 32, 64, 100):
        xs = O.ipfb_stream_from_spectra(y, w, N, p, 0.1, 256, halo).reshape(-1, N)
        diffs.append(np.abs(xs - ref)[200:-200].max())
    assert all(a > 10 * b for a, b in zip(diffs, diffs[1:]))
    assert diffs[-1] < 1e-5


# ---- structured prior mask (Section 4.2.2 sample saving, Section 4.3 results) -

def test_saved_paths_match_the_paper():
    g = GOLD["cg_saved_paths"]["value"]
    assert O.saved_paths(0.01, 4, 2048) == g["0.01"]
    assert O.saved_paths(0.10, 4, 2048) == g["0.10"]


@pytest.mark.parametrize("N,b,R,L", [(2048, 64, 4, 82), (64, 512, 4, 26), (64, 10, 4, 8), (32, 7, 3, 2)])
def test_structured_mask_layout(N, b, R, L):
    m = O.structured_mask(N, b, R, L).reshape(b, N)
    rows = np.arange(b) % R == 0
    assert m[~rows].sum() == 0
    assert int(m.sum()) == L * int(rows.sum())
    assert np.array_equal(m, m[:, ::-1])  # symmetric about the frame centre
    assert m[0, N // 2] == 1 and m[0, N // 2 - L // 2] == 1 and m[0, N // 2 + L // 2 - 1] == 1
    if b % R == 0:
        assert abs(m.mean() - L / (R * N)) < 1e-15  # beta = L / (R N)


def test_structured_prior_beats_wiener_at_the_worst_channel():
    # Section 4.3's trend at a small size: 25 CG iterations from the Wiener
    # solution with a structured prior cut the worst-case delta, roughly
    # halving it at 3 % saved and more at 10 %
    N, p, b, u = 64, 4, 512, 8
    w = O.window_sinc_hamming(p, N)
    x = I.gaussian_timestream(N * b, 21)
    y = O.pfb_forward(x, w, N, p)
    sc = O.channel_scales(y, 1 / GOLD["quantizer_spacing_over_rms"]["value"])
    qr, qi = O.quantize(y, sc)
    yq = O.dequantize(qr, qi, sc)
    xw = O.ipfb_wiener_from_spectra(yq, w, N, p, 0.1)
    wf = O.window_sinc_hamming(4, N * u)
    Yt = O.upchannelize(x, N * u, 4, wf)
    dw = O.autospectrum_error(Yt, O.upchannelize(xw, N * u, 4, wf)).max()
    d = O.row_inverse(yq, N)
    worst = {}
    for beta in (0.03, 0.10):
        m = O.structured_mask(N, b, 4, O.saved_paths(beta, 4, N))
        xm, _ = O.ml_pcg(d, w, N, p, m, x, 1.0, 0.1, 25, xw)
        worst[beta] = O.autospectrum_error(Yt, O.upchannelize(xm, N * u, 4, wf)).max()
    assert 0.04 < dw < 0.25  # the Wiener worst case, as at N = 2048
    assert worst[0.03] < 0.6 * dw
    assert worst[0.10] < 0.5 * dw and worst[0.10] < worst[0.03]


# ---- other eigenvalue filters (Section 4.1: arbitrary filtering of the eigenspectrum)

def test_threshold_filter_is_the_truncated_pseudo_inverse():
    # numpy's SVD-based pinv of the dense circulant with the same cut: the
    # circulant's singular values are |W_n(f)|
    N, p, b = 8, 4, 24
    w = O.window_sinc_hamming(p, N)
    d = np.random.default_rng(31).standard_normal((b, N))
    W = O.column_spectra(w, N, p, b)
    for n in range(N):
        tau = np.quantile(np.abs(W[:, n]), 0.3)  # drop about 30 % of the eigenvalues
        wn = w.reshape(p, N)[:, n]
        C = O.dense_circulant(wn, b)
        sv = np.linalg.svd(C, compute_uv=False)
        rc = (tau * (1 - 1e-9)) / sv.max()  # keep singular values >= tau
        ref = np.linalg.pinv(C, rcond=rc) @ d[:, n]
        got = O.column_inverse_filter(d, w, N, p, "threshold", tau * (1 - 1e-9))[:, n]
        assert np.abs(got - ref).max() < 1e-10 * max(1.0, np.abs(ref).max())


def test_psd_filter_is_a_dense_map_solve_and_reduces_to_wiener():
    N, p, b = 8, 4, 20
    w = O.window_sinc_hamming(p, N)
    d = np.random.default_rng(32).standard_normal((b, N))
    f = np.arange(b)
    nu = 0.01 + 0.2 * np.cos(np.pi * f / b) ** 2  # symmetric: nu(f) = nu(b - f)
    got = O.column_inverse_filter(d, w, N, p, "psd", nu=nu, normalise=False)
    # (C^T C + Nu) x = C^T d with Nu the circulant whose eigenvalues are nu
    Nu = np.real(np.fft.ifft(np.fft.fft(np.eye(b), axis=0) * nu[:, None], axis=0))
    for n in range(N):
        C = O.dense_circulant(w.reshape(p, N)[:, n], b)
        ref = np.linalg.solve(C.T @ C + Nu, C.T @ d[:, n])
        assert np.abs(got[:, n] - ref).max() < 1e-10
    const = O.column_inverse_filter(d, w, N, p, "psd", nu=np.full(b, 0.09))
    assert np.abs(const - O.column_inverse(d, w, N, p, 0.3)).max() < 1e-12


# --- the noise-to-signal filter at nu = 0 is the truncated naive inverse -------
@pytest.mark.parametrize("window", ["sinc_hamming", "symmetric_hann"])
def test_psd_filter_with_zero_nu_is_the_naive_inverse(window):
    # with nu = 0 the filter is H = 1, i.e. G = 1/conj(W) (Section 3.1), and an
    # exact zero eigenvalue (Appendix A's symmetric window, path N/2 at f = b/2)
    # is dropped as the naive inverse drops it, not divided by
    N, p, b = 16, 4, 8
    w = getattr(O, "window_" + window)(p, N)
    d = np.random.default_rng(33).standard_normal((b, N))
    got = O.column_inverse_filter(d, w, N, p, "psd", nu=np.zeros(b))
    ref = O.column_inverse(d, w, N, p, 0.0)
    assert np.all(np.isfinite(got))
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()
