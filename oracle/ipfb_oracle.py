"""CPU FP64 oracle for the circulant inverse PFB and up-channelization.

TEST INFRASTRUCTURE ONLY. This module is the plain, slow, obviously correct
reference that the HIP library is checked against. Only the test suite, the
package smoke check and the CPU-baseline leg of the benchmark may import it.
The library never calls it, and it shares no code with the library: it uses
numpy (float64 / complex128) and nothing from the HIP side.

Every function follows a passage of the paper (Fay et al., "Inverting and
Up-channelizing Critically-Sampled Polyphase Filter Banks"); the passage is
named in its docstring. numpy.fft and numpy.linalg serve as library steps.
Readings taken where the paper is silent or garbled are marked READING.

Notation: N = lblock (real samples per frame, FFT length), p = ntap, M = pN
the window length, b = nblock (frames in the timestream), n = column (sub-filter
path) index, j = frame index. A timestream x is stored frame-major: x[j*N + n].
Spectra are [nspec][N/2+1] complex.
"""
from __future__ import annotations

import numpy as np

# ----------------------------------------------------------------------------
# Window (Section 2.2: truncated sinc times a taper; Appendix A: numpy's
# Hamming normalisation cos(2 pi m/(M-1))).
# ----------------------------------------------------------------------------


def window_sinc_hamming(ntap: int, lblock: int) -> np.ndarray:
    """h[m] = sinc((m - M/2)/N) * (0.54 - 0.46 cos(2 pi m/(M-1))), m = 0..M-1.

    READING: the sinc argument is scaled by 1/N so that its main lobe spans one
    channel (the paper writes sinc[m - M/2] with the scale implied by its
    substitution t_m = m/2B); the window is not normalised.
    """
    M = ntap * lblock
    m = np.arange(M, dtype=np.float64)
    sinc = np.sinc((m - M / 2.0) / lblock)
    taper = 0.54 - 0.46 * np.cos(2.0 * np.pi * m / (M - 1))
    return sinc * taper


def window_symmetric_hann(ntap: int, lblock: int) -> np.ndarray:
    """An exactly symmetric window with h[0] = 0 and h[m] = h[M-m] (Appendix A's
    two requirements): sinc((m - M/2)/N) times the periodic Hann taper
    0.5 - 0.5 cos(2 pi m/M)."""
    M = ntap * lblock
    m = np.arange(M, dtype=np.float64)
    return np.sinc((m - M / 2.0) / lblock) * (0.5 - 0.5 * np.cos(2.0 * np.pi * m / M))


# ----------------------------------------------------------------------------
# Forward PFB (Section 2.2, the polyphase equation; Section 2.3, y = F S W x and
# the sliding window over the [frames, N] data array).
# ----------------------------------------------------------------------------


def polyphase_sum(x: np.ndarray, window: np.ndarray, lblock: int, ntap: int,
                  circular: bool = True) -> np.ndarray:
    """s_j[n] = sum_{r<p} h[rN+n] x[(j+r)N + n]  (the W then S step).

    Spectrum j uses frames j..j+p-1 (Section 2.2: the next spectrum starts one
    frame later). circular=True wraps frame indices modulo b, so nspec = b
    (the circulant model of Section 3.1); otherwise nspec = b - p + 1.
    """
    N, p = lblock, ntap
    X = np.asarray(x, dtype=np.float64).reshape(-1, N)
    b = X.shape[0]
    H = np.asarray(window, dtype=np.float64).reshape(p, N)
    nspec = b if circular else b - p + 1
    if nspec <= 0:
        raise ValueError("need at least ntap frames for the linear PFB")
    s = np.zeros((nspec, N), dtype=np.float64)
    j = np.arange(nspec)
    for r in range(p):
        rows = (j + r) % b
        s += H[r][None, :] * X[rows]
    return s


def pfb_forward(x: np.ndarray, window: np.ndarray, lblock: int, ntap: int,
                circular: bool = True) -> np.ndarray:
    """y_j[k] = sum_n e^{-2 pi i n k/N} s_j[n], k = 0..N/2 (the F step)."""
    s = polyphase_sum(x, window, lblock, ntap, circular)
    return np.fft.rfft(s, axis=1)


# ----------------------------------------------------------------------------
# 4-bit quantiser (Section 3.2 additive noise model; Section 4.3: 15-level
# mid-tread quantiser, levels -7..7, applied to Re and Im of each channel).
# ----------------------------------------------------------------------------


def channel_scales(y: np.ndarray, levels_rms: float = 2.5) -> np.ndarray:
    """s_k = float32(levels_rms / sigma_k), sigma_k = sqrt(mean_j |y_jk|^2 / 2).

    READING: the scale is set per channel from the RMS of one real component
    (Section 4.3 sets the level spacing from the RMS of the channelised
    spectra); levels_rms = 1/0.353 reproduces the paper's spacing. A channel
    with zero power gets scale 1.
    """
    p2 = np.mean(np.abs(y) ** 2, axis=0) / 2.0
    sig = np.sqrt(p2)
    s = np.where(sig > 0, levels_rms / np.where(sig > 0, sig, 1.0), 1.0)
    return s.astype(np.float32)


def quantize(y: np.ndarray, scales_f32: np.ndarray, qmax: int = 7):
    """q = clip(rint(s_k Re y), -7, 7) + i clip(rint(s_k Im y), -7, 7), int8 each.

    The product is formed in float64 from the float32 scale. rint rounds half
    to even.
    """
    s = np.asarray(scales_f32, dtype=np.float32).astype(np.float64)[None, :]
    qr = np.clip(np.rint(s * y.real), -qmax, qmax).astype(np.int8)
    qi = np.clip(np.rint(s * y.imag), -qmax, qmax).astype(np.int8)
    return qr, qi


def pack_c4(qr: np.ndarray, qi: np.ndarray) -> np.ndarray:
    """One byte per complex value: Re in the high nibble, Im in the low nibble,
    both 4-bit two's complement (READING: the paper does not fix a layout)."""
    return (((qr.astype(np.int16) & 0xF) << 4) | (qi.astype(np.int16) & 0xF)).astype(np.uint8)


def unpack_c4(packed: np.ndarray):
    """Inverse of pack_c4: sign-extend each nibble."""
    p = packed.astype(np.int16)
    hi = (p >> 4) & 0xF
    lo = p & 0xF
    hi = np.where(hi >= 8, hi - 16, hi)
    lo = np.where(lo >= 8, lo - 16, lo)
    return hi.astype(np.int8), lo.astype(np.int8)


def pack_ci8(qr: np.ndarray, qi: np.ndarray) -> np.ndarray:
    """Two bytes per complex value, the real then the imaginary code, each an
    8-bit two's complement integer: [..., 2] int8 (READING: the paper
    quantises to 4 bits only; this is the finer format of the interface)."""
    return np.stack([qr.astype(np.int8), qi.astype(np.int8)], axis=-1)


def unpack_ci8(packed: np.ndarray):
    """Inverse of pack_ci8."""
    return packed[..., 0].astype(np.int8), packed[..., 1].astype(np.int8)


def dequantize(qr: np.ndarray, qi: np.ndarray, scales_f32: np.ndarray) -> np.ndarray:
    """yhat = q / s_k with s_k read back from its float32 value."""
    s = np.asarray(scales_f32, dtype=np.float32).astype(np.float64)[None, :]
    return (qr.astype(np.float64) + 1j * qi.astype(np.float64)) / s


# ----------------------------------------------------------------------------
# Inverse PFB (Section 3: undo F with an N-point inverse FFT per spectrum, then
# decorrelate each column with a b-point circulant inverse; Section 4.1 Wiener).
# ----------------------------------------------------------------------------


def row_inverse(yhat: np.ndarray, lblock: int) -> np.ndarray:
    """d_j = N-point inverse real FFT of spectrum j (undoes F, Section 3).

    d_j[n] = (1/N)[Re y_0 + (-1)^n Re y_{N/2} + 2 Re sum_{k=1}^{N/2-1} y_k e^{2 pi i n k/N}];
    the imaginary parts of the DC and Nyquist bins carry no information for a
    real frame and are dropped.
    """
    y = np.array(yhat, dtype=np.complex128, copy=True)
    y[:, 0] = y[:, 0].real
    y[:, -1] = y[:, -1].real
    return np.fft.irfft(y, n=lblock, axis=1)


def column_kernels(window: np.ndarray, lblock: int, ntap: int, nblock: int) -> np.ndarray:
    """w_n zero-padded to b frames: K[j, n] = sum_{r<p, r = j mod b} h[rN + n].

    Row r of the reshaped [p, N] window is the r-th tap of every column
    (Section 2.3); for b < p the taps wrap around the circulant."""
    H = np.asarray(window, dtype=np.float64).reshape(ntap, lblock)
    K = np.zeros((nblock, lblock), dtype=np.float64)
    for r in range(ntap):
        K[r % nblock] += H[r]
    return K


def column_spectra(window: np.ndarray, lblock: int, ntap: int, nblock: int) -> np.ndarray:
    """W_n(f) = F w_n: b-point DFT of each zero-padded column kernel,
    [b, N] complex (Section 3.1, the eigenvalues of W_n^circ)."""
    return np.fft.fft(column_kernels(window, lblock, ntap, nblock), axis=0)


def wiener_gain(W: np.ndarray, phi: float, normalise: bool = True,
                trunc: float = 1e-12, tapsum: np.ndarray | None = None) -> np.ndarray:
    """Gain G applied to F d_n so that xhat_n = F^dagger[G F d_n].

    G = H / conj(W) with the Wiener weights of Section 4.1,
    H = |W|^2 (1 + phi^2) / (|W|^2 + phi^2), i.e. G = W (1+phi^2)/(|W|^2+phi^2).
    normalise=False drops the (1+phi^2) factor (Appendix B calls it optional).
    phi = 0 is the plain division of Section 3.1; eigenvalues at rounding level,
    |W| <= trunc * sum_r |h[rN+n]| (tapsum, per column; the largest |W| a column
    can reach), are set to zero (READING: the pseudo-inverse truncation that
    Section 4.2.2 uses for the toy model).
    """
    W = np.asarray(W, dtype=np.complex128)
    a2 = np.abs(W) ** 2
    if phi == 0.0:
        bound = np.abs(W).max() if tapsum is None else np.broadcast_to(tapsum, W.shape)
        ok = np.abs(W) > trunc * bound
        G = np.zeros_like(W)
        G[ok] = 1.0 / np.conj(W[ok])
        return G
    c = (1.0 + phi * phi) if normalise else 1.0
    return W * c / (a2 + phi * phi)


def column_inverse(d: np.ndarray, window: np.ndarray, lblock: int, ntap: int,
                   phi: float, normalise: bool = True) -> np.ndarray:
    """xhat_n = F^dagger[ G_n . F d_n ] for every column n (Section 3.1's
    decorrelation equation with the Wiener weights of Section 4.1).
    d is [b, N]; the DFT runs down each column (over the frame index)."""
    d = np.asarray(d, dtype=np.float64)
    b = d.shape[0]
    W = column_spectra(window, lblock, ntap, b)
    tapsum = np.sum(np.abs(np.asarray(window, dtype=np.float64).reshape(ntap, lblock)), axis=0)
    G = wiener_gain(W, phi, normalise, tapsum=tapsum[None, :])
    D = np.fft.fft(d, axis=0)
    return np.fft.ifft(G * D, axis=0).real


def filter_gain(W: np.ndarray, kind: str, param: float = 0.0, nu: np.ndarray | None = None,
                normalise: bool = True, tapsum: np.ndarray | None = None) -> np.ndarray:
    """Other eigenvalue filters (Section 4.1: the circulant form gives the
    eigenspectrum W_n(f), so any filter H_n(f) applies as G = H / conj(W)).

    kind "threshold": H = 1 where |W| >= param, else 0 (the truncated
    pseudo-inverse; eigenvalues below the threshold are dropped).
    kind "psd": the general Wiener filter S/(S+N) with a noise-to-signal ratio
    per frequency, nu[f] = N(f)/S(f) (an array of length b, read as
    nu[min(f, b - f)]), H = |W|^2 (1 + nu) / (|W|^2 + nu), the (1 + nu) factor
    dropped with normalise=False; a constant nu = phi^2 is the Wiener filter.
    READING (as the naive inverse's truncation, Section 4.2.2): where
    |W|^2 + nu <= (1e-12 tapsum)^2, e.g. nu = 0 at an exact zero of W, G = 0.
    W: [b, N]; tapsum: [N] sum_r |h[rN+n]| (default max |W|); returns G [b, N].
    """
    W = np.asarray(W, dtype=np.complex128)
    b = W.shape[0]
    a2 = np.abs(W) ** 2
    if kind == "threshold":
        keep = np.abs(W) >= param
        G = np.zeros_like(W)
        G[keep] = 1.0 / np.conj(W[keep])
        return G
    if kind == "psd":
        f = np.arange(b)
        v = np.asarray(nu, dtype=np.float64)[np.minimum(f, b - f) % b][:, None]
        c = (1.0 + v) if normalise else 1.0
        den = a2 + v
        bound = np.abs(W).max() if tapsum is None else np.broadcast_to(tapsum, W.shape)
        ok = den > (1e-12 * bound) ** 2
        G = np.zeros_like(W)
        G[ok] = (W * c)[ok] / den[ok]
        return G
    raise ValueError(kind)


def column_inverse_filter(d: np.ndarray, window: np.ndarray, lblock: int, ntap: int, kind: str,
                          param: float = 0.0, nu: np.ndarray | None = None,
                          normalise: bool = True) -> np.ndarray:
    """xhat_n = F^dagger[ G_n . F d_n ] with a filter_gain eigenvalue filter."""
    d = np.asarray(d, dtype=np.float64)
    W = column_spectra(window, lblock, ntap, d.shape[0])
    tapsum = np.sum(np.abs(np.asarray(window, dtype=np.float64).reshape(ntap, lblock)), axis=0)
    G = filter_gain(W, kind, param, nu, normalise, tapsum=tapsum[None, :])
    return np.fft.ifft(G * np.fft.fft(d, axis=0), axis=0).real


def ipfb_wiener_from_spectra(yhat: np.ndarray, window: np.ndarray, lblock: int,
                             ntap: int, phi: float, normalise: bool = True) -> np.ndarray:
    """Full circulant inverse of (dequantised) spectra; returns x[j*N+n] float64."""
    d = row_inverse(yhat, lblock)
    return column_inverse(d, window, lblock, ntap, phi, normalise).reshape(-1)


def ipfb_wiener(packed: np.ndarray, scales_f32: np.ndarray, window: np.ndarray,
                lblock: int, ntap: int, phi: float, normalise: bool = True) -> np.ndarray:
    """Dequantise packed 4-bit spectra, then invert (steps a1..a5)."""
    qr, qi = unpack_c4(packed)
    return ipfb_wiener_from_spectra(dequantize(qr, qi, scales_f32), window, lblock,
                                    ntap, phi, normalise)


def ipfb_wiener_ci8(packed: np.ndarray, scales_f32: np.ndarray, window: np.ndarray,
                    lblock: int, ntap: int, phi: float, normalise: bool = True) -> np.ndarray:
    """Dequantise 8-bit spectra ([nspec][N/2+1][2] int8), then invert (a1..a5)."""
    qr, qi = unpack_ci8(packed)
    return ipfb_wiener_from_spectra(dequantize(qr, qi, scales_f32), window, lblock,
                                    ntap, phi, normalise)


# ----------------------------------------------------------------------------
# Linear boundary and streaming inversion (Section 3.1: real data are not
# circulant; the data are extended to b frames and the circulant inverse
# corrupts only samples within a decorrelation-kernel width of the ends, the
# kernel widths shown with the decorrelation-kernel figure).
# ----------------------------------------------------------------------------


def ipfb_linear_from_spectra(yhat: np.ndarray, window: np.ndarray, lblock: int, ntap: int,
                             phi: float, normalise: bool = True) -> np.ndarray:
    """Inverse of nspec spectra of a linear (non-wrapping) PFB over
    b = nspec + p - 1 frames: d_j from the row inverse for j < nspec, the p - 1
    appended rows set to zero (READING: the extension of d_n to b frames is a
    zero extension), then the circulant inverse over b frames. Returns
    x[j*N + n] for the b frames."""
    d = row_inverse(yhat, lblock)
    nspec = d.shape[0]
    dpad = np.zeros((nspec + ntap - 1, lblock), dtype=np.float64)
    dpad[:nspec] = d
    return column_inverse(dpad, window, lblock, ntap, phi, normalise).reshape(-1)


def stream_chunks(nspec: int, ntap: int, chunk: int, halo: int):
    """Chunk geometry of the streaming (overlap-save) inverse.

    READING (the paper announces a streaming inverse without details): a stream
    of nspec spectra covers nframes = nspec + p - 1 frames. Each window holds
    m = chunk - (p - 1) consecutive spectra, zero-extended to chunk frames, and
    is inverted on its own; a window keeps L = m - 2*halo frames, those at least
    halo frames from its first frame and from its last spectrum. Window c keeps
    output frames [c L, min((c+1) L, nframes)); it starts at spectrum
    s0 = max(0, min(c L - halo, nspec - m)) (the stream's ends pull it inwards)
    and holds min(m, nspec - s0) spectra. Returns a list of
    (s0, nvalid, k0, offset, nkeep): window frames [offset, offset + nkeep)
    become output frames [k0, k0 + nkeep).
    """
    m = chunk - (ntap - 1)
    L = m - 2 * halo
    if nspec < 1 or m < 1 or L < 1:
        raise ValueError("need nspec >= 1 and chunk - (ntap - 1) - 2*halo >= 1")
    nframes = nspec + ntap - 1
    out = []
    k0 = 0
    while k0 < nframes:
        s0 = max(0, min(k0 - halo, nspec - m))
        nvalid = min(m, nspec - s0)
        nkeep = min(L, nframes - k0)
        out.append((s0, nvalid, k0, k0 - s0, nkeep))
        k0 += L
    return out


def ipfb_stream_from_spectra(yhat: np.ndarray, window: np.ndarray, lblock: int, ntap: int,
                             phi: float, chunk: int, halo: int, normalise: bool = True) -> np.ndarray:
    """Streaming inverse: every window of stream_chunks inverted as in
    ipfb_linear_from_spectra but over `chunk` frames, the kept frames
    assembled. Returns x[j*N + n] for nspec + p - 1 frames."""
    y = np.asarray(yhat)
    nspec = y.shape[0]
    x = np.zeros((nspec + ntap - 1, lblock), dtype=np.float64)
    for s0, nvalid, k0, off, nkeep in stream_chunks(nspec, ntap, chunk, halo):
        d = np.zeros((chunk, lblock), dtype=np.float64)
        d[:nvalid] = row_inverse(y[s0:s0 + nvalid], lblock)
        xw = column_inverse(d, window, lblock, ntap, phi, normalise)
        x[k0:k0 + nkeep] = xw[off:off + nkeep]
    return x.reshape(-1)


def ipfb_stream(packed: np.ndarray, scales_f32: np.ndarray, window: np.ndarray, lblock: int,
                ntap: int, phi: float, chunk: int, halo: int, normalise: bool = True) -> np.ndarray:
    """Dequantise packed 4-bit spectra of a linear PFB, then the streaming inverse."""
    qr, qi = unpack_c4(packed)
    return ipfb_stream_from_spectra(dequantize(qr, qi, scales_f32), window, lblock, ntap, phi,
                                    chunk, halo, normalise)


# ----------------------------------------------------------------------------
# Dense references for tiny sizes (Section 3.1 circulant matrix; Appendix C's
# Tikhonov-regularised pseudo-inverse).
# ----------------------------------------------------------------------------


def dense_circulant(wn: np.ndarray, nblock: int) -> np.ndarray:
    """(C x)[j] = sum_r w_n[r] x[(j + r) mod b]: the circulant correlation
    matrix W_n^circ of Section 3.1 built entry by entry."""
    C = np.zeros((nblock, nblock))
    for j in range(nblock):
        for r, wr in enumerate(wn):
            C[j, (j + r) % nblock] += wr
    return C


def dense_pfb_matrix(window: np.ndarray, lblock: int, ntap: int, nblock: int,
                     circular: bool = True) -> np.ndarray:
    """The full real-to-complex PFB as a dense [nspec*(N/2+1), b*N] complex
    matrix, from y = F S W x applied to successive segments shifted one frame
    (Section 2.3), with F_{n,k} = exp(-2 pi i n k / N)."""
    N, p, b = lblock, ntap, nblock
    nspec = b if circular else b - p + 1
    K = N // 2 + 1
    P = np.zeros((nspec * K, b * N), dtype=np.complex128)
    for j in range(nspec):
        for k in range(K):
            row = j * K + k
            for n in range(N):
                ph = np.exp(-2j * np.pi * n * k / N)
                for r in range(p):
                    col = ((j + r) % b) * N + n
                    P[row, col] += ph * window[r * N + n]
    return P


def dense_column_wiener(d_col: np.ndarray, wn: np.ndarray, phi: float,
                        normalise: bool = True) -> np.ndarray:
    """(1+phi^2) (C^T C + phi^2 I)^{-1} C^T d for one column: the Tikhonov form
    that Appendix C equates with the Wiener machinery."""
    b = d_col.shape[0]
    C = dense_circulant(wn, b)
    c = (1.0 + phi * phi) if normalise else 1.0
    return c * np.linalg.solve(C.T @ C + phi * phi * np.eye(b), C.T @ d_col)


# ----------------------------------------------------------------------------
# Up-channelization and the autospectrum error (Section 4.1's error metric,
# Section 4.3: re-channelise the inverse with a longer frame).
# ----------------------------------------------------------------------------


def upchannelize(x: np.ndarray, lblock_fine: int, ntap_fine: int,
                 window_fine: np.ndarray) -> np.ndarray:
    """Forward PFB at the fine frame length N' (circular over b' = S/N')."""
    return pfb_forward(x, window_fine, lblock_fine, ntap_fine, circular=True)


def autospectrum(Y: np.ndarray) -> np.ndarray:
    """A(f) = (1/b') sum_j |Y_j(f)|^2."""
    return np.mean(np.abs(Y) ** 2, axis=0)


def autospectrum_error(Y_true: np.ndarray, Y_hat: np.ndarray) -> np.ndarray:
    """delta(f) = <|X - Xhat|^2> / <|X|^2>, averages over spectra (Section 4.1)."""
    return np.sum(np.abs(Y_true - Y_hat) ** 2, axis=0) / np.sum(np.abs(Y_true) ** 2, axis=0)


# ----------------------------------------------------------------------------
# Adjoint of the forward PFB (needed for the maximum-likelihood form, Section
# 4.2, and for differentiation). Inner products: real dot on x; Re<.,.> on the
# half spectrum.
# ----------------------------------------------------------------------------


def pfb_adjoint(y: np.ndarray, window: np.ndarray, lblock: int, ntap: int,
                nblock: int) -> np.ndarray:
    """(F S W)^T y for the circular PFB.

    z_j[n] = Re sum_{k=0}^{N/2} y_jk e^{2 pi i n k/N} (the transpose of the
    half-spectrum DFT), then x[iN+n] = sum_r h[rN+n] z_{(i-r) mod b}[n]
    (the transpose of the sliding multiply-and-sum)."""
    N, p, b = lblock, ntap, nblock
    y = np.asarray(y, dtype=np.complex128)
    c = np.ones(N // 2 + 1)
    c[0] = 2.0
    c[-1] = 2.0
    z = (N / 2.0) * np.fft.irfft(y * c[None, :], n=N, axis=1)
    H = np.asarray(window, dtype=np.float64).reshape(p, N)
    x = np.zeros((b, N))
    i = np.arange(b)
    for r in range(p):
        x += H[r][None, :] * z[(i - r) % b]
    return x.reshape(-1)


# ----------------------------------------------------------------------------
# Maximum-likelihood reconstruction with a time-domain prior (Section 4.2):
# minimise |d - A x|^2 + lam |D (x - prior)|^2 with A = S W (circular) acting
# after the N-point inverse FFT, D = diag(mask). Solved by preconditioned CG.
# ----------------------------------------------------------------------------


def sw_apply(x: np.ndarray, window: np.ndarray, lblock: int, ntap: int) -> np.ndarray:
    """A x = S W x (circular), returns [b, N]."""
    return polyphase_sum(x, window, lblock, ntap, circular=True)


def sw_adjoint(d: np.ndarray, window: np.ndarray, lblock: int, ntap: int) -> np.ndarray:
    """A^T d: x[iN+n] = sum_r h[rN+n] d[(i-r) mod b][n]; returns [b, N]."""
    N, p = lblock, ntap
    d = np.asarray(d, dtype=np.float64).reshape(-1, N)
    b = d.shape[0]
    H = np.asarray(window, dtype=np.float64).reshape(p, N)
    x = np.zeros_like(d)
    i = np.arange(b)
    for r in range(p):
        x += H[r][None, :] * d[(i - r) % b]
    return x


def ml_normal_apply(x, window, lblock, ntap, mask2d, lam):
    """(A^T A + lam D) x."""
    return sw_adjoint(sw_apply(x, window, lblock, ntap), window, lblock, ntap) + lam * mask2d * x


def ml_preconditioner(r, window, lblock, ntap, phi, W=None):
    """M^{-1} r = F^dagger[ F r_n / (|W_n|^2 + phi^2) ] per column: the inverse of
    A^T A + phi^2 I, which is diagonal in the Fourier basis (Section 3.1).
    W: column_spectra(window, lblock, ntap, b) if the caller already holds it."""
    b = r.shape[0]
    if W is None:
        W = column_spectra(window, lblock, ntap, b)
    return np.fft.ifft(np.fft.fft(r, axis=0) / (np.abs(W) ** 2 + phi * phi), axis=0).real


def ml_pcg(d: np.ndarray, window: np.ndarray, lblock: int, ntap: int,
           mask: np.ndarray, prior: np.ndarray, lam: float, phi_precond: float,
           iters: int, x0: np.ndarray):
    """Preconditioned conjugate gradient (the CG method the paper cites,
    Shewchuk 1994) on (A^T A + lam D) x = A^T d + lam D prior.

    Runs exactly `iters` iterations from x0 (the Wiener solution in the paper's
    experiments) and returns (x, residual 2-norms for k = 0..iters).
    READING: N^{-1} = I, lam = 1 by default at the call site, mask random.
    """
    N = lblock
    d = np.asarray(d, dtype=np.float64).reshape(-1, N)
    m2 = np.asarray(mask, dtype=np.float64).reshape(-1, N)
    pr = np.asarray(prior, dtype=np.float64).reshape(-1, N)
    x = np.array(x0, dtype=np.float64).reshape(-1, N)
    rhs = sw_adjoint(d, window, lblock, ntap) + lam * m2 * pr
    r = rhs - ml_normal_apply(x, window, lblock, ntap, m2, lam)
    W = column_spectra(window, lblock, ntap, d.shape[0])  # the same in every iteration
    z = ml_preconditioner(r, window, lblock, ntap, phi_precond, W)
    pdir = z.copy()
    rho = float(np.sum(r * z))
    norms = [float(np.sqrt(np.sum(r * r)))]
    for _ in range(iters):
        q = ml_normal_apply(pdir, window, lblock, ntap, m2, lam)
        pq = float(np.sum(pdir * q))
        # an exactly converged system (p.q = 0 or rho = 0) stops moving
        alpha = rho / pq if pq != 0.0 else 0.0
        x = x + alpha * pdir
        r = r - alpha * q
        z = ml_preconditioner(r, window, lblock, ntap, phi_precond, W)
        rho_new = float(np.sum(r * z))
        beta = rho_new / rho if rho != 0.0 else 0.0
        rho = rho_new
        pdir = z + beta * pdir
        norms.append(float(np.sqrt(np.sum(r * r))))
    return x.reshape(-1), np.array(norms)


def saved_paths(beta: float, R: int, lblock: int) -> int:
    """L from beta = L/(RN) (Section 4.2.2). READING: L is rounded to the
    nearest even number, so that the saved paths sit symmetrically around the
    frame centre (Section 4.3: 1% -> 82 and 10% -> 820 paths at N = 2048, R = 4)."""
    return int(2 * round(beta * R * lblock / 2.0))


def structured_mask(lblock: int, nblock: int, R: int, L: int) -> np.ndarray:
    """Prior mask of the sample-saving strategy (Section 4.2.2): every R-th
    sample (frames j = 0, R, 2R, ...) of the L sub-filter paths
    n in [N/2 - L/2, N/2 + L/2), the paths around N/2 that the quantisation
    noise corrupts most. uint8 [nblock * lblock], time order."""
    m = np.zeros((nblock, lblock), dtype=np.uint8)
    n0 = lblock // 2 - L // 2
    m[::R, n0:n0 + L] = 1
    return m.reshape(-1)


def ml_dense_solve(d, window, lblock, ntap, mask, prior, lam):
    """The converged ML answer on tiny sizes by a dense solve of the normal
    equations (A^T A + lam D) x = A^T d + lam D prior."""
    N = lblock
    d = np.asarray(d, dtype=np.float64).reshape(-1, N)
    b = d.shape[0]
    S = b * N
    A = np.zeros((S, S))
    for col in range(S):
        e = np.zeros(S)
        e[col] = 1.0
        A[:, col] = sw_apply(e, window, lblock, ntap).reshape(-1)
    D = np.diag(np.asarray(mask, dtype=np.float64).reshape(-1))
    H = A.T @ A + lam * D
    rhs = A.T @ d.reshape(-1) + lam * D @ np.asarray(prior, dtype=np.float64).reshape(-1)
    return np.linalg.solve(H, rhs)


# ----------------------------------------------------------------------------
# Appendix B closed forms (white input): naive and Wiener delta(f) on the
# full-rate frequency grid, via the polyphase decomposition of the spectrum.
# ----------------------------------------------------------------------------


def analytic_delta(window, lblock, ntap, nfreq, phi=None, snr=None):
    """delta at normalised sub-stream frequencies f_s = k/nfreq, k < nfreq.

    Naive (phi None): (1/SNR) (1/N) sum_n 1/|W_n(f_s)|^2.
    Wiener: 1 - (1/N) sum_n H_n(f_s), H without the (1+phi^2) factor.
    """
    W = column_spectra(window, lblock, ntap, nfreq)
    a2 = np.abs(W) ** 2
    if phi is None:
        return (1.0 / snr) * np.mean(1.0 / a2, axis=1)
    return 1.0 - np.mean(a2 / (a2 + phi * phi), axis=1)


# ----------------------------------------------------------------------------
# The alternative solvers of Appendix C (time complexity): a Tikhonov-
# regularised solve of the linear sub-problem by banded Cholesky, and FIR
# filtering with truncated decorrelation kernels.
# ----------------------------------------------------------------------------


def linear_subproblem(wn: np.ndarray, nblock: int) -> np.ndarray:
    """W_n of the sub-filter equation (Section 2.3): the [b-p+1, b] Toeplitz
    matrix with W[k][k+r] = w_n[r], built entry by entry."""
    p = len(wn)
    W = np.zeros((nblock - p + 1, nblock))
    for k in range(nblock - p + 1):
        for r in range(p):
            W[k, k + r] = wn[r]
    return W


def tikhonov_banded(d_lin: np.ndarray, window: np.ndarray, lblock: int, ntap: int, phi: float,
                    normalise: bool = True) -> np.ndarray:
    """Per column, the Tikhonov-regularised solution of the linear sub-problem
    d_n = W_n x_n (Appendix C: the Wiener machinery replicated by a
    pseudo-inverse with Tikhonov regularisation, solved by banded Cholesky):
    x_n = c (W_n^T W_n + phi^2 I)^{-1} W_n^T d_n, c = 1 + phi^2 (normalise)
    or 1. d_lin: [b - p + 1, N] frames after the row inverse of a linear PFB;
    returns [b, N]. W^T W + phi^2 I has bandwidth p - 1; scipy's banded
    Cholesky solver (LAPACK pbsv) is the library step."""
    from scipy.linalg import solveh_banded
    d_lin = np.asarray(d_lin, dtype=np.float64)
    nspec = d_lin.shape[0]
    b = nspec + ntap - 1
    H = np.asarray(window, dtype=np.float64).reshape(ntap, lblock)
    c = (1.0 + phi * phi) if normalise else 1.0
    x = np.zeros((b, lblock))
    for n in range(lblock):
        W = linear_subproblem(H[:, n], b)
        A = W.T @ W + phi * phi * np.eye(b)
        # lower banded storage: ab[t, i] = A[i + t, i]
        ab = np.zeros((ntap, b))
        for t in range(ntap):
            ab[t, :b - t] = np.diagonal(A, -t)
        x[:, n] = c * solveh_banded(ab, W.T @ d_lin[:, n], lower=True)
    return x


def fir_kernels(window: np.ndarray, lblock: int, ntap: int, nblock: int, phi: float, ltaps: int,
                normalise: bool = True) -> np.ndarray:
    """The decorrelation kernels of Section 3.1 / Appendix C, truncated to
    ltaps (odd) lags: the circulant Wiener inverse's impulse response (its
    output for d = a unit sample at frame 0), g_n[t] for the lags
    t = c - T .. c + T, T = (ltaps-1)/2, taken mod b. READING: the kernels are
    centred on c = p // 2, the delay of the window's main lobe (the sinc peaks
    at sample M/2 = (p/2) N, so the inverse filters peak at lag p/2); the
    paper does not say where its truncated kernels start. Returns [ltaps, N]."""
    T = (ltaps - 1) // 2
    delta = np.zeros((nblock, lblock))
    delta[0] = 1.0
    c = column_inverse(delta, window, lblock, ntap, phi, normalise)
    return c[(np.arange(-T, T + 1) + ntap // 2) % nblock]


def fir_apply(d: np.ndarray, g: np.ndarray, center: int) -> np.ndarray:
    """x_n[j] = sum_t g_n[t] d_n[(j - t) mod b] over the kernels' lags
    t = center - T .. center + T (FIR filtering of each sub-filter path with
    its decorrelation kernel, Appendix C)."""
    d = np.asarray(d, dtype=np.float64)
    b = d.shape[0]
    T = (g.shape[0] - 1) // 2
    x = np.zeros_like(d)
    j = np.arange(b)
    for i, t in enumerate(range(center - T, center + T + 1)):
        x += g[i][None, :] * d[(j - t) % b]
    return x


def ipfb_fir(packed: np.ndarray, scales_f32: np.ndarray, window: np.ndarray, lblock: int, ntap: int,
             phi: float, ltaps: int, normalise: bool = True) -> np.ndarray:
    """Dequantise 4-bit spectra, row inverse, FIR decorrelation with the
    truncated kernels; returns x[j*N + n]."""
    qr, qi = unpack_c4(packed)
    d = row_inverse(dequantize(qr, qi, scales_f32), lblock)
    g = fir_kernels(window, lblock, ntap, d.shape[0], phi, ltaps, normalise)
    return fir_apply(d, g, ntap // 2).reshape(-1)
