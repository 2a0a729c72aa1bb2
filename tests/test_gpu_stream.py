"""GPU tests of the linear-boundary streaming inverse (overlap-save windows of
the circulant Wiener inverse) against the FP64 oracle's streaming inverse on
the same 4-bit ints (or the same complex spectra)."""
import numpy as np
import pytest

from oracle import ipfb_oracle as O
from paper_2608_23441_amd import inputs as I
from paper_2608_23441_amd import ipfb

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def _linear_spectra(N, p, nspec, seed, window):
    x = I.gaussian_timestream(N * (nspec + p - 1), seed)
    return O.pfb_forward(x, window, N, p, circular=False)


# (N, p, chunk, halo, nspec): one-pass windows (chunk <= 512: copy of the kept
# frames) and larger windows (4 taps: the recursive column stage; else the
# three FFT passes; either way the kept frames written by the last pass);
# several windows with a ragged last one, a stream shorter than one window,
# exactly one window, one spectrum, a few spectra in a large window
CASES = [(64, 4, 64, 8, 300), (64, 4, 1024, 100, 3000), (128, 4, 2048, 256, 700), (64, 3, 64, 0, 62),
         (64, 4, 64, 8, 1), (32, 5, 512, 30, 2000), (256, 4, 4096, 300, 9000), (64, 4, 1024, 100, 5),
         (32, 5, 1024, 60, 2500)]


@pytest.mark.parametrize("prec,tol", [(ipfb.F64, 1e-11), (ipfb.F32, 1e-5)])
@pytest.mark.parametrize("N,p,chunk,halo,nspec", CASES)
def test_stream_c4_matches_oracle(prec, tol, N, p, chunk, halo, nspec):
    print(f"case stream c4 prec={prec} N={N} p={p} chunk={chunk} halo={halo} nspec={nspec}", flush=True)
    w = O.window_sinc_hamming(p, N)
    y = _linear_spectra(N, p, nspec, 5000 + N + nspec, w)
    sc = O.channel_scales(y)
    qr, qi = O.quantize(y, sc)
    pk = O.pack_c4(qr, qi)
    ref = O.ipfb_stream(pk, sc, w, N, p, 0.1, chunk, halo)
    sp = ipfb.StreamPlan(N, p, w, chunk, halo, prec)
    out = ipfb.wiener_stream(sp, torch.from_numpy(pk).cuda(), torch.from_numpy(sc).cuda(), 0.1)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    assert got.shape == ref.shape
    assert _rel(got, ref) < tol


@pytest.mark.parametrize("prec,tol", [(ipfb.F64, 1e-11), (ipfb.F32, 1e-5)])
def test_stream_ci8_matches_oracle(prec, tol):
    N, p, chunk, halo, nspec = 64, 4, 1024, 100, 3000
    print(f"case stream ci8 prec={prec}", flush=True)
    w = O.window_sinc_hamming(p, N)
    y = _linear_spectra(N, p, nspec, 5200, w)
    sc = O.channel_scales(y, levels_rms=40.0)
    qr, qi = O.quantize(y, sc, qmax=127)
    pk = O.pack_ci8(qr, qi)
    ref = O.ipfb_stream_from_spectra(O.dequantize(qr, qi, sc), w, N, p, 0.1, chunk, halo)
    sp = ipfb.StreamPlan(N, p, w, chunk, halo, prec)
    out = ipfb.wiener_stream(sp, torch.from_numpy(pk).cuda(), torch.from_numpy(sc).cuda(), 0.1)
    torch.cuda.synchronize()
    assert _rel(out.cpu().numpy().astype(np.float64), ref) < tol


@pytest.mark.parametrize("prec,tol", [(ipfb.F64, 1e-11), (ipfb.F32, 1e-5)])
def test_stream_complex_input_and_phi_zero(prec, tol):
    N, p, chunk, halo, nspec = 64, 4, 1024, 64, 2500
    w = O.window_sinc_hamming(p, N)
    y = _linear_spectra(N, p, nspec, 5100, w)
    sp = ipfb.StreamPlan(N, p, w, chunk, halo, prec)
    cdt = torch.complex128 if prec == ipfb.F64 else torch.complex64
    yt = torch.from_numpy(y).to(cdt).cuda()
    yin = yt.cpu().numpy().astype(np.complex128)  # the values the GPU reads
    for phi, norm in [(0.1, True), (0.3, False), (0.0, True)]:
        ref = O.ipfb_stream_from_spectra(yin, w, N, p, phi, chunk, halo, norm)
        got = ipfb.wiener_stream(sp, yt, None, phi, normalise=norm).cpu().numpy().astype(np.float64)
        assert _rel(got, ref) < (tol if phi > 0 else 100 * tol), (phi, norm)


def test_stream_single_window_equals_block_inverse_of_padded_data():
    # nspec = chunk - (p - 1): one window, i.e. the zero-extended block inverse
    N, p, chunk = 128, 4, 1024
    w = O.window_sinc_hamming(p, N)
    nspec = chunk - (p - 1)
    y = _linear_spectra(N, p, nspec, 5200, w)
    ref = O.ipfb_linear_from_spectra(y, w, N, p, 0.1)
    sp = ipfb.StreamPlan(N, p, w, chunk, 50, ipfb.F64)
    got = ipfb.wiener_stream(sp, torch.from_numpy(y).cuda(), None, 0.1).cpu().numpy()
    assert _rel(got, ref) < 1e-11


def test_stream_production_shape_fp32():
    # production frame length, 16384-frame windows with a 256-frame halo, two windows
    N, p, chunk, halo, nspec = 4096, 4, 16384, 256, 20000
    print("case stream production shape", flush=True)
    w = O.window_sinc_hamming(p, N)
    y = _linear_spectra(N, p, nspec, 5300, w)
    sc = O.channel_scales(y)
    qr, qi = O.quantize(y, sc)
    del y
    pk = O.pack_c4(qr, qi)
    ref = O.ipfb_stream(pk, sc, w, N, p, 0.1, chunk, halo)
    sp = ipfb.StreamPlan(N, p, w, chunk, halo, ipfb.F32)
    got = ipfb.wiener_stream(sp, torch.from_numpy(pk).cuda(), torch.from_numpy(sc).cuda(), 0.1)
    torch.cuda.synchronize()
    err = _rel(got.cpu().numpy().astype(np.float64), ref)
    print(f"stream production rel RMS {err:.2e}")
    assert err < 1e-5


def test_stream_rejects_bad_plans():
    w = O.window_sinc_hamming(4, 64)
    for chunk, halo in [(100, 8), (64, 31), (2, 0), (64, -1), (1 << 16, 8)]:
        with pytest.raises(ipfb.IpfbError):
            ipfb.StreamPlan(64, 4, w, chunk, halo, ipfb.F32)
