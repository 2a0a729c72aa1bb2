"""Appendix C's comparison solvers on the GPU against the FP64 oracle: the
Tikhonov-regularised linear sub-problems by banded Cholesky, and FIR
decorrelation with truncated kernels (the kernels themselves, and the
inverse made with them)."""
import numpy as np
import pytest

from oracle import ipfb_oracle as O
from paper_2608_23441_amd import inputs as I
from paper_2608_23441_amd import ipfb
from parity_metrics import rel, worst_column_rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = {ipfb.F64: 1e-12, ipfb.F32: 1e-5}


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("prec", [ipfb.F64, ipfb.F32])
@pytest.mark.parametrize("N,p,b,phi", [(16, 4, 64, 0.1), (8, 2, 20, 0.3), (32, 3, 50, 0.1), (16, 5, 40, 0.2),
                                       (64, 8, 200, 0.1), (32, 16, 100, 0.1), (256, 4, 1024, 0.1)])
def test_tikhonov_matches_oracle(prec, N, p, b, phi):
    print(f"case tikhonov prec={prec} N={N} p={p} b={b} phi={phi}", flush=True)
    w = O.window_sinc_hamming(p, N)
    x = I.gaussian_timestream(N * b, 500 + N + p)
    y = O.pfb_forward(x, w, N, p, circular=False)  # b - p + 1 spectra
    s = O.channel_scales(y)
    qr, qi = O.quantize(y, s)
    packed = O.pack_c4(qr, qi)
    d = O.row_inverse(O.dequantize(qr, qi, s), N)
    ref = O.tikhonov_banded(d, w, N, p, phi)
    plan = ipfb.Plan(N, p, w, b, prec)
    got = _host(ipfb.tikhonov(plan, _dev(packed), _dev(s), phi)).reshape(b, N)
    ec, nc = worst_column_rel(got, ref, N)
    print(f"rel RMS {rel(got, ref):.3e}, worst path {ec:.3e} at n={nc}", flush=True)
    assert rel(got, ref) < TOL[prec]
    # a second call reuses the workspace; unnormalised
    got2 = _host(ipfb.tikhonov(plan, _dev(packed), _dev(s), phi, normalise=False)).reshape(b, N)
    assert rel(got2, ref / (1 + phi * phi)) < TOL[prec]


def test_tikhonov_rejects_bad_arguments():
    N, b = 16, 32
    plan = ipfb.Plan(N, 4, O.window_sinc_hamming(4, N), b, ipfb.F64)
    spec = torch.zeros((b - 3, N // 2 + 1), dtype=torch.complex128, device="cuda")
    with pytest.raises(ipfb.IpfbError) as e:
        ipfb.tikhonov(plan, spec, None, 0.0)
    assert e.value.status == ipfb.EINVAL
    plan6 = ipfb.Plan(N, 6, O.window_sinc_hamming(6, N), b, ipfb.F64)
    with pytest.raises(ipfb.IpfbError) as e:
        ipfb.tikhonov(plan6, torch.zeros((b - 5, N // 2 + 1), dtype=torch.complex128, device="cuda"), None, 0.1)
    assert e.value.status == ipfb.EUNSUPPORTED


@pytest.mark.parametrize("prec", [ipfb.F64, ipfb.F32])
@pytest.mark.parametrize("N,p,b,L", [(64, 4, 256, 51), (32, 8, 512, 101), (64, 4, 300, 31), (16, 16, 1024, 255),
                                     (8, 4, 64, 1)])
def test_fir_kernels_and_inverse_match_oracle(prec, N, p, b, L):
    # power-of-two nblock: the FFT column stage makes the kernels (8, 16 taps)
    # or the recursive one (4 taps); 300 frames: the recursive one
    phi = 0.1
    print(f"case fir prec={prec} N={N} p={p} b={b} L={L}", flush=True)
    w = O.window_sinc_hamming(p, N)
    gref = O.fir_kernels(w, N, p, b, phi, L)
    plan = ipfb.Plan(N, p, w, b, prec)
    g = _host(ipfb.fir_kernels(plan, phi, L))
    assert rel(g, gref) < TOL[prec]
    y = O.pfb_forward(I.gaussian_timestream(N * b, 600 + N), w, N, p)
    s = O.channel_scales(y)
    packed = O.pack_c4(*O.quantize(y, s))
    ref = O.ipfb_fir(packed, s, w, N, p, phi, L)
    got = _host(ipfb.fir(plan, _dev(packed), _dev(s), phi, L))
    assert rel(got, ref) < TOL[prec]
    assert worst_column_rel(got, ref, N)[0] < 10 * TOL[prec]
    # other phi / length / normalisation: the kernels are made again
    ref2 = O.ipfb_fir(packed, s, w, N, p, 0.2, 7, normalise=False)
    got2 = _host(ipfb.fir(plan, _dev(packed), _dev(s), 0.2, 7, normalise=False))
    assert rel(got2, ref2) < TOL[prec]


def test_fir_converges_to_the_circulant_inverse():
    # with more taps the FIR inverse approaches the circulant Wiener inverse
    N, p, b, phi = 128, 4, 1024, 0.1
    w = O.window_sinc_hamming(p, N)
    y = O.pfb_forward(I.gaussian_timestream(N * b, 610), w, N, p)
    s = O.channel_scales(y)
    packed = O.pack_c4(*O.quantize(y, s))
    plan = ipfb.Plan(N, p, w, b, ipfb.F64)
    exact = _host(ipfb.ipfb_wiener(plan, _dev(packed), _dev(s), phi))
    errs = [rel(_host(ipfb.fir(plan, _dev(packed), _dev(s), phi, L)), exact) for L in (11, 51, 101, 201)]
    print(f"FIR vs circulant rel RMS by length: {errs}", flush=True)
    assert all(errs[i + 1] < 0.5 * errs[i] for i in range(3)) and errs[-1] < 1e-6


def test_fir_rejects_bad_arguments():
    N, b = 16, 100
    plan = ipfb.Plan(N, 5, O.window_sinc_hamming(5, N), b, ipfb.F64)  # Bluestein columns: no in-place stage
    with pytest.raises(ipfb.IpfbError) as e:
        ipfb.fir_kernels(plan, 0.1, 11)
    assert e.value.status == ipfb.EUNSUPPORTED
    plan4 = ipfb.Plan(N, 4, O.window_sinc_hamming(4, N), 64, ipfb.F64)
    for bad in (0, 2, 257):
        with pytest.raises(ipfb.IpfbError):
            ipfb.fir_kernels(plan4, 0.1, bad)
    with pytest.raises(ipfb.IpfbError):
        ipfb.fir_kernels(plan4, 0.0, 11)
