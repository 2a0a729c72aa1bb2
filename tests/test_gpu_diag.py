"""GPU tests of the Appendix B diagnostics (predicted and measured delta(f))
and of the structured prior mask with the ML-CG form (Section 4.2.2 sample
saving), against the FP64 oracle."""
import numpy as np
import pytest

from oracle import ipfb_oracle as O
from paper_2608_23441_amd import inputs as I
from paper_2608_23441_amd import ipfb
from maskbits import pack_bits, unpack_bits

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


@pytest.mark.parametrize("N,p,nfreq", [(64, 4, 512), (2048, 4, 4096), (32, 5, 7), (16, 4, 3)])
def test_delta_analytic_matches_oracle(N, p, nfreq):
    w = O.window_sinc_hamming(p, N)
    plan = ipfb.Plan(N, p, w, 16, ipfb.F32)  # the prediction uses the FP64 window in either precision
    for phi, snr in [(0.1, 0.0), (0.35, 0.0), (0.0, 80.0)]:
        got = _host(ipfb.delta_analytic(plan, nfreq, phi, snr))
        ref = O.analytic_delta(w, N, p, nfreq, phi=phi if phi > 0 else None, snr=snr)
        assert np.max(np.abs(got - ref) / np.abs(ref)) < 1e-10, (phi, snr)


@pytest.mark.parametrize("prec,tol", [(ipfb.F64, 1e-10), (ipfb.F32, 1e-4)])
@pytest.mark.parametrize("Nf,bf", [(512, 64), (65536, 8)])
def test_autospectrum_error_matches_oracle(prec, tol, Nf, bf):
    # small fine frames (LDS path) and long ones (two-pass path with the power sums)
    wf = O.window_sinc_hamming(4, Nf)
    x = I.gaussian_timestream(Nf * bf, 600)
    xh = x + 0.1 * I.gaussian_timestream(Nf * bf, 601)
    fine = ipfb.Plan(Nf, 4, wf, bf, prec)
    dt = torch.float64 if prec == ipfb.F64 else torch.float32
    xt, xht = _dev(x).to(dt), _dev(xh).to(dt)
    got = _host(ipfb.autospectrum_error(fine, xt, xht))
    xin, xhin = _host(xt).astype(np.float64), _host(xht).astype(np.float64)  # the values the GPU read
    ref = O.autospectrum_error(O.upchannelize(xin, Nf, 4, wf), O.upchannelize(xhin, Nf, 4, wf))
    assert np.max(np.abs(got - ref) / ref) < tol
    # a second call reuses the plan's workspace
    got2 = _host(ipfb.autospectrum_error(fine, xt, xt))
    assert np.all(got2 == 0.0)


@pytest.mark.parametrize("N,b,R,L", [(2048, 64, 4, 82), (64, 512, 4, 26), (64, 10, 4, 8), (32, 7, 3, 2),
                                     (16, 5, 1, 16), (16, 4, 2, 0)])
def test_mask_structured_matches_oracle(N, b, R, L):
    plan = ipfb.Plan(N, 4, O.window_sinc_hamming(4, N), b, ipfb.F32)
    words = _host(ipfb.mask_structured(plan, R, L))
    assert words.size == (N * b + 31) // 32
    assert np.array_equal(unpack_bits(words, N * b), O.structured_mask(N, b, R, L).astype(bool))
    # bits past the last sample are zero
    assert np.array_equal(words, pack_bits(O.structured_mask(N, b, R, L)))


# The byte-to-bit packer: ragged lengths (not a multiple of 32 or 64), a
# whole-wavefront length, one sample, and a length past one grid sweep.
@pytest.mark.parametrize("S", [1, 31, 33, 64, 100, 4097, 8192 * 256 + 77])
def test_mask_pack_bit_exact(S):
    m = I.random_mask(S, 0.3, 40 + S % 1000)
    words = _host(ipfb.mask_pack(_dev(m.astype(np.uint8))))
    assert np.array_equal(words, pack_bits(m))
    words_b = _host(ipfb.mask_pack(_dev(m)))  # bool input, same bytes
    assert np.array_equal(words_b, words)


@pytest.mark.parametrize("prec,tol", [(ipfb.F64, 1e-6), (ipfb.F32, 2e-4)])
def test_ml_cg_structured_prior_matches_oracle(prec, tol):
    # Section 4.3's setting at a small size: 4-bit at the 0.353 sigma spacing,
    # 25 iterations from the Wiener solution, every 4th sample of the paths
    # around N/2 saved (beta = 10 %)
    N, p, b, iters = 64, 4, 512, 25
    w = O.window_sinc_hamming(p, N)
    x = I.gaussian_timestream(N * b, 21)
    y = O.pfb_forward(x, w, N, p)
    sc = O.channel_scales(y, 1 / 0.353)
    qr, qi = O.quantize(y, sc)
    packed = O.pack_c4(qr, qi)
    L = O.saved_paths(0.10, 4, N)
    plan = ipfb.Plan(N, p, w, b, prec)
    mask = ipfb.mask_structured(plan, 4, L)
    d = O.row_inverse(O.dequantize(qr, qi, sc), N)
    x0 = O.column_inverse(d, w, N, p, 0.1).reshape(-1)
    ref_x, ref_n = O.ml_pcg(d, w, N, p, O.structured_mask(N, b, 4, L), x, 1.0, 0.1, iters, x0)
    dt = torch.float64 if prec == ipfb.F64 else torch.float32
    xg, ng = ipfb.ml_cg(plan, _dev(packed), _dev(sc), mask, _dev(x).to(dt), 1.0, 0.1, 0.1, iters)
    assert _rel(_host(xg).astype(np.float64), ref_x) < tol
    ng = _host(ng)
    if prec == ipfb.F64:
        k = ref_n > 1e-4 * ref_n[0]
        assert np.max(np.abs(ng[k] - ref_n[k]) / ref_n[k]) < 1e-6
    else:  # FP32 vectors: the first residual agrees, then the trajectories part by rounding
        assert abs(ng[0] - ref_n[0]) / ref_n[0] < 1e-5
        assert ng[-1] < ng[0]
