"""Full-size parity at the production workload, in the launch configuration
the benchmark times: white noise + 5 tones, lblock = 4096, ntap = 4,
nblock = 16384 (2^26 samples), 4-bit spectra, Wiener phi = 0.1, x64
up-channelization with autospectrum. Every output element is compared with
the FP64 oracle (the oracle finishes this size in well under a minute)."""
import numpy as np
import pytest

from oracle import ipfb_oracle as O
from paper_2608_23441_amd import inputs as I
from paper_2608_23441_amd import ipfb
from parity_metrics import worst_column_rel

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

torch = pytest.importorskip("torch")

N, P, B, U, PHI = 4096, 4, 16384, 64, 0.1


@pytest.fixture(scope="module")
def production_case():
    x = I.timestream_with_tones(N * B, 2, 5, 102, 0.1)
    w = O.window_sinc_hamming(P, N)
    y = O.pfb_forward(x, w, N, P)
    s = O.channel_scales(y, 2.5)
    qr, qi = O.quantize(y, s)
    packed = O.pack_c4(qr, qi)
    del y, qr, qi
    xh = O.ipfb_wiener(packed, s, w, N, P, PHI)
    Nf = N * U
    wf = O.window_sinc_hamming(4, Nf)
    Y = O.upchannelize(xh, Nf, 4, wf)
    A = O.autospectrum(Y)
    return dict(x=x, w=w, wf=wf, packed=packed, s=s, xh=xh, Y=Y, A=A, Nf=Nf)


def _rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


@pytest.mark.parametrize("method", [ipfb.COLS_AUTO, ipfb.COLS_FFT])
@pytest.mark.parametrize("prec,tol_x,tol_A,tol_col", [(ipfb.F32, 1e-5, 1e-4, 1e-4), (ipfb.F64, 1e-12, 1e-10, 1e-11)])
def test_production_size_parity(production_case, prec, tol_x, tol_A, tol_col, method):
    # AUTO is the recursive column stage here (the benchmark's launch
    # configuration); COLS_FFT the three-pass FFT stage
    c = production_case
    print(f"case full-size prec={prec} method={method}", flush=True)
    coarse = ipfb.Plan(N, P, c["w"], B, prec)
    coarse.set_column_method(method)
    fine = ipfb.Plan(c["Nf"], 4, c["wf"], (N * B) // c["Nf"], prec)
    xh = ipfb.ipfb_wiener(coarse, torch.from_numpy(c["packed"]).cuda(), torch.from_numpy(c["s"]).cuda(), PHI)
    Y, A = ipfb.upchannelize(fine, xh)
    torch.cuda.synchronize()
    ex = _rel(xh.cpu().numpy().astype(np.float64), c["xh"])
    eY = _rel(Y.cpu().numpy().astype(np.complex128), c["Y"])
    Ah = A.cpu().numpy()
    eA = float(np.max(np.abs(Ah - c["A"]) / c["A"]))
    # the worst sub-filter path of the inverse and the worst fine channel
    ec, nc = worst_column_rel(xh.cpu().numpy().astype(np.float64), c["xh"], N)
    eYc, kc = worst_column_rel(Y.cpu().numpy().astype(np.complex128), c["Y"], c["Nf"] // 2 + 1)
    print(f"prec={prec}: timestream rel RMS {ex:.3e} (worst path {ec:.3e} at n={nc}), fine spectra rel RMS "
          f"{eY:.3e} (worst channel {eYc:.3e} at k={kc}), autospectrum max rel {eA:.3e}")
    assert ex < tol_x and eY < tol_x and eA < tol_A
    assert ec < tol_col and eYc < tol_col
    # the injected tones: each lands in its fine channel in the GPU autospectrum
    f, _ = I.tone_parameters(5, 102)
    for fi in f:
        k = int(round(fi * c["Nf"]))
        assert k - 3 + int(np.argmax(Ah[k - 3:k + 4])) == k
