"""GPU tests of the differentiation form (autograd over the HIP forward PFB and
adjoint) and the maximum-likelihood CG form, against the FP64 oracle."""
import numpy as np
import pytest

from oracle import ipfb_oracle as O
from paper_2608_23441_amd import inputs as I
from paper_2608_23441_amd import ipfb
from maskbits import pack_bits

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def _ml_case(N, p, b, seed, frac=0.1, window=None):
    w = O.window_sinc_hamming(p, N) if window is None else window
    x = I.gaussian_timestream(N * b, seed)
    y = O.pfb_forward(x, w, N, p)
    s = O.channel_scales(y)
    qr, qi = O.quantize(y, s)
    packed = O.pack_c4(qr, qi)
    mask = I.random_mask(N * b, frac, seed + 1)
    d = O.row_inverse(O.dequantize(qr, qi, s), N)
    return w, x, packed, s, mask, d


# --- F4: maximum-likelihood PCG -------------------------------------------------
@pytest.mark.parametrize("N,b,iters", [(8, 16, 100), (256, 64, 30)])
def test_ml_cg_fp64_matches_oracle(N, b, iters):
    p = 4
    print(f"case ml_cg fp64 N={N} b={b} iters={iters}", flush=True)
    w, x, packed, s, mask, d = _ml_case(N, p, b, 300 + N)
    x0 = O.column_inverse(d, w, N, p, 0.1).reshape(-1)
    ref_x, ref_n = O.ml_pcg(d, w, N, p, mask, x, 1.0, 0.1, iters, x0)
    plan = ipfb.Plan(N, p, w, b, ipfb.F64)
    xg, ng = ipfb.ml_cg(plan, _dev(packed), _dev(s), _dev(pack_bits(mask)), _dev(x), 1.0, 0.1, 0.1, iters)
    xg, ng = _host(xg), _host(ng)
    # residual histories agree while the residual is well above rounding
    # (once |r_k| nears 1e-7 |r_0| CG's rounding, which differs in summation
    # order, takes over and the two trajectories legitimately part)
    k = ref_n > 1e-4 * ref_n[0]
    assert k.sum() >= 5
    assert np.max(np.abs(ng[k] - ref_n[k]) / ref_n[k]) < 1e-6
    assert _rel(xg, ref_x) < 1e-6
    if N * b <= 256:  # converged: the dense ML solution
        dense = O.ml_dense_solve(d, w, N, p, mask, x, 1.0)
        assert _rel(xg, dense) < 1e-6


def test_ml_cg_ci8_matches_oracle():
    N, p, b, iters = 256, 4, 64, 30
    print("case ml_cg fp64 ci8", flush=True)
    w = O.window_sinc_hamming(p, N)
    x = I.gaussian_timestream(N * b, 310)
    y = O.pfb_forward(x, w, N, p)
    s = O.channel_scales(y, levels_rms=40.0)
    qr, qi = O.quantize(y, s, qmax=127)
    mask = I.random_mask(N * b, 0.1, 311)
    d = O.row_inverse(O.dequantize(qr, qi, s), N)
    x0 = O.column_inverse(d, w, N, p, 0.1).reshape(-1)
    ref_x, ref_n = O.ml_pcg(d, w, N, p, mask, x, 1.0, 0.1, iters, x0)
    plan = ipfb.Plan(N, p, w, b, ipfb.F64)
    xg, ng = ipfb.ml_cg(plan, _dev(O.pack_ci8(qr, qi)), _dev(s), _dev(pack_bits(mask)), _dev(x), 1.0, 0.1,
                        0.1, iters)
    xg, ng = _host(xg), _host(ng)
    k = ref_n > 1e-4 * ref_n[0]
    assert k.sum() >= 5
    assert np.max(np.abs(ng[k] - ref_n[k]) / ref_n[k]) < 1e-6
    assert _rel(xg, ref_x) < 1e-6


def test_ml_cg_bitwise_deterministic():
    # the dot products reduce in a fixed order (wavefront butterflies, then
    # wavefronts, then workgroups in index order): two runs agree bit for bit
    N, p, b = 256, 4, 1024
    print("case ml_cg determinism", flush=True)
    w, x, packed, s, mask, d = _ml_case(N, p, b, 320)
    plan = ipfb.Plan(N, p, w, b, ipfb.F32)
    runs = []
    for _ in range(2):
        xg, ng = ipfb.ml_cg(plan, _dev(packed), _dev(s), _dev(pack_bits(mask)),
                            _dev(x).to(torch.float32), 1.0, 0.1, 0.1, 20)
        runs.append((_host(xg).copy(), _host(ng).copy()))
    assert np.array_equal(runs[0][0].view(np.uint8), runs[1][0].view(np.uint8))
    assert np.array_equal(runs[0][1].view(np.uint8), runs[1][1].view(np.uint8))


def test_ml_cg_zero_iterations_is_wiener():
    N, p, b = 64, 4, 32
    w, x, packed, s, mask, d = _ml_case(N, p, b, 310)
    plan = ipfb.Plan(N, p, w, b, ipfb.F64)
    xg, ng = ipfb.ml_cg(plan, _dev(packed), _dev(s), _dev(pack_bits(mask)), _dev(x), 1.0, 0.1, 0.1, 0)
    xw = ipfb.ipfb_wiener(plan, _dev(packed), _dev(s), 0.1)
    # the same Wiener estimate through two column-stage layouts: equal up to
    # FP64 rounding order
    assert _rel(_host(xg), _host(xw)) < 1e-13


def test_ml_cg_toy_model_one_saved_sample():
    # Section 4.2.2: symmetric window, no quantisation, one saved sample on
    # path N/2 pins the Nyquist null mode; CG converges to the true timestream
    N, p, b = 8, 4, 16
    w = O.window_symmetric_hann(p, N)
    x = I.gaussian_timestream(N * b, 24)
    y = O.pfb_forward(x, w, N, p)
    mask = np.zeros(N * b, dtype=np.uint8)
    mask[3 * N + N // 2] = 1
    plan = ipfb.Plan(N, p, w, b, ipfb.F64)
    xg, ng = ipfb.ml_cg(plan, _dev(y), None, _dev(pack_bits(mask)), _dev(x), 1.0, 0.1, 0.1, 80)
    assert np.abs(_host(xg) - x).max() < 1e-8


def test_ml_cg_fp32_form():
    # ML-form shapes scaled down: FP32 vectors, FP64 dots; trajectories differ
    # from FP64 only by rounding, so the iterate is compared with a loose bound
    N, p, b, iters = 2048, 4, 256, 100
    print("case ml_cg fp32", flush=True)
    w, x, packed, s, mask, d = _ml_case(N, p, b, 320)
    x0 = O.column_inverse(d, w, N, p, 0.1).reshape(-1)
    ref_x, ref_n = O.ml_pcg(d, w, N, p, mask, x, 1.0, 0.1, iters, x0)
    plan = ipfb.Plan(N, p, w, b, ipfb.F32)
    xg, ng = ipfb.ml_cg(plan, _dev(packed), _dev(s), _dev(pack_bits(mask)),
                        _dev(x.astype(np.float32)), 1.0, 0.1, 0.1, iters)
    xg, ng = _host(xg), _host(ng)
    err = _rel(xg.astype(np.float64), ref_x)
    print(f"fp32 ML-CG x_100 rel err vs FP64 oracle: {err:.2e}; resid {ng[0]:.3e} -> {ng[-1]:.3e}")
    assert err < 1e-4
    assert abs(ng[0] - ref_n[0]) / ref_n[0] < 1e-5
    assert ng[-1] < 1e-2 * ng[0]
    # the prior improves on the Wiener start where samples were saved
    assert np.sqrt(np.mean((xg - x) ** 2)) < np.sqrt(np.mean((x0 - x) ** 2))


def test_ml_cg_rejects_bad_arguments():
    N, p, b = 64, 4, 16
    w, x, packed, s, mask, d = _ml_case(N, p, b, 330)
    plan = ipfb.Plan(N, p, w, b, ipfb.F64)
    with pytest.raises(ipfb.IpfbError):
        ipfb.ml_cg(plan, _dev(packed), _dev(s), _dev(pack_bits(mask)), _dev(x), 1.0, 0.1, 0.0, 5)
    with pytest.raises(ipfb.IpfbError):
        ipfb.ml_cg(plan, _dev(packed), _dev(s), _dev(pack_bits(mask)), _dev(x), -1.0, 0.1, 0.1, 5)


# --- F3: autograd through the forward PFB ------------------------------------------
def test_autograd_gradcheck_fp64():
    from paper_2608_23441_amd.autograd import pfb
    N, p, b = 16, 4, 6
    w = O.window_sinc_hamming(p, N)
    plan = ipfb.Plan(N, p, w, b, ipfb.F64)
    x = _dev(I.gaussian_timestream(N * b, 340)).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda v: pfb(v, plan), (x,), eps=1e-6, atol=1e-8, rtol=1e-6)


def test_autograd_backward_is_adjoint_and_finite_differences_fp32():
    from paper_2608_23441_amd.autograd import pfb
    N, p, b = 512, 4, 16
    w = O.window_sinc_hamming(p, N)
    plan = ipfb.Plan(N, p, w, b, ipfb.F32)
    x0 = I.gaussian_timestream(N * b, 341)
    c = I.complex_block((b, N // 2 + 1), 342)
    x = _dev(x0.astype(np.float32)).requires_grad_(True)
    cw = _dev(c.astype(np.complex64))
    loss = torch.real(torch.sum(torch.conj(cw) * pfb(x, plan)))
    loss.backward()
    g = _host(x.grad).astype(np.float64)
    # the adjoint oracle: d loss / d x = Re[(FSW)^H c]
    ref = O.pfb_adjoint(c, w, N, p, b)
    assert _rel(g, ref) < 1e-5
    # central finite differences along a random direction (FP64 oracle loss)
    v = I.gaussian_timestream(N * b, 343)
    h = 1e-3
    lp = np.real(np.vdot(c, O.pfb_forward(x0 + h * v, w, N, p)))
    lm = np.real(np.vdot(c, O.pfb_forward(x0 - h * v, w, N, p)))
    fd = (lp - lm) / (2 * h)
    assert abs(fd - np.dot(g, v)) / abs(fd) < 1e-4


@pytest.mark.parametrize("prec", [ipfb.F32, ipfb.F64])
def test_ml_cg_reads_no_workspace_before_writing_it(prec):
    # device memory handed back with NaN in it; the CG workspace is allocated
    # afterwards and may land on those pages: the first search direction must
    # be set, not updated from whatever the workspace held
    N, p, b = 64, 4, 512
    w, x, packed, s, mask, d = _ml_case(N, p, b, 330)
    poison = torch.full((64 << 20,), float("nan"), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    del poison
    torch.cuda.empty_cache()
    plan = ipfb.Plan(N, p, w, b, prec)
    dt = torch.float64 if prec == ipfb.F64 else torch.float32
    xg, ng = ipfb.ml_cg(plan, _dev(packed), _dev(s), _dev(pack_bits(mask)), _dev(x).to(dt), 1.0, 0.1, 0.1, 3)
    assert np.all(np.isfinite(_host(xg))) and np.all(np.isfinite(_host(ng)))


def test_ml_cg_long_columns_take_the_separate_dot_product():
    # 2^14 frames in FP64: the column kernel runs one column per workgroup,
    # 2048 workgroups, more than the partial-sum slots, so r.z is its own pass
    N, p, b, iters = 2048, 4, 16384, 2
    print(f"case ml_cg separate dot N={N} b={b}", flush=True)
    w, x, packed, s, mask, d = _ml_case(N, p, b, 340)
    x0 = O.column_inverse(d, w, N, p, 0.1).reshape(-1)
    ref_x, ref_n = O.ml_pcg(d, w, N, p, mask, x, 1.0, 0.1, iters, x0)
    plan = ipfb.Plan(N, p, w, b, ipfb.F64)
    xg, ng = ipfb.ml_cg(plan, _dev(packed), _dev(s), _dev(pack_bits(mask)), _dev(x), 1.0, 0.1, 0.1, iters)
    assert np.max(np.abs(_host(ng) - ref_n) / ref_n) < 1e-9
    assert _rel(_host(xg), ref_x) < 1e-9
