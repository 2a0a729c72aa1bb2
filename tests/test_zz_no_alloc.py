"""The allocation-free CG entry point, called through the C ABI: its results
equal ipfb_ml_cg's (same kernels on the same inputs, so bit for bit) on two
calls in a row, the second on a smaller plan, in both the transposed and the
natural-layout form, and a plan whose solve does not fit its static scratch
array is rejected before anything runs."""
import ctypes

import numpy as np
import pytest

from maskbits import pack_bits
from oracle import ipfb_oracle as O
from paper_2608_23441_amd import inputs as I
from paper_2608_23441_amd import ipfb

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _case(N, p, b, seed, prec):
    w = O.window_sinc_hamming(p, N)
    x = I.gaussian_timestream(N * b, seed)
    y = O.pfb_forward(x, w, N, p)
    s = O.channel_scales(y)
    packed = O.pack_c4(*O.quantize(y, s))
    mask = I.random_mask(N * b, 0.1, seed + 1)
    dt = np.float32 if prec == ipfb.F32 else np.float64
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    return w, dev(packed), dev(s), dev(pack_bits(mask)), dev(x.astype(dt))


def _call(fn, plan, packed, s, mask, prior, iters, dt):
    S = plan.nblock * plan.lblock
    x = torch.empty(S, dtype=dt, device="cuda")
    norms = torch.empty(iters + 1, dtype=torch.float64, device="cuda")
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    status = fn(plan.handle, ipfb.IN_C4, ctypes.c_void_p(packed.data_ptr()), ctypes.c_void_p(s.data_ptr()),
                ctypes.c_void_p(mask.data_ptr()), ctypes.c_void_p(prior.data_ptr()), 1.0, 0.1, 0.1, iters, None,
                ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(norms.data_ptr()), st)
    assert status == ipfb.OK, ipfb.lib().ipfb_last_error().decode()
    torch.cuda.synchronize()
    return x.cpu().numpy(), norms.cpu().numpy()


@pytest.mark.parametrize("prec", [ipfb.F32, ipfb.F64])
def test_noalloc_matches_ml_cg_twice_then_smaller(prec):
    L = ipfb.lib()
    dt = torch.float32 if prec == ipfb.F32 else torch.float64
    # the largest power-of-two shape that fits the scratch array, then a smaller one
    shapes = [(2048, 1024, 20), (256, 64, 30)] if prec == ipfb.F32 else [(1024, 1024, 20), (256, 64, 30)]
    for k, (N, b, iters) in enumerate(shapes):
        print(f"case ml_cg_noalloc prec={prec} N={N} b={b} iters={iters}", flush=True)
        w, packed, s, mask, prior = _case(N, 4, b, 600 + 7 * k + prec, prec)
        plan = ipfb.Plan(N, 4, w, b, prec)
        xr, nr = _call(L.ipfb_ml_cg, plan, packed, s, mask, prior, iters, dt)
        xa, na = _call(L.ipfb_ml_cg_noalloc, plan, packed, s, mask, prior, iters, dt)
        assert np.array_equal(xa, xr) and np.array_equal(na, nr)
        assert nr[-1] < nr[0]


@pytest.mark.parametrize("prec", [ipfb.F32, ipfb.F64])
def test_noalloc_natural_layout_twice_then_smaller(prec):
    # nblock not a power of two: the natural-layout solve (recursive
    # preconditioner, whose coefficients the plan holds from its creation)
    L = ipfb.lib()
    dt = torch.float32 if prec == ipfb.F32 else torch.float64
    for k, (N, b, iters) in enumerate([(512, 1500, 20), (64, 300, 30)]):
        print(f"case ml_cg_noalloc natural prec={prec} N={N} b={b} iters={iters}", flush=True)
        w, packed, s, mask, prior = _case(N, 4, b, 640 + 7 * k + prec, prec)
        plan = ipfb.Plan(N, 4, w, b, prec)
        xr, nr = _call(L.ipfb_ml_cg, plan, packed, s, mask, prior, iters, dt)
        xa, na = _call(L.ipfb_ml_cg_noalloc, plan, packed, s, mask, prior, iters, dt)
        assert np.array_equal(xa, xr) and np.array_equal(na, nr)
        assert nr[-1] < nr[0]


def test_noalloc_rejects_a_solve_beyond_the_scratch_array():
    L = ipfb.lib()
    N, b = 2048, 2048  # 2^22 FP32 samples: 7 vectors alone are 112 MiB
    w = O.window_sinc_hamming(4, N)
    plan = ipfb.Plan(N, 4, w, b, ipfb.F32)
    dummy = torch.zeros(N * b, dtype=torch.float32, device="cuda")
    spec = torch.zeros((b, N // 2 + 1), dtype=torch.uint8, device="cuda")
    sc = torch.ones(N // 2 + 1, dtype=torch.float32, device="cuda")
    mask = torch.zeros((N * b + 31) // 32, dtype=torch.int32, device="cuda")
    p = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    status = L.ipfb_ml_cg_noalloc(plan.handle, ipfb.IN_C4, p(spec), p(sc), p(mask), p(dummy), 1.0, 0.1, 0.1, 5,
                                  None, p(dummy), None, None)
    assert status == ipfb.EUNSUPPORTED
    assert "scratch" in L.ipfb_last_error().decode()
