"""GPU tests of the batched form: streams of uneven (arbitrary) nblock in one
call, Bluestein column DFTs for lengths that are not powers of two, replayed
from one captured HIP graph; every stream against the FP64 oracle."""
import numpy as np
import pytest

from oracle import ipfb_oracle as O
from paper_2608_23441_amd import inputs as I
from paper_2608_23441_amd import ipfb

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def _streams(N, p, nblocks, seed0):
    w = O.window_sinc_hamming(p, N)
    out = []
    for s, b in enumerate(nblocks):
        x = I.gaussian_timestream(N * b, seed0 + s)
        y = O.pfb_forward(x, w, N, p)
        sc = O.channel_scales(y)
        qr, qi = O.quantize(y, sc)
        out.append((O.pack_c4(qr, qi), sc))
    return w, out


@pytest.mark.parametrize("prec,tol", [(ipfb.F64, 1e-11), (ipfb.F32, 1e-5)])
def test_batched_small_uneven(prec, tol):
    N, p = 64, 4
    nblocks = [12, 37, 64, 100, 129, 5, 3, 2, 16, 1031]
    print(f"case batched small prec={prec}", flush=True)
    w, data = _streams(N, p, nblocks, 4000)
    bp = ipfb.BatchedPlan(N, p, w, nblocks, prec)
    specs = [torch.from_numpy(pk).cuda() for pk, _ in data]
    scs = [torch.from_numpy(sc).cuda() for _, sc in data]
    for phi in (0.1, 0.0):
        outs = ipfb.wiener_batched(bp, specs, scs, phi)
        torch.cuda.synchronize()
        for (pk, sc), b, xo in zip(data, nblocks, outs):
            ref = O.ipfb_wiener(pk, sc, w, N, p, phi)
            assert _rel(xo.cpu().numpy().astype(np.float64), ref) < (tol if phi > 0 else 50 * tol), (b, phi)


def test_batched_production_lengths_fp32():
    # production frame length with Bluestein lengths up to M = 65536
    N, p = 4096, 4
    nblocks = [1031, 3000, 16385, 2048]
    print("case batched production lengths", flush=True)
    w, data = _streams(N, p, nblocks, 4100)
    bp = ipfb.BatchedPlan(N, p, w, nblocks, ipfb.F32)
    outs = ipfb.wiener_batched(bp, [torch.from_numpy(pk).cuda() for pk, _ in data],
                               [torch.from_numpy(sc).cuda() for _, sc in data], 0.1)
    torch.cuda.synchronize()
    for (pk, sc), b, xo in zip(data, nblocks, outs):
        ref = O.ipfb_wiener(pk, sc, w, N, p, 0.1)
        err = _rel(xo.cpu().numpy().astype(np.float64), ref)
        print(f"b={b}: rel RMS {err:.2e}")
        assert err < 1e-5


def test_batched_graph_replays_match_eager():
    N, p = 128, 4
    nblocks = [40, 64, 77, 300]
    w, data = _streams(N, p, nblocks, 4200)
    specs = [torch.from_numpy(pk).cuda() for pk, _ in data]
    scs = [torch.from_numpy(sc).cuda() for _, sc in data]
    eager = ipfb.BatchedPlan(N, p, w, nblocks, ipfb.F32)
    eager.use_graph(False)
    ref = [t.cpu().numpy() for t in ipfb.wiener_batched(eager, specs, scs, 0.1)]
    bp = ipfb.BatchedPlan(N, p, w, nblocks, ipfb.F32)
    outs = [torch.empty(b * N, dtype=torch.float32, device="cuda") for b in nblocks]
    for rep in range(4):
        for o in outs:
            o.fill_(float("nan"))  # eager work between replays
        torch.cuda.synchronize()
        ipfb.wiener_batched(bp, specs, scs, 0.1, x_outs=outs)
        torch.cuda.synchronize()
        for r, o in zip(ref, outs):
            assert np.array_equal(r, o.cpu().numpy()), rep
    # new output buffers: the graph is captured again for the new pointers
    outs2 = ipfb.wiener_batched(bp, specs, scs, 0.1)
    torch.cuda.synchronize()
    for r, o in zip(ref, outs2):
        assert np.array_equal(r, o.cpu().numpy())


def test_batched_rejects_bad_plans():
    w = O.window_sinc_hamming(4, 64)
    with pytest.raises(ipfb.IpfbError):
        ipfb.BatchedPlan(64, 4, w, [12, 40000], ipfb.F32)
    with pytest.raises(ipfb.IpfbError):
        ipfb.BatchedPlan(64, 4, w, [1], ipfb.F32)
