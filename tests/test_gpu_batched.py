"""GPU tests of the batched form: streams of uneven (arbitrary) nblock in one
call, replayed from one captured HIP graph; every stream against the FP64
oracle. Two column stages: the recursive one over all streams at once (the
default for 4 taps and phi > 0) and the per-stream FFT path with Bluestein
column DFTs for lengths that are not powers of two (COLS_FFT; its shapes and
autotuner are tested with it forced)."""
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


@pytest.mark.parametrize("method", [ipfb.COLS_AUTO, ipfb.COLS_FFT])
@pytest.mark.parametrize("prec,tol", [(ipfb.F64, 1e-11), (ipfb.F32, 1e-5)])
def test_batched_small_uneven(prec, tol, method):
    N, p = 64, 4
    nblocks = [12, 37, 64, 100, 129, 5, 3, 2, 16, 1031]
    print(f"case batched small prec={prec} method={method}", flush=True)
    w, data = _streams(N, p, nblocks, 4000)
    bp = ipfb.BatchedPlan(N, p, w, nblocks, prec)
    bp.set_column_method(method)
    specs = [torch.from_numpy(pk).cuda() for pk, _ in data]
    scs = [torch.from_numpy(sc).cuda() for _, sc in data]
    for phi in (0.1, 0.0):
        outs = ipfb.wiener_batched(bp, specs, scs, phi)
        torch.cuda.synchronize()
        for (pk, sc), b, xo in zip(data, nblocks, outs):
            ref = O.ipfb_wiener(pk, sc, w, N, p, phi)
            assert _rel(xo.cpu().numpy().astype(np.float64), ref) < (tol if phi > 0 else 50 * tol), (b, phi)


@pytest.mark.parametrize("prec,tol", [(ipfb.F64, 1e-11), (ipfb.F32, 1e-5)])
def test_batched_ci8_uneven(prec, tol):
    N, p = 64, 4
    nblocks = [12, 64, 129, 5, 1031]
    print(f"case batched ci8 prec={prec}", flush=True)
    w = O.window_sinc_hamming(p, N)
    data = []
    for s_, b in enumerate(nblocks):
        y = O.pfb_forward(I.gaussian_timestream(N * b, 4100 + s_), w, N, p)
        sc = O.channel_scales(y, levels_rms=40.0)
        data.append((O.pack_ci8(*O.quantize(y, sc, qmax=127)), sc))
    bp = ipfb.BatchedPlan(N, p, w, nblocks, prec)
    outs = ipfb.wiener_batched(bp, [torch.from_numpy(pk).cuda() for pk, _ in data],
                               [torch.from_numpy(sc).cuda() for _, sc in data], 0.1)
    torch.cuda.synchronize()
    for (pk, sc), b, xo in zip(data, nblocks, outs):
        ref = O.ipfb_wiener_ci8(pk, sc, w, N, p, 0.1)
        assert _rel(xo.cpu().numpy().astype(np.float64), ref) < tol, b


@pytest.mark.parametrize("method", [ipfb.COLS_AUTO, ipfb.COLS_FFT])
def test_batched_production_lengths_fp32(method):
    # production frame length with Bluestein lengths up to M = 65536 (FFT),
    # up to 257 segments of a stream (recursive)
    N, p = 4096, 4
    nblocks = [1031, 3000, 16385, 2048]
    print(f"case batched production lengths method={method}", flush=True)
    w, data = _streams(N, p, nblocks, 4100)
    bp = ipfb.BatchedPlan(N, p, w, nblocks, ipfb.F32)
    bp.set_column_method(method)
    outs = ipfb.wiener_batched(bp, [torch.from_numpy(pk).cuda() for pk, _ in data],
                               [torch.from_numpy(sc).cuda() for _, sc in data], 0.1)
    torch.cuda.synchronize()
    for (pk, sc), b, xo in zip(data, nblocks, outs):
        ref = O.ipfb_wiener(pk, sc, w, N, p, 0.1)
        err = _rel(xo.cpu().numpy().astype(np.float64), ref)
        print(f"b={b}: rel RMS {err:.2e}")
        assert err < 1e-5


@pytest.mark.parametrize("method", [ipfb.COLS_AUTO, ipfb.COLS_FFT])
def test_batched_graph_replays_match_eager(method):
    N, p = 128, 4
    nblocks = [40, 64, 77, 300]
    w, data = _streams(N, p, nblocks, 4200)
    specs = [torch.from_numpy(pk).cuda() for pk, _ in data]
    scs = [torch.from_numpy(sc).cuda() for _, sc in data]
    eager = ipfb.BatchedPlan(N, p, w, nblocks, ipfb.F32)
    eager.use_graph(False)
    eager.set_column_method(method)
    ref = [t.cpu().numpy() for t in ipfb.wiener_batched(eager, specs, scs, 0.1)]
    bp = ipfb.BatchedPlan(N, p, w, nblocks, ipfb.F32)
    bp.set_column_method(method)
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


def _check_streams(bp, data, nblocks, w, N, p, tol, what):
    outs = ipfb.wiener_batched(bp, [torch.from_numpy(pk).cuda() for pk, _ in data],
                               [torch.from_numpy(sc).cuda() for _, sc in data], 0.1)
    torch.cuda.synchronize()
    for (pk, sc), b, xo in zip(data, nblocks, outs):
        ref = O.ipfb_wiener(pk, sc, w, N, p, 0.1)
        err = _rel(xo.cpu().numpy().astype(np.float64), ref)
        assert err < tol, (what, b, err)


@pytest.mark.parametrize("prec,tol,p", [(ipfb.F64, 1e-11, 4), (ipfb.F32, 1e-5, 4), (ipfb.F64, 1e-11, 5)])
def test_batched_every_shape_matches_oracle(prec, tol, p):
    # every split, both non-default tile widths and ragged launch groups; 5
    # taps take the generic gain code of every path
    N = 64
    nblocks = [37, 300, 1031]  # convolution lengths 2^7, 2^10, 2^12
    print(f"case batched shapes prec={prec} ntap={p}", flush=True)
    w, data = _streams(N, p, nblocks, 4300)
    bp = ipfb.BatchedPlan(N, p, w, nblocks, prec)
    bp.use_graph(False)
    bp.set_column_method(ipfb.COLS_FFT)
    assert bp.conv_lengths() == [7, 10, 12]
    for m in bp.conv_lengths():
        d = (m + 1) // 2
        assert bp.get_shape(m) == (d, 16, 16, 0, 1, 0)
        shapes = []
        for fuse in (1, 0):
            shapes += [(l1, 16, 16, 0, fuse, 0) for l1 in range(max(1, m - 8), min(8, m - 1) + 1)]
            shapes += [(d, 8, 16, 0, fuse, 0), (d, 32, 16, 0, fuse, 0), (d, 16, 8, 0, fuse, 0),
                       (d, 16, 32, 0, fuse, 0), (d, 8, 32, 5, fuse, 0), (d, 32, 8, 7, fuse, 0)]
        # natural layout: every split, one tile per launch group (ragged: 32 pairs = 2 or 4 tiles)
        shapes += [(l1, 16, 16, 0, 1, 1) for l1 in range(max(1, m - 8), min(8, m - 1) + 1)]
        shapes += [(d, 16, 16, 1, 1, 1)]
        for sh in shapes:
            bp.set_shape(m, sh)
            assert bp.get_shape(m) == sh
            _check_streams(bp, data, nblocks, w, N, p, tol, (m, sh))
        bp.set_shape(m, (d, 16, 16, 0, 1, 0))


def test_batched_shape_rejects_invalid():
    N, p = 64, 4
    w = O.window_sinc_hamming(p, N)
    bp = ipfb.BatchedPlan(N, p, w, [300], ipfb.F32)
    for bad in [(9, 16, 16, 0, 1, 0), (1, 16, 16, 0, 1, 0), (5, 12, 16, 0, 1, 0), (5, 16, 64, 0, 1, 0),
                (5, 16, 16, -1, 1, 0), (5, 16, 16, 0, 2, 0), (5, 16, 16, 0, 1, 2)]:
        with pytest.raises(ipfb.IpfbError):
            bp.set_shape(10, bad)
    with pytest.raises(ipfb.IpfbError):
        bp.get_shape(11)  # no stream of that length
    assert bp.get_shape(10) == (5, 16, 16, 0, 1, 0)


def test_batched_autotuner_and_cache(tmp_path, monkeypatch):
    import json
    N, p = 256, 4
    nblocks = [300, 1031, 777]
    print("case batched autotuner", flush=True)
    w, data = _streams(N, p, nblocks, 4400)
    cache = tmp_path / "tune.json"
    bp = ipfb.BatchedPlan(N, p, w, nblocks, ipfb.F32)
    bp.set_column_method(ipfb.COLS_FFT)
    tuned = bp.tune(str(cache))
    assert set(tuned) == {10, 11, 12}
    doc = json.loads(cache.read_text())
    keys = sorted(doc["entries"])
    assert len(keys) == 3 and all("|f32|N256|T4|m" in k for k in keys)
    for k, e in doc["entries"].items():
        m = int(k.rsplit("|m", 1)[1])
        assert (e["l1"], e["mb"], e["kb"], e["pchunk"], e["fuse"], e["nat"]) == tuned[m]
        assert e["us"] > 0
    _check_streams(bp, data, nblocks, w, N, p, 1e-5, "tuned")
    # a plan created with the cache in the environment installs the same shapes
    monkeypatch.setenv("IPFB_TUNE_CACHE", str(cache))
    bp2 = ipfb.BatchedPlan(N, p, w, nblocks, ipfb.F32)
    bp2.set_column_method(ipfb.COLS_FFT)
    assert {m: bp2.get_shape(m) for m in bp2.conv_lengths()} == tuned
    _check_streams(bp2, data, nblocks, w, N, p, 1e-5, "from cache")
    # a hand-edited entry (other spacing, extra field) is read as well
    key = [k for k in keys if k.endswith("|m11")][0]
    cache.write_text('{ "entries" : { "%s" : { "note": "manual", "l1" : 4, "mb": 32, "kb": 8, "pchunk": 3, '
                     '"us": 1.0 } }, "version": 1 }' % key)
    bp3 = ipfb.BatchedPlan(N, p, w, nblocks, ipfb.F32)
    bp3.set_column_method(ipfb.COLS_FFT)
    assert bp3.get_shape(11) == (4, 32, 8, 3, 1, 0)  # no "fuse" or "nat" field: fused, transposed
    assert bp3.get_shape(10) == (5, 16, 16, 0, 1, 0)  # no entry: default
    _check_streams(bp3, data, nblocks, w, N, p, 1e-5, "hand-edited")
    # tune with the env cache: the entry found is kept, the missing ones are timed and merged
    bp3.tune()
    doc = json.loads(cache.read_text())
    assert len(doc["entries"]) == 3
    assert doc["entries"][key]["l1"] == 4


@pytest.mark.parametrize("method", [ipfb.COLS_AUTO, ipfb.COLS_FFT])
def test_batched_full_workload_sampled_columns(method):
    # the benchmarked configuration itself: 256 streams, nblock ~ U[1024, 32768]
    # (seed 4), lblock 4096, 4-bit, one graph launch with autotuned shapes;
    # sampled columns of four streams (the shortest, the longest, a prime
    # length, one more) against the oracle, whose column inverse is exact per
    # column (sub-filter paths are independent)
    import math
    N, p, phi = 4096, 4, 0.1
    nbl = [int(b) for b in I.batched_nblocks(256, 1024, 32768, 4)]
    print(f"case batched full workload: {sum(nbl) * N} samples, method={method}", flush=True)
    w = O.window_sinc_hamming(p, N)
    specs, scales, outs = [], [], []
    for s_, b in enumerate(nbl):
        g = torch.Generator(device="cuda")
        g.manual_seed(4000 + s_)
        x = torch.randn(b * N, generator=g, device="cuda", dtype=torch.float32)
        plan = ipfb.Plan(N, p, w, b, ipfb.F32)
        pk, sc = ipfb.quantize_c4(plan, ipfb.pfb_forward(plan, x), 2.5)
        specs.append(pk)
        scales.append(sc)
        outs.append(torch.empty(b * N, dtype=torch.float32, device="cuda"))
        del x, plan
    bp = ipfb.BatchedPlan(N, p, w, nbl, ipfb.F32)
    bp.set_column_method(method)
    if method == ipfb.COLS_FFT:
        shapes = bp.tune()
        print(f"tuned shapes {shapes}", flush=True)
    ipfb.wiener_batched(bp, specs, scales, phi, x_outs=outs)
    torch.cuda.synchronize()
    isprime = lambda v: v > 1 and all(v % q for q in range(2, int(math.isqrt(v)) + 1))
    pick = [int(np.argmin(nbl)), int(np.argmax(nbl)), next(i for i, b in enumerate(nbl) if isprime(b)), 17]
    cols = np.array([0, 1, 1023, 2047, 2048, 2049, 4094, 4095])
    wsub = w.reshape(p, N)[:, cols].reshape(-1)
    for s_ in pick:
        b = nbl[s_]
        qr, qi = O.unpack_c4(specs[s_].cpu().numpy())
        d = O.row_inverse(O.dequantize(qr, qi, scales[s_].cpu().numpy()), N)
        ref = O.column_inverse(d[:, cols], wsub, len(cols), p, phi)
        got = outs[s_].view(b, N)[:, torch.from_numpy(cols).cuda()].cpu().numpy().astype(np.float64)
        err = _rel(got, ref)
        print(f"stream {s_} b={b}: sampled columns rel RMS {err:.2e}", flush=True)
        assert err < 1e-5
    if method == ipfb.COLS_AUTO:
        # every column of 16 streams (the four above and 12 drawn at random)
        # against the FFT form of the same inverse, an independent algorithm
        # (Bluestein's identity for the lengths that are not powers of two)
        rng = np.random.default_rng(7)
        more = [int(v) for v in rng.choice(len(nbl), 16, replace=False) if int(v) not in pick][:12]
        for s_ in pick + more:
            plan = ipfb.Plan(N, p, w, nbl[s_], ipfb.F32)
            plan.set_column_method(ipfb.COLS_FFT)
            ref2 = ipfb.ipfb_wiener(plan, specs[s_], scales[s_], phi)
            torch.cuda.synchronize()
            err = float(torch.linalg.vector_norm(outs[s_] - ref2) / torch.linalg.vector_norm(ref2))
            print(f"stream {s_} b={nbl[s_]}: every column, recursive vs FFT form rel RMS {err:.2e}", flush=True)
            assert err < 2e-6
            del plan, ref2
    del outs, specs, scales, bp
    torch.cuda.empty_cache()


@pytest.mark.parametrize("method", [ipfb.COLS_AUTO, ipfb.COLS_RECURSIVE, ipfb.COLS_FFT])
@pytest.mark.parametrize("prec,tol", [(ipfb.F64, 1e-11), (ipfb.F32, 1e-5)])
def test_batched_single_stream(prec, tol, method):
    # a batched plan of exactly one stream: the multi-stream recursive launches
    # read its table entry (regression: they once took the unused by-value
    # stream, a zero-length one, for a table of one entry)
    N, p, b = 64, 4, 100
    print(f"case batched one stream prec={prec} method={method}", flush=True)
    w, data = _streams(N, p, [b], 4300)
    bp = ipfb.BatchedPlan(N, p, w, [b], prec)
    bp.set_column_method(method)
    (pk, sc), = data
    for phi in (0.1, 0.3):
        out, = ipfb.wiener_batched(bp, [torch.from_numpy(pk).cuda()], [torch.from_numpy(sc).cuda()], phi)
        torch.cuda.synchronize()
        assert _rel(out.cpu().numpy().astype(np.float64), O.ipfb_wiener(pk, sc, w, N, p, phi)) < tol, phi


@pytest.mark.parametrize("prec,tol", [(ipfb.F64, 1e-11), (ipfb.F32, 1e-5)])
def test_single_plan_fft_form_for_any_nblock(prec, tol):
    # COLS_FFT on a plan whose nblock is not a power of two: the FFT form by
    # Bluestein's identity (through a one-stream batched plan), phi > 0
    N, p, b = 256, 4, 1031
    print(f"case single plan FFT form nblock={b} prec={prec}", flush=True)
    w, data = _streams(N, p, [b], 4400)
    (pk, sc), = data
    plan = ipfb.Plan(N, p, w, b, prec)
    plan.set_column_method(ipfb.COLS_FFT)
    for phi in (0.1, 0.0):
        out = ipfb.ipfb_wiener(plan, torch.from_numpy(pk).cuda(), torch.from_numpy(sc).cuda(), phi)
        torch.cuda.synchronize()
        ref = O.ipfb_wiener(pk, sc, w, N, p, phi)
        assert _rel(out.cpu().numpy().astype(np.float64), ref) < (tol if phi > 0 else 50 * tol), phi


def test_batched_recursive_equals_single_stream_plans():
    # the multi-stream launches give each stream what its own plan gives
    N, p = 256, 4
    nblocks = [3, 64, 65, 1000, 4097]
    print("case batched recursive vs single plans", flush=True)
    w, data = _streams(N, p, nblocks, 4500)
    specs = [torch.from_numpy(pk).cuda() for pk, _ in data]
    scs = [torch.from_numpy(sc).cuda() for _, sc in data]
    bp = ipfb.BatchedPlan(N, p, w, nblocks, ipfb.F64)
    bp.set_column_method(ipfb.COLS_RECURSIVE)
    for phi in (0.1, 0.3):
        outs = ipfb.wiener_batched(bp, specs, scs, phi)
        for b, sp, sc, o in zip(nblocks, specs, scs, outs):
            plan = ipfb.Plan(N, p, w, b, ipfb.F64)
            plan.set_column_method(ipfb.COLS_RECURSIVE)
            single = ipfb.ipfb_wiener(plan, sp, sc, phi)
            torch.cuda.synchronize()
            assert _rel(o.cpu().numpy(), single.cpu().numpy()) < 1e-14, (b, phi)
