#!/usr/bin/env python3
"""Throughput of the circulant inverse PFB + up-channelization on one MI355X.

One step = the whole hot path over one batch of synthetic input already
resident in HBM: dequantise the 4-bit spectra, row inverse FFTs, column
Wiener decorrelation (inverse PFB), then the forward PFB at a 64x longer frame
(up-channelization) and its autospectrum.

Workload (production size): white Gaussian noise (sigma = 1) plus 5 narrow
tones (amplitude 0.1), lblock = 4096, ntap = 4, sinc x Hamming window,
nblock = 16384 (2^26 samples), channelised by the library's forward PFB in
FP64 and quantised to 4 bits per component (per-channel RMS = 2.5 levels);
Wiener phi = 0.1; up-channelize x64: lblock' = 262144, ntap' = 4,
nblock' = 256. The headline is the FP32 form; the FP64 form is timed beside it.

Prints one JSON line. Only the `cpu_baseline` leg touches the CPU oracle.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "reconstructed samples/s + HBM GB/s, FP32 vs FP64 form at ≤1e-5 rel RMS"
HBM_PEAK_GBPS = 8000.0

# Bytes per launch, by kernel (FP32 unless esz = 8), in two senses:
#  compulsory share: the kernel's part of the step's compulsory traffic
#    (step_bytes), each compulsory byte assigned to the kernel that moves it
#    to or from HBM, intermediate round trips priced at zero:
#      ipfb_rows            packed input + scales in, d written
#      first column kernel  d read (the three-pass FFT stage: pass A; the
#                           recursive stage: pass 1)
#      last column kernel   xhat written (pass C; recursive pass 2; the
#                           one-pass FFT stage does both)
#      pfb_fwd_long_p1      xhat read + the fine window
#      pfb_fwd_long_p2      fine spectra written
#  moved: what the kernel reads and writes by its design (the three FFT
#    passes each read and rewrite the frames; recursive pass 2 reads d again
#    and the segment states; the long-frame passes move the per-spectrum
#    intermediate between them).
# The roofline object prices the dominant kernel at its compulsory share.
COLUMN_FIRST = ("ipfb_cols_fwd", "ipfb_cols_rec_pass1")
COLUMN_LAST = ("ipfb_cols_inv", "ipfb_cols_rec_pass2")


def progress(msg):
    """One line per finished section on stderr (the JSON line stays alone on stdout)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def kernel_bytes(name, N, b, Nf, bf, esz, kind="compulsory", one_pass=False):
    S = N * b
    K = Nf // 2 + 1
    inter = bf * (Nf // 2) * 2 * esz  # the long-frame passes' intermediate
    nseg = (b + 63) // 64
    states = nseg * N * 6 * esz  # recursive stage: 3 + 3 states per column and segment
    if name == "ipfb_rows":
        return b * (N // 2 + 1) * 1 + (N // 2 + 1) * 4 + S * esz
    if name == "ipfb_cols_gain":
        if kind == "moved" or one_pass:
            return 2 * S * esz
        return 0
    if name in COLUMN_FIRST:
        return S * esz + (states if kind == "moved" and name == "ipfb_cols_rec_pass1" else 0) + \
            (S * esz if kind == "moved" and name == "ipfb_cols_fwd" else 0)
    if name in COLUMN_LAST:
        if kind == "moved":
            return 2 * S * esz + (states if name == "ipfb_cols_rec_pass2" else 0)
        return S * esz
    if name == "ipfb_cols_rec_carry":
        return 2 * states if kind == "moved" else 0
    if name == "pfb_fwd_long_p1":
        return S * esz + 4 * Nf * esz + (inter if kind == "moved" else 0)
    if name == "pfb_fwd_long_p2":
        return bf * K * 2 * esz + (inter if kind == "moved" else 0)
    return 0


def step_bytes(N, b, Nf, bf, esz):
    """Compulsory HBM bytes of one step: packed input + scales, d written and
    read once, xhat written, xhat read by the fine PFB, fine window, fine
    spectra written."""
    S = N * b
    return (b * (N // 2 + 1) + 4 * (N // 2 + 1) + 2 * S * esz + S * esz + S * esz + 4 * Nf * esz
            + bf * (Nf // 2 + 1) * 2 * esz)


def source_digest():
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2608_23441_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".hpp")):
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(kernel):
    """HBM bytes per launch from committed rocprofv3 counter runs, valid only if
    the kernel sources are unchanged since the counters were taken."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        t = json.load(open(p))
    except Exception:
        return None
    if t.get("source_digest") != source_digest():
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else k.get("hbm_bytes_per_launch")


def make_inputs(torch, ipfb, inputs, N, p, b, seed, ntones, tone_seed, amp, levels):
    """Synthetic 4-bit spectra made on the GPU by the library's own FP64
    forward PFB and quantiser (input synthesis, not timed)."""
    x = inputs.timestream_with_tones(N * b, seed, ntones, tone_seed, amp)
    w = ipfb.window_sinc_hamming(p, N)
    plan64 = ipfb.Plan(N, p, w, b, ipfb.F64)
    xd = torch.from_numpy(x).cuda()
    y = ipfb.pfb_forward(plan64, xd)
    packed, scales = ipfb.quantize_c4(plan64, y, levels)
    torch.cuda.synchronize()
    del xd, y
    plan64.close()
    return x, w, packed, scales


def time_steps(torch, step, steps, warmup):
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def copy_peak_GBps(torch, nbytes=1 << 30):
    """A plain device copy (read + write of nbytes each), the practical HBM
    ceiling the roofline fraction is also stated against."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / 10
    del src, dst
    return 2 * nbytes / sec / 1e9


def small_config(torch, ipfb, inputs):
    """The small configuration (N = 2048, p = 4, b = 128, phi = 0.1, x8
    up-channelize): latency-bound, so its time per step (median of 20 after 3
    warm-ups, each step synchronised) is what it reports, per precision."""
    N, p, b, u, phi = 2048, 4, 128, 8, 0.1
    Nf = N * u
    _, w, packed, scales = make_inputs(torch, ipfb, inputs, N, p, b, 1, 0, 0, 0.0, 2.5)
    wf = ipfb.window_sinc_hamming(4, Nf)
    out = {"config": {"lblock": N, "ntap": p, "nblock": b, "phi": phi, "lblock_fine": Nf,
                      "nblock_fine": (N * b) // Nf}}
    for tag, prec in (("f64", ipfb.F64), ("f32", ipfb.F32)):
        coarse = ipfb.Plan(N, p, w, b, prec)
        fine = ipfb.Plan(Nf, 4, wf, (N * b) // Nf, prec)
        xh = torch.empty(N * b, dtype=coarse.real_dtype, device="cuda")
        Y = torch.empty(((N * b) // Nf, Nf // 2 + 1), dtype=fine.complex_dtype, device="cuda")
        A = torch.empty(Nf // 2 + 1, dtype=torch.float64, device="cuda")
        times = []
        for i in range(23):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ipfb.ipfb_wiener(coarse, packed, scales, phi, x_out=xh)
            ipfb.upchannelize(fine, xh, Y, A)
            torch.cuda.synchronize()
            if i >= 3:
                times.append(time.perf_counter() - t0)
        times.sort()
        out[tag] = {"us_per_step_median": 1e6 * times[len(times) // 2], "us_per_step_min": 1e6 * times[0]}
        del coarse, fine
    return out


def cpu_oracle_step(O, packed, s, w, wf, N, p, Nf, phi, pool, nchunks):
    """The oracle's steps on chunks: dequantise + row inverse over blocks of
    frames, the column inverse over blocks of sub-filter paths (each its own
    window slice), the fine PFB over blocks of fine frames (each with the
    next three frames appended, wrapping at the end), the autospectrum. The
    chunks run on `pool` (numpy's FFT releases the interpreter lock)."""
    import numpy as np
    b = packed.shape[0]

    def rows(r):
        r0, r1 = r
        qr, qi = O.unpack_c4(packed[r0:r1])
        return O.row_inverse(O.dequantize(qr, qi, s), N)

    rb = [(i * b // nchunks, (i + 1) * b // nchunks) for i in range(nchunks)]
    d = np.concatenate(list(pool.map(rows, rb)), axis=0)
    H = w.reshape(p, N)
    cb = [(i * N // nchunks, (i + 1) * N // nchunks) for i in range(nchunks)]

    def cols(c):
        c0, c1 = c
        return O.column_inverse(np.ascontiguousarray(d[:, c0:c1]), H[:, c0:c1].reshape(-1), c1 - c0, p, phi)

    xh = np.concatenate(list(pool.map(cols, cb)), axis=1).reshape(-1)
    bf = xh.size // Nf
    X = xh.reshape(bf, Nf)
    fb = [(i * bf // nchunks, (i + 1) * bf // nchunks) for i in range(nchunks) if (i + 1) * bf // nchunks > i * bf // nchunks]

    def fine(f):
        f0, f1 = f
        seg = X[[(j % bf) for j in range(f0, f1 + 3)]].reshape(-1)
        return O.pfb_forward(seg, wf, Nf, 4, circular=False)

    Y = np.concatenate(list(pool.map(fine, fb)), axis=0)
    return O.autospectrum(Y)


def cpu_baseline(N, p, Nf, phi, frames, seed):
    """The FP64 numpy oracle on a bounded sample of the same workload: the
    same steps (dequantise, row inverse, column Wiener inverse, x64
    up-channelize with autospectrum) over `frames` frames, on the host's
    cores (at most 16 threads, the GPU's share of its host) and on one."""
    from concurrent.futures import ThreadPoolExecutor

    from oracle import ipfb_oracle as O
    from paper_2608_23441_amd import inputs as I

    S = N * frames
    x = I.timestream_with_tones(S, seed, 5, 102, 0.1)
    w = O.window_sinc_hamming(p, N)
    y = O.pfb_forward(x, w, N, p)
    s = O.channel_scales(y, 2.5)
    qr, qi = O.quantize(y, s)
    packed = O.pack_c4(qr, qi)
    del x, y, qr, qi
    wf = O.window_sinc_hamming(4, Nf)
    threads = max(1, min(16, int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)))
    out = {}
    for nt in (threads, 1):
        with ThreadPoolExecutor(nt) as pool:
            times = []
            for rep in range(2 if nt > 1 else 1):  # the threaded run: one warm-up, then timed
                t0 = time.perf_counter()
                cpu_oracle_step(O, packed, s, w, wf, N, p, Nf, phi, pool, 4 * nt)
                times.append(time.perf_counter() - t0)
            out[nt] = times[-1]
    dt = out[threads]
    return {"value": S / dt, "unit": "samples/s", "cores": threads, "kind": "oracle",
            "sample": f"lblock={N}, ntap={p}, nblock={frames} ({S} samples, "
                      f"{S / (N * 16384):.3f} of the workload), phi={phi}, x{Nf // N} up-channelize "
                      f"(lblock'={Nf}, nblock'={S // Nf}) with autospectrum; FP64 numpy oracle in chunks of "
                      f"frames and paths on {threads} threads ({os.cpu_count()} visible host cores), "
                      f"{dt:.1f} s; one thread: {out[1]:.1f} s",
            "seconds": dt, "single_thread": {"value": S / out[1], "seconds": out[1], "cores": 1}}


def ml_form(torch, ipfb, inputs):
    """Maximum-likelihood CG form: lblock = 2048, ntap = 4, nblock = 8192,
    4-bit spectra, saved samples on a random 10% mask (prior = the true
    timestream), Wiener x0 and preconditioner (phi = 0.1), 100 iterations,
    FP32 vectors with FP64 dots. Samples/s = S / (setup + 100 iterations)."""
    N, p, b, iters = 2048, 4, 8192, 100
    S = N * b
    x, w, packed, scales = make_inputs(torch, ipfb, inputs, N, p, b, 5, 0, 0, 0.0, 2.5)
    mask = ipfb.mask_pack(torch.from_numpy(inputs.random_mask(S, 0.1, 505).astype("uint8")).cuda())
    prior = torch.from_numpy(x.astype("float32")).cuda()
    plan = ipfb.Plan(N, p, w, b, ipfb.F32)
    xo = torch.empty(S, dtype=torch.float32, device="cuda")
    ipfb.ml_cg(plan, packed, scales, mask, prior, 1.0, 0.1, 0.1, iters, x_out=xo)  # warm-up, allocates
    torch.cuda.synchronize()
    reps = 3
    ipfb.profile_reset()
    ipfb.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(reps):
        _, norms = ipfb.ml_cg(plan, packed, scales, mask, prior, 1.0, 0.1, 0.1, iters, x_out=xo)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / reps
    ipfb.profile_enable(False)
    it_ms, it_n = ipfb.profile_query("cg_iter")
    ipfb.profile_reset()
    nrm = norms.cpu().numpy()
    # per-iteration compulsory traffic (FP32 vectors): H p (read p and the
    # 1-bit mask, write q) 8.125 B, x/r update (read x, p, r, q; write x, r)
    # 24 B, z = M^-1 r with r.z formed on the way out (read r, write z) 8 B,
    # p update (read z, p; write p) 12 B -> 52.125 B/sample
    it_bytes = 52.125 * S
    it_us = 1e3 * it_ms / max(it_n, 1)
    return {"value": S / sec, "unit": "samples/s", "ms_per_solve": sec * 1e3, "iterations": iters,
            "config": {"lblock": N, "ntap": p, "nblock": b, "mask_fraction": 0.1, "lambda": 1.0, "phi": 0.1},
            "us_per_iteration": it_us, "iteration_hbm_GBps": it_bytes / (it_us * 1e-6) / 1e9,
            "resid_norm_first_last": [float(nrm[0]), float(nrm[-1])]}


def batched_form(torch, ipfb, inputs, nstreams):
    """Batched form: nstreams independent streams, lblock = 4096, ntap = 4,
    nblock ~ U[1024, 32768] (seed 4), stream s signal seed 4000+s, 4-bit
    spectra, Wiener phi = 0.1, FP32; one graph launch per step. Inputs are
    made on the GPU by the library's FP32 forward PFB and quantiser."""
    N, p, phi = 4096, 4, 0.1
    nbl = [int(b) for b in inputs.batched_nblocks(256, 1024, 32768, 4)[:nstreams]]
    w = ipfb.window_sinc_hamming(p, N)
    specs, scales, outs = [], [], []
    for s_, b in enumerate(nbl):
        g = torch.Generator(device="cuda")
        g.manual_seed(4000 + s_)
        x = torch.randn(b * N, generator=g, device="cuda", dtype=torch.float32)
        plan = ipfb.Plan(N, p, w, b, ipfb.F32)
        y = ipfb.pfb_forward(plan, x)
        pk, sc = ipfb.quantize_c4(plan, y, 2.5)
        torch.cuda.synchronize()
        specs.append(pk)
        scales.append(sc)
        outs.append(torch.empty(b * N, dtype=torch.float32, device="cuda"))
        del x, y
        plan.close()
    bp = ipfb.BatchedPlan(N, p, w, nbl, ipfb.F32)
    steps = 3

    def timed():
        ipfb.wiener_batched(bp, specs, scales, phi, x_outs=outs)  # (re)captures the graph
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ipfb.wiener_batched(bp, specs, scales, phi, x_outs=outs)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    # the default: the recursive column stage over every stream at once
    sec = timed()
    # per-kernel times from one step launched directly (events are not
    # recorded inside a replayed graph)
    bp.use_graph(False)
    ipfb.wiener_batched(bp, specs, scales, phi, x_outs=outs)
    torch.cuda.synchronize()
    ipfb.profile_reset()
    ipfb.profile_enable(True)
    ipfb.wiener_batched(bp, specs, scales, phi, x_outs=outs)
    torch.cuda.synchronize()
    ipfb.profile_enable(False)
    bp.use_graph(True)
    per_kernel = {}
    for k in ("batched_rows", "batched_cols_rec_pass1", "batched_cols_rec_carry", "batched_cols_rec_pass2"):
        ms, n = ipfb.profile_query(k)
        if n:
            per_kernel[k] = round(1e3 * ms / n, 1)
    ipfb.profile_reset()
    # beside it: the per-stream FFT path (Bluestein columns), default shapes, then the autotuner's
    bp.set_column_method(ipfb.COLS_FFT)
    default_shapes = {m: bp.get_shape(m) for m in bp.conv_lengths()}
    sec_fft_default = timed()
    # autotuner: shapes from IPFB_TUNE_CACHE when it names a cache holding them, else timed now
    t0 = time.perf_counter()
    shapes = bp.tune()
    tune_s = time.perf_counter() - t0
    sec_fft = timed()
    S = sum(b * N for b in nbl)
    npow2 = sum(1 for b in nbl if b & (b - 1) == 0)
    # compulsory traffic of the inverse (packed input, one d round trip, xhat out): 12.5 B/sample
    alg = sum(b * (N // 2 + 1) + 4 * (N // 2 + 1) for b in nbl) + 12 * S
    return {"value": S / sec, "unit": "samples/s", "s_per_step": sec, "steps": steps, "streams": len(nbl),
            "samples": S, "power_of_two_streams": npow2, "graph": True, "column_stage": "recursive",
            "per_kernel_ms": per_kernel,
            "hbm_GBps": alg / sec / 1e9, "hbm_roofline_frac": alg / sec / 1e9 / HBM_PEAK_GBPS,
            "fft_path": {"value": S / sec_fft, "s_per_step": sec_fft, "s_per_step_default_shapes": sec_fft_default,
                         "tune_s": tune_s,
                         "shapes": {f"2^{m}": {"default": list(default_shapes[m]), "tuned": list(shapes[m])}
                                    for m in shapes},
                         "shape_fields": ["l1", "mb", "kb", "pchunk", "fuse", "nat"]},
            "config": {"lblock": N, "ntap": p, "nblock": "U[1024, 32768], seed 4", "phi": phi,
                       "dtype": "f32"}}


def streaming_form(torch, ipfb, nframes=65536, chunk=8192, halo=256):
    """Linear-boundary streaming inverse: one stream of nframes = 65536 frames
    (lblock 4096, ntap 4: 2^28 samples), white noise seed 6, the linear PFB's
    nframes - 3 spectra (the first spectra of the circular PFB over the same
    frames), 4-bit; windows of 8192 frames (134 MB: one window stays in the
    256 MB last-level cache through its column passes) with a 256-frame halo,
    phi = 0.1, FP32. Inputs made on the GPU by the library's forward PFB and
    quantiser."""
    N, p, phi = 4096, 4, 0.1
    w = ipfb.window_sinc_hamming(p, N)
    g = torch.Generator(device="cuda")
    g.manual_seed(6)
    x = torch.randn(nframes * N, generator=g, device="cuda", dtype=torch.float32)
    plan = ipfb.Plan(N, p, w, nframes, ipfb.F32)
    y = ipfb.pfb_forward(plan, x)
    pk, sc = ipfb.quantize_c4(plan, y, 2.5)
    nspec = nframes - (p - 1)
    pk = pk[:nspec].contiguous()
    torch.cuda.synchronize()
    del x, y, plan
    sp = ipfb.StreamPlan(N, p, w, chunk, halo, ipfb.F32)
    out = torch.empty(nframes * N, dtype=torch.float32, device="cuda")
    steps = 5
    for _ in range(2):
        ipfb.wiener_stream(sp, pk, sc, phi, x_out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ipfb.wiener_stream(sp, pk, sc, phi, x_out=out)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    S = nframes * N
    L = chunk - (p - 1) - 2 * halo
    nwin = (nframes + L - 1) // L
    # compulsory traffic as for the block inverse: packed in, one d round trip, x out
    alg = nspec * (N // 2 + 1) + 4 * (N // 2 + 1) + 12 * S
    return {"value": S / sec, "unit": "samples/s", "s_per_step": sec, "steps": steps, "samples": S,
            "windows": nwin, "window_frames_per_output_frame": nwin * chunk / nframes,
            "hbm_GBps": alg / sec / 1e9, "hbm_roofline_frac": alg / sec / 1e9 / HBM_PEAK_GBPS,
            "config": {"lblock": N, "ntap": p, "nframes": nframes, "nspec": nspec, "chunk": chunk,
                       "halo": halo, "phi": phi, "dtype": "f32", "boundary": "linear"}}


def pipelined_form(torch, ipfb, packed, scales, w, wf, N, p, b, Nf, bf, phi, steps=40, warmup=4):
    """The headline step with two batches in flight: consecutive steps
    alternate between two HIP streams, each with its own plans and buffers
    (the same inputs, copied), so one step's up-channelization overlaps the
    next step's inverse. Reported beside the one-stream headline: every step
    still does the whole path over one batch."""
    ctx = []
    for k in range(2):
        s = torch.cuda.Stream()
        ctx.append((ipfb.Plan(N, p, w, b, ipfb.F32), ipfb.Plan(Nf, 4, wf, bf, ipfb.F32),
                    torch.empty(N * b, dtype=torch.float32, device="cuda"),
                    torch.empty((bf, Nf // 2 + 1), dtype=torch.complex64, device="cuda"),
                    torch.empty(Nf // 2 + 1, dtype=torch.float64, device="cuda"), s.cuda_stream,
                    packed if k == 0 else packed.clone(), scales if k == 0 else scales.clone()))
    torch.cuda.synchronize()

    def step(c):
        plan, fine, xo, Y, A, st, pk, sc = c
        ipfb.ipfb_wiener(plan, pk, sc, phi, x_out=xo, stream=st)
        ipfb.upchannelize(fine, xo, y_fine=Y, autospec=A, stream=st)

    for k in range(warmup):
        step(ctx[k & 1])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        step(ctx[k & 1])
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    for c in ctx:
        c[0].close()
        c[1].close()
    return {"value": N * b / sec, "unit": "samples/s", "ms_per_step": sec * 1e3, "steps": steps, "streams": 2}


def alt_solvers(torch, ipfb, taps=(4, 8, 16), ltaps=(51, 101, 201), N=4096, b=16384, phi=0.1):
    """Appendix C's cost comparison, measured: the circulant Wiener inverse
    beside the Tikhonov solve of the linear sub-problems (banded Cholesky,
    O(b p^2) per path) and FIR decorrelation with kernels truncated to L lags
    (O(b L) per path), FP32, phi = 0.1, at p = 4, 8, 16 taps. Input: white
    noise (torch seed 8), 2^26 samples (lblock 4096, nblock 16384), channelised
    by the library's FP64 forward PFB and quantised to 4 bits (RMS 2.5 levels);
    the Tikhonov solver takes the first nblock - p + 1 spectra (the ones that
    do not wrap: a linear PFB's). Each solver's error is its relative RMS
    difference from the original timestream (Tikhonov: over all frames, its
    ends included); the FIR forms also against the circulant result."""
    out = {"config": {"lblock": N, "nblock": b, "samples": N * b, "phi": phi, "dtype": "f32", "levels_rms": 2.5}}
    g = torch.Generator(device="cuda")
    g.manual_seed(8)
    x = torch.randn(N * b, generator=g, device="cuda", dtype=torch.float64)

    def rel(a, ref):
        return float(torch.linalg.vector_norm(a.double() - ref) / torch.linalg.vector_norm(ref))

    for p in taps:
        w = ipfb.window_sinc_hamming(p, N)
        plan64 = ipfb.Plan(N, p, w, b, ipfb.F64)
        pk, sc = ipfb.quantize_c4(plan64, ipfb.pfb_forward(plan64, x), 2.5)
        plan64.close()
        plan = ipfb.Plan(N, p, w, b, ipfb.F32)
        xo = torch.empty(N * b, dtype=torch.float32, device="cuda")
        r = {}
        sec = time_steps(torch, lambda: ipfb.ipfb_wiener(plan, pk, sc, phi, x_out=xo), 10, 2)
        xc = xo.clone()
        r["circulant"] = {"s_per_call": sec, "samples_per_s": N * b / sec, "rel_err": rel(xc, x)}
        pl = pk[:b - p + 1].contiguous()
        sec = time_steps(torch, lambda: ipfb.tikhonov(plan, pl, sc, phi, x_out=xo), 3, 1)
        r["tikhonov"] = {"s_per_call": sec, "samples_per_s": N * b / sec, "rel_err": rel(xo, x)}
        for L in ltaps:
            ipfb.fir(plan, pk, sc, phi, L, x_out=xo)  # makes the kernels (not timed)
            sec = time_steps(torch, lambda: ipfb.fir(plan, pk, sc, phi, L, x_out=xo), 10, 2)
            r[f"fir_L{L}"] = {"s_per_call": sec, "samples_per_s": N * b / sec, "rel_err": rel(xo, x),
                              "rel_diff_vs_circulant": rel(xo, xc.double())}
        out[f"p{p}"] = r
        del pk, sc, pl, xo, xc
        plan.close()
    return out


def structured_sweep(torch, ipfb, betas=(0.01, 0.03, 0.05, 0.10), iters=25):
    """Section 4.3's experiment on synthetic data at the paper's size: 2^27
    samples of white noise (torch seed 7) through a 2048-channel 4-tap PFB
    (FP32 form, 65536 frames), 4-bit at the 0.353 sigma spacing; inverted with
    the Wiener filter (phi = 0.1) and by 25 PCG iterations from it with every
    4th sample of the L paths around N/2 saved (beta = L/(4N)); delta(f) of the
    x64 up-channelized autospectrum measured on the GPU. Each delta(f) is
    summarised by its maximum over all fine channels (with where it falls),
    its 99th percentile, and the profile folded over the original channels
    (mean over channels at each of the 64 fine positions): its values at the
    channel edge and centre are what the paper's one-channel plot shows. The
    naive inverse (phi = 0) is not run at this length (the recursive column
    stage needs phi >= 1e-3; the FFT stage takes at most 2^15 frames)."""
    import numpy as np
    N, p, b, u, R, phi = 2048, 4, 65536, 64, 4, 0.1
    Nf, bf = N * u, (N * b) // (N * u)
    w = ipfb.window_sinc_hamming(p, N)
    wf = ipfb.window_sinc_hamming(4, Nf)
    g = torch.Generator(device="cuda")
    g.manual_seed(7)
    x = torch.randn(N * b, generator=g, device="cuda", dtype=torch.float32)
    plan = ipfb.Plan(N, p, w, b, ipfb.F32)
    fine = ipfb.Plan(Nf, 4, wf, bf, ipfb.F32)
    y = ipfb.pfb_forward(plan, x)
    pk, sc = ipfb.quantize_c4(plan, y, 1.0 / 0.353)
    del y

    def summary(xh):
        d = ipfb.autospectrum_error(fine, x, xh).cpu().numpy()
        K = d.size
        prof = np.array([d[m:K - 1:u].mean() for m in range(u)])
        return {"delta_max": float(d.max()), "delta_max_at_fine_channel": int(d.argmax()),
                "delta_p99": float(np.quantile(d, 0.99)), "delta_median": float(np.median(d)),
                "delta_edge_folded": float(prof[u // 2]), "delta_centre_folded": float(prof[0])}

    out = {"config": {"lblock": N, "ntap": p, "nblock": b, "samples": N * b, "u": u, "R": R, "phi": phi,
                      "iters": iters, "levels_rms": 1.0 / 0.353, "dtype": "f32"}}
    t0 = time.perf_counter()
    xw = ipfb.ipfb_wiener(plan, pk, sc, phi)
    torch.cuda.synchronize()
    out["wiener"] = summary(xw)
    out["wiener"]["solve_s"] = time.perf_counter() - t0
    dan = ipfb.delta_analytic(plan, 4096, phi)
    torch.cuda.synchronize()
    out["wiener"]["analytic_delta_max"] = float(dan.max())
    xm = torch.empty_like(x)
    for beta in betas:
        L = int(2 * round(beta * R * N / 2.0))
        mask = ipfb.mask_structured(plan, R, L)
        ipfb.ml_cg(plan, pk, sc, mask, x, 1.0, phi, phi, iters, x_init=xw, x_out=xm)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, nr = ipfb.ml_cg(plan, pk, sc, mask, x, 1.0, phi, phi, iters, x_init=xw, x_out=xm)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        r = summary(xm)
        nr = nr.cpu().numpy()
        r.update({"saved_paths": L, "saved_fraction": float(len(range(0, b, R)) * L) / float(N * b),
                  "solve_s": sec, "samples_per_s": N * b / sec, "resid_drop": float(nr[-1] / nr[0])})
        out[f"cg_beta_{beta:.2f}"] = r
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip timing the FP64 form")
    ap.add_argument("--cpu-frames", type=int, default=16384)
    ap.add_argument("--no-ml", action="store_true", help="skip timing the ML-CG form")
    ap.add_argument("--no-batched", action="store_true", help="skip timing the batched form")
    ap.add_argument("--batched-streams", type=int, default=256)
    ap.add_argument("--no-stream", action="store_true", help="skip timing the streaming (linear boundary) form")
    ap.add_argument("--no-sweep", action="store_true", help="skip the structured-prior sweep (Section 4.3)")
    ap.add_argument("--no-alt", action="store_true", help="skip timing the comparison solvers (Appendix C)")
    ap.add_argument("--no-pipelined", action="store_true", help="skip the two-stream (pipelined) headline step")
    ap.add_argument("--no-small", action="store_true", help="skip the small configuration's latency")
    ap.add_argument("--no-copy-peak", action="store_true", help="skip timing the plain device copy")
    ap.add_argument("--probe-copy", action="store_true",
                    help="only run a plain 256 MiB device copy 5 times (HBM counter calibration) and exit")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path. Independent streams "
              "would shard over GPUs without communication, one long stream with one all-to-all of the "
              "frame matrix between the row and column stages.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2608_23441_amd import build as build_mod
    from paper_2608_23441_amd import inputs, ipfb

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.probe_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"probe": "copy", "bytes_read_per_launch": src.numel() * 4,
                          "bytes_written_per_launch": dst.numel() * 4}))
        return
    N, p, b, u, phi = 4096, 4, 16384, 64, 0.1
    Nf = N * u
    bf = (N * b) // Nf
    S = N * b

    _, w, packed, scales = make_inputs(torch, ipfb, inputs, N, p, b, 2, 5, 102, 0.1, 2.5)
    wf = ipfb.window_sinc_hamming(4, Nf)

    results = {}
    outputs = {}
    kernels = ["ipfb_rows", "ipfb_cols_fwd", "ipfb_cols_gain", "ipfb_cols_inv", "ipfb_cols_rec_setup",
               "ipfb_cols_rec_pass1", "ipfb_cols_rec_carry", "ipfb_cols_rec_pass2", "pfb_fwd_long_p1",
               "pfb_fwd_long_p2", "autospec_final"]
    forms = [("f32", ipfb.F32)] + ([] if args.no_fp64 else [("f64", ipfb.F64)])
    for tag, prec in forms:
        coarse = ipfb.Plan(N, p, w, b, prec)
        fine = ipfb.Plan(Nf, 4, wf, bf, prec)
        xh = torch.empty(S, dtype=coarse.real_dtype, device="cuda")
        Y = torch.empty((bf, Nf // 2 + 1), dtype=fine.complex_dtype, device="cuda")
        A = torch.empty(Nf // 2 + 1, dtype=torch.float64, device="cuda")

        def step():
            ipfb.ipfb_wiener(coarse, packed, scales, phi, x_out=xh)
            ipfb.upchannelize(fine, xh, Y, A)

        steps = args.steps if tag == "f32" else max(5, args.steps // 2)
        # the same steps without the per-kernel events, to show what recording them costs
        sec_plain = time_steps(torch, step, steps, args.warmup)
        ipfb.profile_reset()
        ipfb.profile_enable(True)
        sec = time_steps(torch, step, steps, args.warmup)
        ipfb.profile_enable(False)
        per_kernel = {}
        for k in kernels:
            ms, n = ipfb.profile_query(k)
            if n:
                per_kernel[k] = {"avg_us": 1e3 * ms / n, "launches": n}
        ipfb.profile_reset()
        esz = 4 if tag == "f32" else 8
        progress(f"{tag} form timed: {sec_plain * 1e3:.3f} ms per step")
        results[tag] = {"sec_per_step": sec, "sec_per_step_no_events": sec_plain, "per_kernel": per_kernel,
                        "esz": esz, "steps": steps}
        outputs[tag] = (xh, Y, A)
        del coarse, fine

    # FP32 form against the FP64 form on the same ints (both parity-tested
    # against the oracle elsewhere)
    agree = None
    if "f64" in outputs:
        x32, Y32, A32 = outputs["f32"]
        x64, Y64, A64 = outputs["f64"]
        ex = float(torch.linalg.vector_norm(x32.double() - x64) / torch.linalg.vector_norm(x64))
        eY = float(torch.linalg.vector_norm(Y32.to(torch.complex128) - Y64) / torch.linalg.vector_norm(Y64))
        eA = float(torch.max(torch.abs(A32 - A64) / A64))
        agree = {"timestream_rel_rms": ex, "fine_spectra_rel_rms": eY, "autospec_max_rel": eA}

    r32 = results["f32"]
    # the headline is the run without per-kernel events; the evented run
    # gives the per-kernel durations
    sec = r32["sec_per_step_no_events"]
    pk = r32["per_kernel"]
    one_pass = b <= 512

    def cb(k, esz=4):
        return kernel_bytes(k, N, b, Nf, bf, esz, "compulsory", one_pass)

    def mb(k, esz=4):
        return kernel_bytes(k, N, b, Nf, bf, esz, "moved", one_pass)

    # the dominant kernel: the longest average duration on the launch stream
    dom = max(pk, key=lambda k: pk[k]["avg_us"])
    alg = cb(dom)
    achieved = alg / (pk[dom]["avg_us"] * 1e-6) / 1e9
    sb32 = step_bytes(N, b, Nf, bf, 4)
    tr = load_traffic(dom)
    out = {
        "metric": METRIC,
        "value": S / sec,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": r32["steps"],
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "ms_per_step_with_kernel_events": r32["sec_per_step"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "production: white noise + 5 tones, 4-bit spectra, Wiener inverse PFB, "
                               "x64 up-channelize with autospectrum",
                   "lblock": N, "ntap": p, "nblock": b, "samples": S, "phi": phi,
                   "lblock_fine": Nf, "nblock_fine": bf, "window": "sinc x Hamming",
                   "column_stage": "recursive" if "ipfb_cols_rec_pass2" in pk else "fft"},
        "hbm_GBps": sb32 / sec / 1e9,
        "hbm_roofline_frac": sb32 / sec / 1e9 / HBM_PEAK_GBPS,
        "step_bytes": sb32,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS, "traffic": tr,
                     "compulsory_bytes_per_launch": alg, "moved_bytes_per_launch": mb(dom),
                     "traffic_over_compulsory": (tr / alg) if (tr and alg) else None,
                     "avg_us": pk[dom]["avg_us"]},
        "per_kernel_us": {k: round(v["avg_us"], 2) for k, v in pk.items()},
        "per_kernel_compulsory_GBps": {k: round(cb(k) / (v["avg_us"] * 1e-6) / 1e9, 1) for k, v in pk.items()},
        "per_kernel_moved_GBps": {k: round(mb(k) / (v["avg_us"] * 1e-6) / 1e9, 1) for k, v in pk.items()
                                  if mb(k)},
        "library": {"source_digest": ipfb.library_source_digest(), "tree_source_digest": build_mod.source_digest()},
    }
    if "f64" in results:
        r64 = results["f64"]
        sb64 = step_bytes(N, b, Nf, bf, 8)
        out["fp64_form"] = {"value": S / r64["sec_per_step_no_events"], "unit": "samples/s",
                            "ms_per_step": r64["sec_per_step_no_events"] * 1e3,
                            "hbm_GBps": sb64 / r64["sec_per_step_no_events"] / 1e9,
                            "hbm_roofline_frac": sb64 / r64["sec_per_step_no_events"] / 1e9 / HBM_PEAK_GBPS,
                            "per_kernel_us": {k: round(v["avg_us"], 2) for k, v in r64["per_kernel"].items()}}
        out["fp32_vs_fp64"] = agree
    if not args.no_copy_peak:
        cp = copy_peak_GBps(torch)
        out["copy_peak_GBps"] = cp
        out["hbm_frac_of_copy_peak"] = out["hbm_GBps"] / cp
        out["roofline"]["frac_of_copy_peak"] = achieved / cp
    if not args.no_pipelined:
        out["pipelined_form"] = pipelined_form(torch, ipfb, packed, scales, w, wf, N, p, b, Nf, bf, phi)
        progress("pipelined form done")
    if not args.no_small:
        out["small_config_latency"] = small_config(torch, ipfb, inputs)
        progress("small configuration done")
    if not args.no_ml:
        out["ml_form"] = ml_form(torch, ipfb, inputs)
        progress("ML-CG form done")
    if not args.no_batched:
        out["batched_form"] = batched_form(torch, ipfb, inputs, args.batched_streams)
        progress("batched form done")
    if not args.no_stream:
        out["streaming_form"] = streaming_form(torch, ipfb)
        progress("streaming form done")
    if not args.no_sweep:
        out["structured_prior_sweep"] = structured_sweep(torch, ipfb)
        progress("structured-prior sweep done")
    if not args.no_alt:
        out["alt_solvers"] = alt_solvers(torch, ipfb)
        progress("comparison solvers done")
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(N, p, Nf, phi, args.cpu_frames, 2)
        progress("CPU oracle baseline done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
