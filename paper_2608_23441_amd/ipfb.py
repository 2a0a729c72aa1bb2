"""Thin Python binding of libipfb (ctypes). Argument marshalling only: every
step of the computation runs in the HIP kernels behind the C ABI.

Tensors are torch tensors on the GPU (torch provides device memory and
streams). Real arrays are float32 for F32 plans and float64 for F64 plans;
complex arrays are complex64 / complex128 (interleaved re, im).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libipfb.so")

F32, F64 = 0, 1
IN_C4, IN_CI8, IN_CF32, IN_CF64 = 0, 1, 2, 3
OK, EINVAL, EUNSUPPORTED, ENOMEM, EHIP = 0, -1, -2, -3, -4

# Symbols the C ABI exports (include/ipfb.h).
EXPORTS = (
    "ipfb_last_error", "ipfb_version", "ipfb_window_sinc_hamming", "ipfb_plan_create",
    "ipfb_plan_destroy", "ipfb_plan_workspace_size", "ipfb_plan_device_bytes", "ipfb_plan_set_workspace",
    "pfb_forward", "pfb_adjoint", "ipfb_wiener",
    "ipfb_wiener_ex", "upchannelize", "ipfb_autospectrum", "ipfb_quantize_c4",
    "ipfb_profile_enable", "ipfb_profile_reset", "ipfb_profile_query", "ipfb_ml_cg",
    "ipfb_batched_plan_create", "ipfb_batched_plan_destroy", "ipfb_batched_workspace_size",
    "ipfb_batched_use_graph", "ipfb_wiener_batched", "ipfb_batched_get_shape",
    "ipfb_batched_set_shape", "ipfb_batched_tune", "ipfb_stream_plan_create", "ipfb_stream_plan_destroy",
    "ipfb_wiener_stream", "ipfb_delta_analytic", "ipfb_autospectrum_error", "ipfb_mask_structured",
    "ipfb_wiener_filter", "ipfb_mask_pack", "ipfb_ml_cg_noalloc", "ipfb_plan_set_column_method",
    "ipfb_batched_set_column_method", "ipfb_tikhonov", "ipfb_fir_kernels", "ipfb_fir",
)
COLS_AUTO, COLS_FFT, COLS_RECURSIVE = 0, 1, 2
FILTER_WIENER, FILTER_THRESHOLD, FILTER_NU = 0, 1, 2


class IpfbError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"ipfb status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libipfb.so from the package directory; fails loudly if it is absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libipfb.so not built at {LIB_PATH}; run __graft_entry__.build() "
                              "(or python paper_2608_23441_amd/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
        L.ipfb_last_error.restype = ctypes.c_char_p
        L.ipfb_version.restype = ctypes.c_char_p
        L.ipfb_window_sinc_hamming.argtypes = [vp, i32, i32]
        L.ipfb_plan_create.argtypes = [ctypes.POINTER(vp), i32, i32, vp, i64, i32]
        L.ipfb_plan_destroy.argtypes = [vp]
        L.ipfb_plan_workspace_size.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
        L.ipfb_plan_device_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
        L.ipfb_plan_set_workspace.argtypes = [vp, vp, ctypes.c_size_t]
        L.ipfb_plan_set_column_method.argtypes = [vp, i32]
        L.ipfb_batched_set_column_method.argtypes = [vp, i32]
        L.ipfb_tikhonov.argtypes = [vp, i32, vp, vp, dbl, i32, vp, vp]
        L.ipfb_fir_kernels.argtypes = [vp, dbl, i32, i32, vp, vp]
        L.ipfb_fir.argtypes = [vp, i32, vp, vp, dbl, i32, i32, vp, vp]
        L.pfb_forward.argtypes = [vp, vp, vp, vp]
        L.pfb_adjoint.argtypes = [vp, vp, vp, vp]
        L.ipfb_wiener.argtypes = [vp, i32, vp, vp, dbl, vp, vp]
        L.ipfb_wiener_ex.argtypes = [vp, i32, vp, vp, dbl, i32, vp, vp]
        L.upchannelize.argtypes = [vp, vp, vp, vp, vp]
        L.ipfb_autospectrum.argtypes = [vp, vp, vp, vp]
        L.ipfb_quantize_c4.argtypes = [vp, vp, dbl, vp, vp, vp]
        L.ipfb_ml_cg.argtypes = [vp, i32, vp, vp, vp, vp, dbl, dbl, dbl, i32, vp, vp, vp, vp]
        L.ipfb_ml_cg_noalloc.argtypes = [vp, i32, vp, vp, vp, vp, dbl, dbl, dbl, i32, vp, vp, vp, vp]
        L.ipfb_batched_plan_create.argtypes = [ctypes.POINTER(vp), i32, i32, vp, i32, vp, i32]
        L.ipfb_batched_plan_destroy.argtypes = [vp]
        L.ipfb_batched_workspace_size.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
        L.ipfb_batched_use_graph.argtypes = [vp, i32]
        L.ipfb_wiener_batched.argtypes = [vp, i32, vp, vp, dbl, i32, vp, vp]
        L.ipfb_batched_get_shape.argtypes = [vp, i32, ctypes.POINTER(i32)]
        L.ipfb_batched_set_shape.argtypes = [vp, i32, ctypes.POINTER(i32)]
        L.ipfb_batched_tune.argtypes = [vp, ctypes.c_char_p, i32]
        L.ipfb_stream_plan_create.argtypes = [ctypes.POINTER(vp), i32, i32, vp, i64, i32, i32]
        L.ipfb_stream_plan_destroy.argtypes = [vp]
        L.ipfb_wiener_stream.argtypes = [vp, i32, vp, vp, i64, dbl, i32, vp, vp]
        L.ipfb_delta_analytic.argtypes = [vp, i64, dbl, dbl, vp, vp]
        L.ipfb_autospectrum_error.argtypes = [vp, vp, vp, vp, vp]
        L.ipfb_mask_structured.argtypes = [vp, i32, i32, vp, vp]
        L.ipfb_mask_pack.argtypes = [vp, i64, vp, vp]
        L.ipfb_wiener_filter.argtypes = [vp, i32, vp, vp, i32, dbl, vp, i32, vp, vp]
        L.ipfb_profile_enable.argtypes = [i32]
        L.ipfb_profile_reset.argtypes = []
        L.ipfb_profile_query.argtypes = [ctypes.c_char_p, ctypes.POINTER(dbl), ctypes.POINTER(i64)]
        for name in EXPORTS:
            getattr(L, name).restype = getattr(L, name).restype or ctypes.c_int
        L.ipfb_last_error.restype = ctypes.c_char_p
        L.ipfb_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def library_source_digest() -> str:
    """The source digest compiled into the loaded library (see ipfb_version)."""
    v = lib().ipfb_version().decode()
    return v.rsplit("sources ", 1)[-1] if "sources " in v else "unknown"


def _check(status):
    if status != OK:
        raise IpfbError(status, lib().ipfb_last_error().decode())


def window_sinc_hamming(ntap: int, lblock: int) -> np.ndarray:
    """The library's sinc x Hamming window (host, float64 [ntap*lblock])."""
    out = np.empty(ntap * lblock, dtype=np.float64)
    _check(lib().ipfb_window_sinc_hamming(out.ctypes.data, int(ntap), int(lblock)))
    return out


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, name):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """A plan for frames of `lblock` samples, `ntap` taps and `nblock` frames."""

    def __init__(self, lblock: int, ntap: int, window, nblock: int, prec: int = F32):
        self.lblock, self.ntap, self.nblock, self.prec = int(lblock), int(ntap), int(nblock), int(prec)
        w = np.ascontiguousarray(np.asarray(window, dtype=np.float64))
        if w.size != self.lblock * self.ntap:
            raise ValueError("window must have ntap*lblock taps")
        h = ctypes.c_void_p()
        _check(lib().ipfb_plan_create(ctypes.byref(h), self.lblock, self.ntap, w.ctypes.data,
                                      self.nblock, self.prec))
        self._h = h
        self._ws = None

    @property
    def handle(self):
        return self._h

    @property
    def nchan(self):
        return self.lblock // 2 + 1

    @property
    def real_dtype(self):
        import torch
        return torch.float32 if self.prec == F32 else torch.float64

    @property
    def complex_dtype(self):
        import torch
        return torch.complex64 if self.prec == F32 else torch.complex128

    def workspace_bytes(self) -> int:
        """Size of the workspace set_workspace takes."""
        b = ctypes.c_size_t()
        _check(lib().ipfb_plan_workspace_size(self._h, ctypes.byref(b)))
        return b.value

    def device_bytes(self) -> int:
        """Device bytes the plan itself holds."""
        b = ctypes.c_size_t()
        _check(lib().ipfb_plan_device_bytes(self._h, ctypes.byref(b)))
        return b.value

    def set_column_method(self, method: int):
        """COLS_AUTO, COLS_FFT or COLS_RECURSIVE (see ipfb_plan_set_column_method)."""
        _check(lib().ipfb_plan_set_column_method(self.handle, int(method)))

    def set_workspace(self, buf=None):
        """Give the plan a caller-owned workspace: a CUDA tensor of at least
        workspace_bytes() bytes, 256-byte aligned, kept alive (and otherwise
        unused) while the plan uses it; None returns the plan to its own."""
        if buf is None:
            _check(lib().ipfb_plan_set_workspace(self._h, None, 0))
            self._ws = None
            return
        nbytes = buf.numel() * buf.element_size()
        _check(lib().ipfb_plan_set_workspace(self._h, _ptr(buf, "workspace"), nbytes))
        self._ws = buf  # the plan keeps a reference while it uses the memory

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ipfb_plan_destroy(self._h)
            self._h = None
        self._ws = None  # a caller-provided workspace may go once the plan is gone

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- shape checks (marshalling) --
    def _real(self, t, name):
        if t.dtype != self.real_dtype or t.numel() != self.nblock * self.lblock:
            raise ValueError(f"{name}: expected {self.real_dtype} with {self.nblock * self.lblock} elements")
        return _ptr(t, name)

    def _cplx(self, t, name):
        if t.dtype != self.complex_dtype or t.numel() != self.nblock * self.nchan:
            raise ValueError(f"{name}: expected {self.complex_dtype} with {self.nblock * self.nchan} elements")
        return _ptr(t, name)


def _empty(shape, dtype):
    import torch
    return torch.empty(shape, dtype=dtype, device="cuda")


def pfb_forward(plan: Plan, x, y=None, stream=None):
    if y is None:
        y = _empty((plan.nblock, plan.nchan), plan.complex_dtype)
    _check(lib().pfb_forward(plan.handle, plan._real(x, "x"), plan._cplx(y, "y"), _stream(stream)))
    return y


def pfb_adjoint(plan: Plan, y, x=None, stream=None):
    if x is None:
        x = _empty((plan.nblock * plan.lblock,), plan.real_dtype)
    _check(lib().pfb_adjoint(plan.handle, plan._cplx(y, "y"), plan._real(x, "x"), _stream(stream)))
    return x


def _spec_format(spec, nchan, chan_scale):
    """Input format of a spectrum tensor and the number of complex values it
    holds: uint8 (packed 4-bit, one byte per value), int8 (8-bit codes, two
    bytes per value: real then imaginary), complex64 or complex128. The two
    quantised formats need chan_scale, float32 [nchan]."""
    import torch
    if spec.dtype == torch.uint8:
        fmt, n = IN_C4, spec.numel()
    elif spec.dtype == torch.int8:
        if spec.numel() % 2:
            raise ValueError("int8 spectra hold (real, imaginary) pairs: an even number of bytes")
        fmt, n = IN_CI8, spec.numel() // 2
    elif spec.dtype == torch.complex64:
        fmt, n = IN_CF32, spec.numel()
    elif spec.dtype == torch.complex128:
        fmt, n = IN_CF64, spec.numel()
    else:
        raise ValueError("spec must be uint8 (packed 4-bit), int8 (8-bit pairs), complex64 or complex128")
    if fmt in (IN_C4, IN_CI8) and (chan_scale is None or chan_scale.dtype != torch.float32
                                   or chan_scale.numel() != nchan):
        raise ValueError("chan_scale: float32 [nchan] is required for quantised spectra")
    return fmt, n


def ipfb_wiener(plan: Plan, spec, chan_scale=None, phi: float = 0.1, x_out=None, normalise: bool = True,
                stream=None):
    """spec: uint8 [nblock, nchan] (4-bit packed) or int8 [nblock, nchan, 2]
    (8-bit), both with chan_scale float32 [nchan]; or complex64 / complex128
    [nblock, nchan]."""
    fmt = _spec_fmt(plan, spec, chan_scale)
    if x_out is None:
        x_out = _empty((plan.nblock * plan.lblock,), plan.real_dtype)
    _check(lib().ipfb_wiener_ex(plan.handle, fmt, _ptr(spec, "spec"), _ptr(chan_scale, "chan_scale"),
                                float(phi), int(bool(normalise)), plan._real(x_out, "x_out"),
                                _stream(stream)))
    return x_out


def wiener_filter(plan: Plan, spec, chan_scale=None, kind: int = FILTER_WIENER, param: float = 0.1, nu=None,
                  x_out=None, normalise: bool = True, stream=None):
    """The circulant inverse with another eigenvalue filter (ipfb_wiener_filter);
    nu: float64 [nblock/2 + 1] on the GPU for FILTER_NU."""
    import torch
    fmt = _spec_fmt(plan, spec, chan_scale)
    if kind == FILTER_NU and (nu is None or nu.dtype != torch.float64 or nu.numel() != plan.nblock // 2 + 1):
        raise ValueError("nu: float64 [nblock/2 + 1] is required for FILTER_NU")
    if x_out is None:
        x_out = _empty((plan.nblock * plan.lblock,), plan.real_dtype)
    _check(lib().ipfb_wiener_filter(plan.handle, fmt, _ptr(spec, "spec"), _ptr(chan_scale, "chan_scale"), int(kind),
                                    float(param), _ptr(nu, "nu"), int(bool(normalise)), plan._real(x_out, "x_out"),
                                    _stream(stream)))
    return x_out


def _quantised_dtypes():
    import torch
    return (torch.uint8, torch.int8)


def _spec_fmt(plan, spec, chan_scale):
    fmt, n = _spec_format(spec, plan.nchan, chan_scale)
    if n != plan.nblock * plan.nchan:
        raise ValueError("spec must hold nblock * (lblock/2+1) values")
    return fmt


def tikhonov(plan: Plan, spec, chan_scale=None, phi: float = 0.1, normalise: bool = True, x_out=None,
             stream=None):
    """Appendix C's Tikhonov solver of the linear sub-problems (banded
    Cholesky). spec: [nblock - ntap + 1, nchan] spectra of a linear PFB."""
    fmt, n = _spec_format(spec, plan.nchan, chan_scale)
    if n != (plan.nblock - plan.ntap + 1) * plan.nchan:
        raise ValueError("spec must hold (nblock - ntap + 1) * (lblock/2+1) values")
    if x_out is None:
        x_out = _empty((plan.nblock * plan.lblock,), plan.real_dtype)
    _check(lib().ipfb_tikhonov(plan.handle, fmt, _ptr(spec, "spec"), _ptr(chan_scale, "chan_scale"), float(phi),
                               int(bool(normalise)), plan._real(x_out, "x_out"), _stream(stream)))
    return x_out


def fir_kernels(plan: Plan, phi: float, ltaps: int, normalise: bool = True, out=None, stream=None):
    """The truncated decorrelation kernels [ltaps, lblock] (plan precision)."""
    if out is None:
        out = _empty((int(ltaps), plan.lblock), plan.real_dtype)
    _check(lib().ipfb_fir_kernels(plan.handle, float(phi), int(ltaps), int(bool(normalise)), _ptr(out, "kernels"),
                                  _stream(stream)))
    return out


def fir(plan: Plan, spec, chan_scale=None, phi: float = 0.1, ltaps: int = 51, normalise: bool = True, x_out=None,
        stream=None):
    """The inverse with FIR decorrelation by truncated kernels (Appendix C)."""
    fmt = _spec_fmt(plan, spec, chan_scale)
    if x_out is None:
        x_out = _empty((plan.nblock * plan.lblock,), plan.real_dtype)
    _check(lib().ipfb_fir(plan.handle, fmt, _ptr(spec, "spec"), _ptr(chan_scale, "chan_scale"), float(phi),
                          int(ltaps), int(bool(normalise)), plan._real(x_out, "x_out"), _stream(stream)))
    return x_out


def ml_cg(plan: Plan, spec, chan_scale, mask, prior, lam: float = 1.0, phi_x0: float = 0.1,
          phi_precond: float = 0.1, iters: int = 100, x_init=None, x_out=None, resid=True, stream=None):
    """Maximum-likelihood reconstruction with a time-domain prior (PCG).
    mask: the bitmask of ceil(S/32) 32-bit words (int32 tensor; see
    mask_pack), bit e for time-order sample e; prior: real [S] in the plan
    precision. Returns (x, residual norms [iters+1] float64 or None)."""
    import torch
    fmt = _spec_fmt(plan, spec, chan_scale)
    S = plan.nblock * plan.lblock
    if mask.dtype != torch.int32 or mask.numel() != (S + 31) // 32:
        raise ValueError("mask: int32 [ceil(nblock*lblock/32)] bitmask words")
    if x_out is None:
        x_out = _empty((S,), plan.real_dtype)
    norms = _empty((iters + 1,), torch.float64) if resid else None
    _check(lib().ipfb_ml_cg(plan.handle, fmt, _ptr(spec, "spec"), _ptr(chan_scale, "chan_scale"),
                            _ptr(mask, "mask"), plan._real(prior, "prior"), float(lam), float(phi_x0),
                            float(phi_precond), int(iters),
                            None if x_init is None else plan._real(x_init, "x_init"),
                            plan._real(x_out, "x_out"), _ptr(norms, "resid"), _stream(stream)))
    return x_out, norms


def upchannelize(fine: Plan, x, y_fine=None, autospec=None, want_autospec: bool = True, stream=None):
    import torch
    if y_fine is None:
        y_fine = _empty((fine.nblock, fine.nchan), fine.complex_dtype)
    if autospec is None and want_autospec:
        autospec = _empty((fine.nchan,), torch.float64)
    if autospec is not None and (autospec.dtype != torch.float64 or autospec.numel() != fine.nchan):
        raise ValueError("autospec: float64 [nchan]")
    _check(lib().upchannelize(fine.handle, fine._real(x, "x"), fine._cplx(y_fine, "y_fine"),
                              _ptr(autospec, "autospec"), _stream(stream)))
    return y_fine, autospec


def autospectrum(plan: Plan, y, out=None, stream=None):
    import torch
    if out is None:
        out = _empty((plan.nchan,), torch.float64)
    _check(lib().ipfb_autospectrum(plan.handle, plan._cplx(y, "y"), _ptr(out, "out"), _stream(stream)))
    return out


def quantize_c4(plan: Plan, y, levels_rms: float = 2.5, stream=None):
    import torch
    packed = _empty((plan.nblock, plan.nchan), torch.uint8)
    scales = _empty((plan.nchan,), torch.float32)
    _check(lib().ipfb_quantize_c4(plan.handle, plan._cplx(y, "y"), float(levels_rms), _ptr(packed, "packed"),
                                  _ptr(scales, "scales"), _stream(stream)))
    return packed, scales


def mask_structured(plan: Plan, R: int, L: int, out=None, stream=None):
    """The structured prior mask as ml_cg's bitmask (int32 [ceil(S/32)] words on the GPU)."""
    import torch
    nw = (plan.nblock * plan.lblock + 31) // 32
    if out is None:
        out = _empty((nw,), torch.int32)
    if out.dtype != torch.int32 or out.numel() != nw:
        raise ValueError("out: int32 [ceil(nblock*lblock/32)]")
    _check(lib().ipfb_mask_structured(plan.handle, int(R), int(L), _ptr(out, "mask"), _stream(stream)))
    return out


def mask_pack(mask, out=None, stream=None):
    """Byte-per-sample mask (uint8 or bool [S] on the GPU, nonzero = saved) to
    ml_cg's bitmask (int32 [ceil(S/32)] words)."""
    import torch
    if mask.dtype not in (torch.uint8, torch.bool):
        raise ValueError("mask: uint8 or bool")
    S = mask.numel()
    if out is None:
        out = _empty(((S + 31) // 32,), torch.int32)
    if out.dtype != torch.int32 or out.numel() != (S + 31) // 32:
        raise ValueError("out: int32 [ceil(S/32)]")
    _check(lib().ipfb_mask_pack(_ptr(mask, "mask"), int(S), _ptr(out, "bits"), _stream(stream)))
    return out


def delta_analytic(plan: Plan, nfreq: int, phi: float = 0.1, snr: float = 0.0, out=None, stream=None):
    """Appendix B's predicted delta(f) at f = k / nfreq (float64 [nfreq] on the GPU)."""
    import torch
    if out is None:
        out = _empty((int(nfreq),), torch.float64)
    _check(lib().ipfb_delta_analytic(plan.handle, int(nfreq), float(phi), float(snr), _ptr(out, "out"),
                                     _stream(stream)))
    return out


def autospectrum_error(fine: Plan, x_true, x_hat, out=None, stream=None):
    """Measured delta on the fine plan's channels (float64 [lblock_f/2+1])."""
    import torch
    if out is None:
        out = _empty((fine.nchan,), torch.float64)
    _check(lib().ipfb_autospectrum_error(fine.handle, fine._real(x_true, "x_true"), fine._real(x_hat, "x_hat"),
                                         _ptr(out, "out"), _stream(stream)))
    return out


def profile_enable(on: bool = True):
    _check(lib().ipfb_profile_enable(int(bool(on))))


def profile_reset():
    _check(lib().ipfb_profile_reset())


def profile_query(name: str):
    """(total milliseconds, launches) recorded for one kernel name."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(lib().ipfb_profile_query(name.encode(), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


class BatchedPlan:
    """Plan for many streams with their own nblock (any integer up to 32768)."""

    def __init__(self, lblock: int, ntap: int, window, nblocks, prec: int = F32):
        self.lblock, self.ntap, self.prec = int(lblock), int(ntap), int(prec)
        self.nblocks = [int(b) for b in nblocks]
        w = np.ascontiguousarray(np.asarray(window, dtype=np.float64))
        nb = np.ascontiguousarray(np.asarray(self.nblocks, dtype=np.int64))
        h = ctypes.c_void_p()
        _check(lib().ipfb_batched_plan_create(ctypes.byref(h), self.lblock, self.ntap, w.ctypes.data,
                                              len(self.nblocks), nb.ctypes.data, self.prec))
        self._h = h

    @property
    def nchan(self):
        return self.lblock // 2 + 1

    @property
    def real_dtype(self):
        import torch
        return torch.float32 if self.prec == F32 else torch.float64

    def set_column_method(self, method: int):
        """COLS_AUTO, COLS_FFT or COLS_RECURSIVE (see ipfb_batched_set_column_method)."""
        _check(lib().ipfb_batched_set_column_method(self._h, int(method)))

    def use_graph(self, on: bool):
        _check(lib().ipfb_batched_use_graph(self._h, int(bool(on))))

    def workspace_bytes(self) -> int:
        b = ctypes.c_size_t()
        _check(lib().ipfb_batched_workspace_size(self._h, ctypes.byref(b)))
        return b.value

    def conv_lengths(self):
        """log2 of the Bluestein convolution length of every stream whose
        nblock is not a power of two (sorted, distinct)."""
        out = set()
        for b in self.nblocks:
            if b >= 4 and b & (b - 1) == 0 and b.bit_length() - 1 <= (15 if self.prec == F32 else 14):
                continue
            m = 2
            while (1 << m) < 2 * b - 1:
                m += 1
            out.add(m)
        return sorted(out)

    def get_shape(self, log2m: int):
        """(l1, mb, kb, pchunk, fuse, nat) used for convolution length 2^log2m."""
        a = (ctypes.c_int * 6)()
        _check(lib().ipfb_batched_get_shape(self._h, int(log2m), a))
        return tuple(a)

    def set_shape(self, log2m: int, shape):
        a = (ctypes.c_int * 6)(*[int(v) for v in shape])
        _check(lib().ipfb_batched_set_shape(self._h, int(log2m), a))

    def tune(self, cache_path=None, force: bool = False):
        """Run the autotuner (see ipfb_batched_tune); returns {log2m: shape}."""
        path = None if cache_path is None else os.fsencode(cache_path)
        _check(lib().ipfb_batched_tune(self._h, path, int(bool(force))))
        return {m: self.get_shape(m) for m in self.conv_lengths()}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ipfb_batched_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def wiener_batched(bp: BatchedPlan, specs, chan_scales=None, phi: float = 0.1, x_outs=None,
                   normalise: bool = True, stream=None):
    """specs: list of per-stream spectra (uint8 packed 4-bit or int8 8-bit,
    with chan_scales; or complex); returns the list of per-stream timestreams."""
    ns = len(bp.nblocks)
    if len(specs) != ns:
        raise ValueError("one spectrum tensor per stream")
    quantised = specs and specs[0].dtype in _quantised_dtypes()
    if quantised and (chan_scales is None or len(chan_scales) != ns):
        raise ValueError("quantised spectra need one float32 scale vector per stream")
    fmt = None
    for i, (s_, b) in enumerate(zip(specs, bp.nblocks)):
        f, n = _spec_format(s_, bp.nchan, chan_scales[i] if quantised else None)
        if fmt is not None and f != fmt:
            raise ValueError("all streams need one spectrum dtype")
        fmt = f
        if n != b * bp.nchan:
            raise ValueError("stream spectra must hold nblock * (lblock/2+1) values")
    if x_outs is None:
        x_outs = [_empty((b * bp.lblock,), bp.real_dtype) for b in bp.nblocks]
    for x, b in zip(x_outs, bp.nblocks):
        if x.dtype != bp.real_dtype or x.numel() != b * bp.lblock:
            raise ValueError("x_outs: one real tensor of nblock*lblock per stream")
    P = ctypes.c_void_p * ns
    sp = P(*[_ptr(t, "spec").value for t in specs])
    xo = P(*[_ptr(t, "x_out").value for t in x_outs])
    sc = P(*[_ptr(t, "chan_scale").value for t in chan_scales]) if fmt in (IN_C4, IN_CI8) else None
    _check(lib().ipfb_wiener_batched(bp._h, fmt, sp, sc, float(phi), int(bool(normalise)), xo, _stream(stream)))
    return x_outs


class StreamPlan:
    """Plan of the streaming (overlap-save) inverse of a linear PFB: windows of
    `chunk` frames, `halo` frames discarded at each window edge."""

    def __init__(self, lblock: int, ntap: int, window, chunk: int, halo: int, prec: int = F32):
        self.lblock, self.ntap, self.chunk, self.halo, self.prec = int(lblock), int(ntap), int(chunk), int(halo), int(prec)
        w = np.ascontiguousarray(np.asarray(window, dtype=np.float64))
        h = ctypes.c_void_p()
        _check(lib().ipfb_stream_plan_create(ctypes.byref(h), self.lblock, self.ntap, w.ctypes.data, self.chunk,
                                             self.halo, self.prec))
        self._h = h

    @property
    def nchan(self):
        return self.lblock // 2 + 1

    @property
    def real_dtype(self):
        import torch
        return torch.float32 if self.prec == F32 else torch.float64

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ipfb_stream_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def wiener_stream(sp: StreamPlan, spec, chan_scale=None, phi: float = 0.1, x_out=None, normalise: bool = True,
                  stream=None):
    """Streaming inverse of nspec linear-PFB spectra (uint8 [nspec][nchan] or
    int8 [nspec][nchan][2] with chan_scale, or complex [nspec][nchan]); returns
    (nspec + ntap - 1) * lblock samples."""
    fmt, n = _spec_format(spec, sp.nchan, chan_scale)
    if fmt not in (IN_C4, IN_CI8):
        chan_scale = None
    if n % sp.nchan != 0 or n == 0:
        raise ValueError("spec must hold nspec * (lblock/2+1) values")
    nspec = n // sp.nchan
    nout = (nspec + sp.ntap - 1) * sp.lblock
    if x_out is None:
        x_out = _empty((nout,), sp.real_dtype)
    elif x_out.numel() != nout or not x_out.is_contiguous():
        raise ValueError(f"x_out must be a contiguous tensor of {nout} samples")
    _check(lib().ipfb_wiener_stream(sp._h, fmt, _ptr(spec, "spec"), _ptr(chan_scale, "chan_scale"), int(nspec),
                                    float(phi), int(bool(normalise)), _ptr(x_out, "x_out"), _stream(stream)))
    return x_out
