"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, validates arguments before touching the device, and its host
window helper matches the oracle's window."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import ipfb_oracle as O
from paper_2608_23441_amd import ipfb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    txt = open(os.path.join(ROOT, "include", "ipfb.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\*?(\w+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


@pytest.mark.parametrize("lang,std", [("c", "-std=c99"), ("c++", "-std=c++11")])
def test_header_is_plain_c_and_cxx(lang, std):
    # the boundary is a C ABI: the header alone compiles as C and as C++
    import shutil
    import subprocess
    cc = shutil.which("gcc" if lang == "c" else "g++")
    if cc is None:
        pytest.skip("no host compiler")
    r = subprocess.run([cc, "-fsyntax-only", "-Wall", "-Wextra", "-Werror", "-x", lang, std,
                        os.path.join(ROOT, "include", "ipfb.h")], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_library_exports_every_header_symbol():
    L = ipfb.lib()
    names = _header_functions()
    assert "ipfb_wiener" in names and "pfb_adjoint" in names and "upchannelize" in names
    for n in names:
        assert hasattr(L, n), f"missing export {n}"
    assert set(ipfb.EXPORTS) <= set(names)
    assert b"gfx950" in L.ipfb_version()


def test_library_built_from_these_sources():
    # the digest compiled into libipfb.so is the one of the tree's sources:
    # a source edited after the last build fails here
    from paper_2608_23441_amd import build as B
    assert ipfb.library_source_digest() == B.source_digest()


def test_window_helper_matches_oracle():
    for ntap, lblock in [(4, 64), (4, 2048), (3, 32), (1, 16)]:
        w = ipfb.window_sinc_hamming(ntap, lblock)
        assert np.abs(w - O.window_sinc_hamming(ntap, lblock)).max() < 1e-15


def _create(lblock, ntap, window, nblock, prec):
    h = ctypes.c_void_p()
    w = np.ascontiguousarray(window, dtype=np.float64)
    st = ipfb.lib().ipfb_plan_create(ctypes.byref(h), lblock, ntap,
                                     w.ctypes.data if w.size else None, nblock, prec)
    return st, h


@pytest.mark.parametrize("lblock,ntap,nblock,prec", [
    (3, 4, 16, 0),       # not a power of two
    (2, 4, 16, 0),       # too short
    (64, 0, 16, 0),      # no taps
    (64, 4, 0, 0),       # no frames
    (64, 4, 16, 7),      # bad precision
])
def test_plan_create_rejects_bad_arguments(lblock, ntap, nblock, prec):
    st, h = _create(lblock, ntap, np.ones(max(1, lblock * max(ntap, 1))), nblock, prec)
    assert st == ipfb.EINVAL
    assert not h.value
    assert len(ipfb.lib().ipfb_last_error()) > 0


def test_plan_create_rejects_null_window_and_huge_frames():
    h = ctypes.c_void_p()
    assert ipfb.lib().ipfb_plan_create(ctypes.byref(h), 64, 4, None, 16, 0) == ipfb.EINVAL
    st, _ = _create(1 << 21, 1, np.ones(1), 4, 0)
    assert st == ipfb.EUNSUPPORTED


def test_calls_reject_null_plan_and_pointers():
    L = ipfb.lib()
    assert L.pfb_forward(None, None, None, None) == ipfb.EINVAL
    assert L.pfb_adjoint(None, None, None, None) == ipfb.EINVAL
    assert L.ipfb_wiener(None, 0, None, None, 0.1, None, None) == ipfb.EINVAL
    assert L.upchannelize(None, None, None, None, None) == ipfb.EINVAL
    assert L.ipfb_autospectrum(None, None, None, None) == ipfb.EINVAL
    assert L.ipfb_quantize_c4(None, None, 2.5, None, None, None) == ipfb.EINVAL
    assert L.ipfb_plan_destroy(None) == ipfb.EINVAL
    assert L.ipfb_plan_set_workspace(None, None, 0) == ipfb.EINVAL
    assert L.ipfb_plan_device_bytes(None, None) == ipfb.EINVAL
    assert L.ipfb_plan_workspace_size(None, None) == ipfb.EINVAL
    assert L.ipfb_window_sinc_hamming(None, 4, 16) == ipfb.EINVAL


def test_new_entry_points_reject_bad_arguments_before_any_device_call():
    L = ipfb.lib()
    i4 = (ctypes.c_int * 6)(5, 16, 16, 0, 1, 0)
    # batched shapes and tuner, streaming, filters, diagnostics, structured mask
    assert L.ipfb_batched_get_shape(None, 10, i4) == ipfb.EINVAL
    assert L.ipfb_batched_set_shape(None, 10, i4) == ipfb.EINVAL
    assert L.ipfb_batched_tune(None, None, 0) == ipfb.EINVAL
    assert L.ipfb_stream_plan_destroy(None) == ipfb.EINVAL
    assert L.ipfb_wiener_stream(None, 0, None, None, 10, 0.1, 1, None, None) == ipfb.EINVAL
    assert L.ipfb_wiener_filter(None, 0, None, None, 1, 0.1, None, 1, None, None) == ipfb.EINVAL
    assert L.ipfb_delta_analytic(None, 16, 0.1, 0.0, None, None) == ipfb.EINVAL
    assert L.ipfb_autospectrum_error(None, None, None, None, None) == ipfb.EINVAL
    assert L.ipfb_mask_structured(None, 4, 8, None, None) == ipfb.EINVAL
    # column method, comparison solvers, ML-CG (both entries), mask packing
    assert L.ipfb_plan_set_column_method(None, 0) == ipfb.EINVAL
    assert L.ipfb_batched_set_column_method(None, 0) == ipfb.EINVAL
    assert L.ipfb_tikhonov(None, 0, None, None, 0.1, 1, None, None) == ipfb.EINVAL
    assert L.ipfb_fir_kernels(None, 0.1, 11, 1, None, None) == ipfb.EINVAL
    assert L.ipfb_fir(None, 0, None, None, 0.1, 11, 1, None, None) == ipfb.EINVAL
    assert L.ipfb_ml_cg(None, 0, None, None, None, None, 1.0, 0.1, 0.1, 5, None, None, None, None) == ipfb.EINVAL
    assert L.ipfb_ml_cg_noalloc(None, 0, None, None, None, None, 1.0, 0.1, 0.1, 5, None, None, None,
                                None) == ipfb.EINVAL
    assert L.ipfb_mask_pack(None, -1, None, None) == ipfb.EINVAL
    assert L.ipfb_mask_pack(None, 64, None, None) == ipfb.EINVAL
    w = np.ones(4 * 64)
    h = ctypes.c_void_p()
    for chunk, halo, prec in [(100, 8, 0), (64, 31, 0), (2, 0, 0), (64, -1, 0), (1 << 16, 8, 0), (1 << 15, 8, 1),
                              (64, 8, 5)]:
        st = L.ipfb_stream_plan_create(ctypes.byref(h), 64, 4, w.ctypes.data, chunk, halo, prec)
        assert st == ipfb.EINVAL and not h.value, (chunk, halo, prec)
        assert len(L.ipfb_last_error()) > 0
    assert L.ipfb_stream_plan_create(None, 64, 4, w.ctypes.data, 64, 8, 0) == ipfb.EINVAL
