"""The benchmark's byte accounting (no GPU): the compulsory traffic of one
production step and the algorithmic bytes of each kernel, counted from the
data each step must move, and the one-GPU contract of the command line."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

N, B, NF, BF = 4096, 16384, 262144, 256  # production: 2^26 samples, x64 up-channelize
S = N * B
MB = 1e6


def test_step_bytes_fp32_and_fp64():
    # packed input (1 B per channel) + scales, d written and read, xhat written
    # and read back, the fine window, the fine spectra: 20.56 B/sample in FP32
    sb = bench.step_bytes(N, B, NF, BF, 4)
    assert sb / MB == pytest.approx(1380.2, abs=0.5)
    assert sb / S == pytest.approx(20.57, abs=0.01)
    # 172.5 us at 8 TB/s
    assert sb / 8e12 * 1e6 == pytest.approx(172.5, abs=0.1)
    assert bench.step_bytes(N, B, NF, BF, 8) / MB == pytest.approx(2726, abs=2)


# each kernel's share of the compulsory bytes (intermediate round trips at
# zero), for the recursive column stage and for the three-pass FFT stage
@pytest.mark.parametrize("name,mb", [("ipfb_rows", 302.0), ("ipfb_cols_rec_pass1", 268.4),
                                     ("ipfb_cols_rec_carry", 0.0), ("ipfb_cols_rec_pass2", 268.4),
                                     ("ipfb_cols_fwd", 268.4), ("ipfb_cols_gain", 0.0), ("ipfb_cols_inv", 268.4),
                                     ("pfb_fwd_long_p1", 272.6), ("pfb_fwd_long_p2", 268.4),
                                     ("autospec_final", 0.0)])
def test_compulsory_share_production_fp32(name, mb):
    assert bench.kernel_bytes(name, N, B, NF, BF, 4) / MB == pytest.approx(mb, abs=0.1)


def test_compulsory_shares_sum_to_the_step():
    rec = ["ipfb_rows", "ipfb_cols_rec_setup", "ipfb_cols_rec_pass1", "ipfb_cols_rec_carry", "ipfb_cols_rec_pass2",
           "pfb_fwd_long_p1", "pfb_fwd_long_p2", "autospec_final"]
    fft = ["ipfb_rows", "ipfb_cols_fwd", "ipfb_cols_gain", "ipfb_cols_inv", "pfb_fwd_long_p1", "pfb_fwd_long_p2"]
    for names in (rec, fft):
        for esz in (4, 8):
            assert sum(bench.kernel_bytes(k, N, B, NF, BF, esz) for k in names) == bench.step_bytes(N, B, NF, BF, esz)
    # the one-pass FFT stage (nblock <= 512) takes both shares in its one kernel
    n, b = 2048, 128
    one = ["ipfb_rows", "ipfb_cols_gain"]
    assert sum(bench.kernel_bytes(k, n, b, 16384, 16, 4, one_pass=True) for k in one) == \
        bench.kernel_bytes("ipfb_rows", n, b, 16384, 16, 4) + 2 * n * b * 4


# what each kernel moves by its design: the intermediates show up here
@pytest.mark.parametrize("name,mb", [("ipfb_cols_fwd", 536.9), ("ipfb_cols_gain", 536.9), ("ipfb_cols_inv", 536.9),
                                     ("ipfb_cols_rec_pass1", 268.4 + 25.2), ("ipfb_cols_rec_carry", 50.3),
                                     ("ipfb_cols_rec_pass2", 536.9 + 25.2), ("pfb_fwd_long_p1", 541.1),
                                     ("pfb_fwd_long_p2", 536.9)])
def test_moved_bytes_production_fp32(name, mb):
    assert bench.kernel_bytes(name, N, B, NF, BF, 4, "moved") / MB == pytest.approx(mb, abs=0.1)


def test_source_digest_is_stable_hex():
    d = bench.source_digest()
    assert d == bench.source_digest() and len(d) == 16
    int(d, 16)


def test_more_than_one_gpu_is_refused_before_any_device_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--steps", "1"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
