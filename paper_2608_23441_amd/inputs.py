"""Seeded synthetic inputs shared by the GPU path's callers and the oracle.

This module draws random numbers and nothing else: it holds none of the
inverse-PFB arithmetic (no window, no filter bank, no FFT, no quantiser).
Both the HIP path and the CPU oracle receive what it returns as plain input.

Signal model (Section 4.3): a real timestream of standard-normal samples, as
the paper's end-to-end simulation uses; optionally a few narrow tones added on
top (the production-size workload, not in the paper), whose frequencies and
phases are drawn here too.
"""
from __future__ import annotations

import numpy as np


def gaussian_timestream(nsamples: int, seed: int, sigma: float = 1.0) -> np.ndarray:
    """float64 [nsamples] ~ N(0, sigma^2), PCG64 stream `seed`."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(int(nsamples)) * float(sigma)


def tone_parameters(ntones: int, seed: int, fmin: float = 0.01, fmax: float = 0.49):
    """Frequencies (cycles/sample, uniform in [fmin, fmax]) and phases (uniform in [0, 2pi))."""
    rng = np.random.default_rng(seed)
    f = rng.uniform(fmin, fmax, int(ntones))
    th = rng.uniform(0.0, 2.0 * np.pi, int(ntones))
    return f, th


def add_tones(x: np.ndarray, freqs, phases, amplitude: float) -> np.ndarray:
    """x + amplitude * cos(2 pi f m + theta) summed over the given tones (in place, returns x)."""
    m = np.arange(x.shape[0], dtype=np.float64)
    for f, th in zip(freqs, phases):
        x += amplitude * np.cos(2.0 * np.pi * f * m + th)
    return x


def timestream_with_tones(nsamples: int, seed: int, ntones: int, tone_seed: int,
                          amplitude: float = 0.1) -> np.ndarray:
    x = gaussian_timestream(nsamples, seed)
    f, th = tone_parameters(ntones, tone_seed)
    return add_tones(x, f, th, amplitude)


def batched_nblocks(nstreams: int = 256, lo: int = 1024, hi: int = 32768, seed: int = 4) -> np.ndarray:
    """Per-stream frame counts, uniform integers in [lo, hi] (both ends included)."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi, int(nstreams), endpoint=True).astype(np.int64)


def random_mask(nsamples: int, fraction: float, seed: int) -> np.ndarray:
    """bool [nsamples] with exactly round(fraction * nsamples) distinct True entries."""
    rng = np.random.default_rng(seed)
    k = int(round(fraction * nsamples))
    idx = rng.choice(int(nsamples), size=k, replace=False)
    m = np.zeros(int(nsamples), dtype=bool)
    m[idx] = True
    return m


def uniform_block(shape, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """float64 array of the given shape, uniform in [lo, hi) (generic test operand)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=shape)


def complex_block(shape, seed: int) -> np.ndarray:
    """complex128 array with standard-normal real and imaginary parts (generic test operand)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
