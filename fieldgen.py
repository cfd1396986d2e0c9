"""Seeded synthetic FP32 3-D fields: the inputs every test, the benchmark and the
smoke run feed to both the GPU library and the CPU oracle.

This module draws random numbers and shapes spectra; it contains none of the
compressor's arithmetic. The fields stand in for the paper's turbulence,
cosmology and seismic datasets (Sec. 6.1.3, Table "datasets"), which are not
available here: smooth Gaussian random fields whose 3-D power spectral density
falls as k^-beta (beta = 11/3 is the Kolmogorov slope), optionally with white
noise or a sharp front added.

Recipe of ``grf(shape, beta, seed)``:
  1. white noise N(0, 1) in float64 from numpy's PCG64 ``default_rng(seed)``;
  2. real FFT over all three axes;
  3. multiply by |k|^(-beta/2), |k| in integer FFT wave numbers, k = 0 set to 0;
  4. inverse FFT, normalise to mean 0 and standard deviation 1, cast to float32.
"""
from __future__ import annotations

import math
import os

import numpy as np

try:  # scipy's FFT takes a worker count; numpy's does not
    import scipy.fft as _fft

    def _rfftn(a, workers):
        return _fft.rfftn(a, axes=(0, 1, 2), workers=workers, overwrite_x=True)

    def _irfftn(a, s, workers):
        return _fft.irfftn(a, s=s, axes=(0, 1, 2), workers=workers, overwrite_x=True)
except ImportError:  # pragma: no cover
    def _rfftn(a, workers):
        return np.fft.rfftn(a, axes=(0, 1, 2))

    def _irfftn(a, s, workers):
        return np.fft.irfftn(a, s=s, axes=(0, 1, 2))


def _workers() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def grf(shape, beta: float, seed: int) -> np.ndarray:
    """Gaussian random field with power spectral density ~ k^-beta (float32, std 1)."""
    shape = tuple(int(s) for s in shape)
    if len(shape) != 3 or min(shape) < 1:
        raise ValueError(f"grf needs a 3-D shape with positive sides, got {shape}")
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(shape)
    spec = _rfftn(w, _workers())
    del w
    nx, ny, nz = shape
    kx = np.fft.fftfreq(nx) * nx
    ky = np.fft.fftfreq(ny) * ny
    kz = np.fft.rfftfreq(nz) * nz
    kyz2 = ky[:, None] ** 2 + kz[None, :] ** 2
    for i in range(nx):  # slab by slab keeps the filter small
        k2 = kx[i] ** 2 + kyz2
        with np.errstate(divide="ignore"):
            filt = np.where(k2 > 0, k2 ** (-beta / 4.0), 0.0)
        spec[i] *= filt
    f = _irfftn(spec, shape, _workers())
    del spec
    f -= f.mean()
    sd = f.std()
    if sd > 0:
        f /= sd
    return f.astype(np.float32)


def minmax01(f: np.ndarray) -> np.ndarray:
    """Scale to [0, 1] in float64, then cast to float32."""
    g = f.astype(np.float64)
    lo, hi = g.min(), g.max()
    if hi > lo:
        g = (g - lo) / (hi - lo)
    return g.astype(np.float32)


# ---------------------------------------------------------------------------
# The five workloads (sizes and spectra of the paper's 3-D datasets, Sec. 6.1.3)
# ---------------------------------------------------------------------------

def field_small(shape=(64, 64, 64), beta=3.0, seed=101) -> np.ndarray:
    """64^3 field, spectrum k^-3, min-max scaled to [0, 1]: the correctness case."""
    return minmax01(grf(shape, beta, seed))


def field_turb(shape=(512, 512, 512), seed=102, noise=0.01, noise_seed=1102) -> np.ndarray:
    """Kolmogorov-slope field (k^-11/3) plus 1 % white noise: the 512^3 headline case."""
    f = grf(shape, 11.0 / 3.0, seed)
    if noise > 0:
        rng = np.random.default_rng(noise_seed)
        f += (noise * rng.standard_normal(f.shape)).astype(np.float32)
    return f


def field_front(shape=(100, 500, 500), seed=103, front_seed=1103, amp=2.0) -> np.ndarray:
    """k^-3 background plus a tanh front of width 2 cells across a random plane."""
    f = grf(shape, 3.0, seed).astype(np.float64)
    rng = np.random.default_rng(front_seed)
    n = rng.standard_normal(3)
    n /= np.linalg.norm(n)
    c = np.array([(s - 1) / 2.0 for s in shape]) * (1.0 + rng.uniform(-0.1, 0.1, 3))
    x = np.arange(shape[0])[:, None, None] - c[0]
    y = np.arange(shape[1])[None, :, None] - c[1]
    z = np.arange(shape[2])[None, None, :] - c[2]
    f += amp * np.tanh((x * n[0] + y * n[1] + z * n[2]) / 2.0)
    return f.astype(np.float32)


def batch_specs(n=64, seed=104, lo=32, hi=384):
    """Shapes, spectral slopes and seeds of the uneven batch (sides uniform in [lo, hi])."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        shape = tuple(int(v) for v in rng.integers(lo, hi + 1, size=3))
        beta = float(rng.uniform(2.0, 4.0))
        out.append((shape, beta, seed * 1000 + i))
    return out


def batch_fields(n=64, seed=104, lo=32, hi=384):
    return [grf(shape, beta, s) for shape, beta, s in batch_specs(n, seed, lo, hi)]


def serving_trace(seed=105, rate=200.0, duration=10.0, side_lo=64, side_hi=512,
                  ebs=(1e-2, 1e-3, 1e-4), pool_sides=8):
    """Poisson arrivals; cube side log-uniform in volume, snapped to a pool of sides.

    Returns (arrival_times_s, sides, ebs, pool_side_list).
    """
    rng = np.random.default_rng(seed)
    t, times = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        times.append(t)
    m = len(times)
    sides = np.round(np.exp(rng.uniform(math.log(side_lo), math.log(side_hi), m))).astype(int)
    pool = np.unique(np.round(np.exp(np.linspace(math.log(side_lo), math.log(side_hi),
                                                 pool_sides))).astype(int))
    snapped = pool[np.abs(sides[:, None] - pool[None, :]).argmin(axis=1)]
    eb = rng.choice(np.asarray(ebs, dtype=np.float64), size=m)
    return np.asarray(times), snapped, eb, [int(p) for p in pool]


def multilinear(shape, scale=1) -> np.ndarray:
    """Integer multilinear field 1+2x-3y+z+xy-yz+2xz+xyz (times scale), float32.

    Every spline stencil reproduces such a field exactly along any axis; with
    |values| below 2^19 every FP32 operation on it is exact.
    """
    x = np.arange(shape[0], dtype=np.float64)[:, None, None]
    y = np.arange(shape[1], dtype=np.float64)[None, :, None]
    z = np.arange(shape[2], dtype=np.float64)[None, None, :]
    f = 1 + 2 * x - 3 * y + z + x * y - y * z + 2 * x * z + x * y * z
    f = f * scale
    if np.abs(f).max() >= 2 ** 19:
        raise ValueError("multilinear field too large for exact FP32 arithmetic")
    return f.astype(np.float32)


def random_small(shape, seed, kind="grf"):
    """Small fields for parity sweeps: a GRF, uniform noise or a constant."""
    if kind == "grf":
        return grf(shape, 3.0, seed)
    rng = np.random.default_rng(seed)
    if kind == "noise":
        return rng.uniform(-1, 1, size=shape).astype(np.float32)
    if kind == "const":
        return np.full(shape, np.float32(rng.uniform(-2, 2)), dtype=np.float32)
    raise ValueError(kind)
