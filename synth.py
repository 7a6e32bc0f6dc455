"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module makes data only: it holds none of the transform's arithmetic and
imports neither the oracle nor the HIP library.  The paper's benchmark fills a
3D array synthetically and checks the round trip (Sec. 4.1); no dataset is
involved.  Every array is C order [nz][ny][nx] (Fortran "XYZ", Table 1).

Recipes (stated again in the design notes):

* ``uniform(seed, shape)``: i.i.d. uniform[-1, 1], float64 (cast by the caller).
* ``grf(seed, shape)``: a real Gaussian random field whose shell energy spectrum
  falls as |k|^(-5/3) (turbulence-like), i.e. modal amplitude |k|^(-11/6).  The
  half spectrum is drawn directly as complex Gaussian noise times that
  amplitude (mode 0 set to zero) and taken to real space with scipy's inverse
  real FFT (a third-party library used only to shape the data), then scaled to
  unit standard deviation.  float32.
* ``complex_half(seed, shape)``: i.i.d. uniform[-1, 1] real and imaginary parts,
  an arbitrary (not Hermitian-consistent) half spectrum for backward tests.
* ``index_field(shape)``: value = linear index, for bitwise permutation tests.
* ``batch_sizes(seed, count)``: 7-smooth lengths in [48, 320] for batched runs.

Large draws are split into fixed chunks, each with its own generator seeded
by (seed, chunk), so results do not depend on the thread count.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_CHUNK = 1 << 24  # elements per independently seeded chunk


def _workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _fill(seed: int, out: np.ndarray, kind: str, tag: int) -> None:
    """Fill a contiguous array chunk-by-chunk from generators seeded (seed, tag, chunk)."""
    flat = out.reshape(-1)
    nchunks = (flat.size + _CHUNK - 1) // _CHUNK

    def work(c: int) -> None:
        g = np.random.default_rng([seed, tag, c])
        seg = flat[c * _CHUNK:(c + 1) * _CHUNK]
        if kind == "normal":
            g.standard_normal(out=seg, dtype=seg.dtype)
        else:
            seg[...] = g.uniform(-1.0, 1.0, seg.size)

    if nchunks <= 1:
        for c in range(nchunks):
            work(c)
    else:
        with ThreadPoolExecutor(_workers()) as ex:
            list(ex.map(work, range(nchunks)))


def uniform(seed: int, shape, dtype=np.float64) -> np.ndarray:
    """i.i.d. uniform[-1, 1] real field [nz][ny][nx]."""
    if int(np.prod(shape)) <= _CHUNK:
        return np.random.default_rng(seed).uniform(-1.0, 1.0, shape).astype(dtype, copy=False)
    out = np.empty(shape, dtype=np.float64)
    _fill(seed, out, "uniform", 0)
    return out.astype(dtype, copy=False)


def complex_half(seed: int, shape, dtype=np.complex128) -> np.ndarray:
    """i.i.d. uniform[-1, 1] real and imaginary parts, shape [nz][ny][nxh]."""
    re = uniform(seed, shape)
    im = uniform(seed + 7919, shape)
    out = np.empty(shape, dtype=dtype)
    out.real = re
    out.imag = im
    return out


def grf(seed: int, shape, slope: float = -11.0 / 6.0) -> np.ndarray:
    """Gaussian random field, modal amplitude |k|^slope (shell spectrum |k|^-5/3), float32, std 1."""
    import scipy.fft as sfft

    nz, ny, nx = shape
    nxh = nx // 2 + 1
    spec = np.empty((nz, ny, nxh), dtype=np.complex64)
    re = np.empty((nz, ny, nxh), dtype=np.float32)
    _fill(seed, re, "normal", 1)
    spec.real = re
    _fill(seed, re, "normal", 2)
    spec.imag = re
    del re
    kx2 = np.arange(nxh, dtype=np.float64) ** 2
    ky2 = (np.fft.fftfreq(ny) * ny) ** 2
    kz = np.fft.fftfreq(nz) * nz
    for z in range(nz):  # plane by plane keeps the float64 temporaries small
        k2 = kz[z] ** 2 + ky2[:, None] + kx2[None, :]
        with np.errstate(divide="ignore"):
            amp = np.where(k2 > 0, k2 ** (0.5 * slope), 0.0)
        spec[z] *= amp.astype(np.float32)
    u = sfft.irfftn(spec, s=(nz, ny, nx), axes=(0, 1, 2), workers=_workers(), overwrite_x=True)
    del spec
    u = np.ascontiguousarray(u, dtype=np.float32)
    sd = float(u.std(dtype=np.float64))
    if sd > 0:
        u /= np.float32(sd)
    return u


def index_field(shape, dtype=np.float32) -> np.ndarray:
    """value = C-order linear index (exact in float32 below 2**24 elements)."""
    return np.arange(int(np.prod(shape)), dtype=np.float64).reshape(shape).astype(dtype)


def smooth7(lo: int = 48, hi: int = 320):
    """All lengths in [lo, hi] whose prime factors are in {2, 3, 5, 7}."""
    out = []
    for n in range(lo, hi + 1):
        m = n
        for p in (2, 3, 5, 7):
            while m % p == 0:
                m //= p
        if m == 1:
            out.append(n)
    return out


def batch_sizes(seed: int = 4, count: int = 64):
    """count (nx, ny, nz) triples drawn uniformly from the 7-smooth lengths in [48, 320]."""
    s = np.array(smooth7())
    return [tuple(int(v) for v in row) for row in np.random.default_rng(seed).choice(s, (count, 3))]
