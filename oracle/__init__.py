"""CPU FP64 oracle for the pencil 3D R2C / C2R transform (arXiv:1905.02803).

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke check
and the CPU-baseline leg of the benchmark may import this package.  It shares
no code with the HIP library (``paper_1905_02803_amd``) and never imports it.

What it computes (Sec. 2 and Fig. 2: three 1D transform stages, X then Y then
Z; Sec. 3.2 and Table 1: real X-pencil input, half-spectrum output of
(Nx+2)/2 complex modes along X in integer division):

* ``r2c3d(u)``: U[kz, ky, kx] = sum u[z, y, x] exp(-2 pi i (kx x/Nx + ky y/Ny +
  kz z/Nz)) for kx <= Nx/2, returned as a C array [nz][ny][nxh] (the paper's
  "STRIDE1 undefined" Z-pencil order, Fortran XYZ).  ``to_stride1`` permutes it
  to the "STRIDE1 defined" Z-pencil order (Fortran ZYX = C [nxh][ny][nz]).
* ``c2r3d(U, nx)``: the staged backward transform -- inverse unnormalised C2C
  along Z, then Y, then the 1D C2R along X that keeps only Re of mode 0 and,
  for even Nx, of mode Nx/2 (Sec. 3.2).  ``c2r3d(r2c3d(u)) == Nx*Ny*Nz * u``
  (Sec. 4.1: the round trip returns the input up to a scale factor).
* ``r2c_points`` / ``c2r_line``: single outputs of the same transforms by direct
  separable sums, for grids too large to transform whole on the host.

All arithmetic is FP64 in ``oracle.c`` (plain C, OpenMP over independent
lines).  Float32 inputs are promoted exactly.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (FP64, -O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def build_sanitized(path: str) -> str:
    """Compile oracle.c with AddressSanitizer and UndefinedBehaviorSanitizer into `path` (a test build:
    load it with the sanitizer runtime preloaded, through ORACLE_LIB)."""
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall", "-o", path,
           _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return path


def _load():
    global _lib
    if _lib is None:
        alt = os.environ.get("ORACLE_LIB")  # another build of oracle.c (the sanitizer test's)
        if alt:
            _lib = bind(ctypes.CDLL(alt))
        else:
            build()
            _lib = bind(ctypes.CDLL(_LIB_PATH))
    return _lib


def bind(lib):
    """Declare the C signatures on a loaded copy of the oracle library."""
    lib.oracle_num_threads.restype = ctypes.c_int
    for name in ("oracle_dft1d", "oracle_fft1d"):
        f = getattr(lib, name)
        f.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_int]
        f.restype = ctypes.c_int
    for name in ("oracle_r2c3d_ex", "oracle_c2r3d_ex"):
        f = getattr(lib, name)
        f.argtypes = [ctypes.c_int] * 4 + [ctypes.c_void_p, ctypes.c_int, _dp]
        f.restype = ctypes.c_int
    lib.oracle_r2c_points.argtypes = [ctypes.c_int] * 3 + [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                                          ctypes.c_int, _ip, _ip, _dp]
    lib.oracle_r2c_points.restype = ctypes.c_int
    lib.oracle_c2r_line.argtypes = [ctypes.c_int] * 3 + [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                                        ctypes.c_int, _dp]
    lib.oracle_c2r_line.restype = ctypes.c_int
    for name in ("oracle_stage_x_r2c", "oracle_stage_x_c2r"):
        f = getattr(lib, name)
        f.argtypes = [ctypes.c_int] * 3 + [ctypes.c_void_p, ctypes.c_int, _dp]
        f.restype = ctypes.c_int
    lib.oracle_stage_c2c.argtypes = [ctypes.c_int] * 3 + [_dp, ctypes.c_int, ctypes.c_int]
    lib.oracle_stage_c2c.restype = ctypes.c_int
    lib.oracle_stage_dct1_z.argtypes = [ctypes.c_int] * 3 + [_dp]
    lib.oracle_stage_dct1_z.restype = ctypes.c_int
    return lib


def num_threads() -> int:
    """Threads the oracle's OpenMP loops use (OMP_NUM_THREADS or all cores)."""
    return int(_load().oracle_num_threads())


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def _c128(x) -> np.ndarray:
    return np.ascontiguousarray(x, dtype=np.complex128)


def _real_in(u: np.ndarray):
    """Real input as float32 or float64, C-contiguous; returns (array, is_f32)."""
    u = np.asarray(u)
    if u.dtype == np.float32:
        return np.ascontiguousarray(u), 1
    return np.ascontiguousarray(u, dtype=np.float64), 0


def _cplx_in(U: np.ndarray):
    U = np.asarray(U)
    if U.dtype == np.complex64:
        return np.ascontiguousarray(U), 1
    return np.ascontiguousarray(U, dtype=np.complex128), 0


def dft1d(x, sign: int = -1) -> np.ndarray:
    """Direct DFT of one line: out[k] = sum_j x[j] exp(sign 2 pi i j k / n)."""
    x = _c128(x).reshape(-1)
    out = np.empty_like(x)
    _check(_load().oracle_dft1d(x.size, x.view(np.float64).ctypes.data_as(_dp),
                                out.view(np.float64).ctypes.data_as(_dp), int(sign)), "dft1d")
    return out


def fft1d(x, sign: int = -1) -> np.ndarray:
    """Recursive mixed-radix FFT of one line (same definition as dft1d)."""
    x = _c128(x).reshape(-1)
    out = np.empty_like(x)
    _check(_load().oracle_fft1d(x.size, x.view(np.float64).ctypes.data_as(_dp),
                                out.view(np.float64).ctypes.data_as(_dp), int(sign)), "fft1d")
    return out


def r2c3d(u: np.ndarray, engine: str = "fft") -> np.ndarray:
    """Forward 3D R2C of real u[nz][ny][nx] -> complex128 U[nz][ny][nx//2+1].

    engine "fft" (recursive mixed radix) or "direct" (dense DFT per axis).
    """
    u, is32 = _real_in(u)
    if u.ndim != 3:
        raise ValueError("u must be 3D [nz][ny][nx]")
    nz, ny, nx = u.shape
    U = np.empty((nz, ny, nx // 2 + 1), dtype=np.complex128)
    eng = {"direct": 0, "fft": 1}[engine]
    _check(_load().oracle_r2c3d_ex(eng, nx, ny, nz, u.ctypes.data, is32,
                                   U.view(np.float64).ctypes.data_as(_dp)), "r2c3d")
    return U


def c2r3d(U: np.ndarray, nx: int, engine: str = "fft") -> np.ndarray:
    """Staged backward 3D C2R of U[nz][ny][nx//2+1] -> float64 u[nz][ny][nx]."""
    U, is32 = _cplx_in(U)
    if U.ndim != 3 or U.shape[2] != nx // 2 + 1:
        raise ValueError("U must be [nz][ny][nx//2+1]")
    nz, ny, _ = U.shape
    u = np.empty((nz, ny, nx), dtype=np.float64)
    eng = {"direct": 0, "fft": 1}[engine]
    _check(_load().oracle_c2r3d_ex(eng, nx, ny, nz, U.ctypes.data, is32,
                                   u.ctypes.data_as(_dp)), "c2r3d")
    return u


def stage_x_r2c(u: np.ndarray) -> np.ndarray:
    """The X stage alone: 1D R2C of every line of u[nz][ny][nx] -> [nz][ny][nxh]."""
    u, is32 = _real_in(u)
    nz, ny, nx = u.shape
    U = np.empty((nz, ny, nx // 2 + 1), dtype=np.complex128)
    _check(_load().oracle_stage_x_r2c(nx, ny, nz, u.ctypes.data, is32, U.view(np.float64).ctypes.data_as(_dp)),
           "stage_x_r2c")
    return U


def stage_c2c(U: np.ndarray, nx: int, axis: str, sign: int) -> np.ndarray:
    """One C2C stage along "y" or "z" of a copy of U[nz][ny][nxh] (sign -1 forward, +1 backward)."""
    V = _c128(U).copy()
    nz, ny, _ = V.shape
    ax = {"y": 1, "z": 2}[axis]
    _check(_load().oracle_stage_c2c(nx, ny, nz, V.view(np.float64).ctypes.data_as(_dp), ax, int(sign)),
           "stage_c2c")
    return V


def stage_x_c2r(U: np.ndarray, nx: int) -> np.ndarray:
    """The X stage of the backward transform alone: 1D C2R of every line of U[nz][ny][nxh]."""
    U, is32 = _cplx_in(U)
    nz, ny, _ = U.shape
    u = np.empty((nz, ny, nx), dtype=np.float64)
    _check(_load().oracle_stage_x_c2r(nx, ny, nz, U.ctypes.data, is32, u.ctypes.data_as(_dp)), "stage_x_c2r")
    return u


def r2c3d_third_empty(u: np.ndarray) -> np.ndarray:
    """Forward transform with an empty third transform (Sec. 3.1): the X stage
    (R2C) then the Y stage (C2C, sign -1), z left untransformed -> [nz][ny][nxh]."""
    nx = np.asarray(u).shape[2]
    return stage_c2c(stage_x_r2c(u), nx, "y", -1)


def c2r3d_third_empty(U: np.ndarray, nx: int) -> np.ndarray:
    """Backward transform with an empty third transform: the Y stage (C2C,
    sign +1) then the staged 1D C2R along X -> real [nz][ny][nx]."""
    return stage_x_c2r(stage_c2c(U, nx, "y", +1), nx)


def stage_dct1_z(U: np.ndarray, nx: int) -> np.ndarray:
    """Type-I DCT (unnormalised, Gauss-Lobatto points) along z of a copy of U[nz][ny][nxh]."""
    V = _c128(U).copy()
    nz, ny, _ = V.shape
    _check(_load().oracle_stage_dct1_z(nx, ny, nz, V.view(np.float64).ctypes.data_as(_dp)), "stage_dct1_z")
    return V


def r2c3d_cheb(u: np.ndarray) -> np.ndarray:
    """Forward transform with the Chebyshev third transform (Sec. 3.1): X R2C,
    Y C2C (sign -1), then the type-I DCT along z -> [nz][ny][nxh]."""
    nx = np.asarray(u).shape[2]
    return stage_dct1_z(stage_c2c(stage_x_r2c(u), nx, "y", -1), nx)


def c2r3d_cheb(U: np.ndarray, nx: int) -> np.ndarray:
    """Backward transform with the Chebyshev third transform: type-I DCT along
    z (its own inverse up to 2 (nz - 1)), Y C2C (sign +1), staged C2R along X."""
    return stage_x_c2r(stage_c2c(stage_dct1_z(U, nx), nx, "y", +1), nx)


def to_stride1(U: np.ndarray) -> np.ndarray:
    """[nz][ny][nxh] (Fortran XYZ) -> [nxh][ny][nz] (Fortran ZYX), Table 1."""
    return np.ascontiguousarray(np.asarray(U).transpose(2, 1, 0))


def from_stride1(Z: np.ndarray) -> np.ndarray:
    """[nxh][ny][nz] -> [nz][ny][nxh]; inverse of to_stride1."""
    return np.ascontiguousarray(np.asarray(Z).transpose(2, 1, 0))


def r2c_points(u: np.ndarray, kx: int, ky, kz) -> np.ndarray:
    """Exact forward values U[kz[i], ky[i], kx] by direct separable sums (O(N) + O(ny nz) each)."""
    u, is32 = _real_in(u)
    nz, ny, nx = u.shape
    ky = np.ascontiguousarray(ky, dtype=np.int32).reshape(-1)
    kz = np.ascontiguousarray(kz, dtype=np.int32).reshape(-1)
    if ky.size != kz.size:
        raise ValueError("ky and kz must have equal length")
    out = np.empty(ky.size, dtype=np.complex128)
    _check(_load().oracle_r2c_points(nx, ny, nz, u.ctypes.data, is32, int(kx), ky.size,
                                     ky.ctypes.data_as(_ip), kz.ctypes.data_as(_ip),
                                     out.view(np.float64).ctypes.data_as(_dp)), "r2c_points")
    return out


def c2r_line(U: np.ndarray, nx: int, y0: int, z0: int) -> np.ndarray:
    """Exact staged-C2R output line u[z0, y0, :] from the half spectrum U[nz][ny][nxh]."""
    U, is32 = _cplx_in(U)
    nz, ny, nxh = U.shape
    if nxh != nx // 2 + 1:
        raise ValueError("U must be [nz][ny][nx//2+1]")
    out = np.empty(nx, dtype=np.float64)
    _check(_load().oracle_c2r_line(nx, ny, nz, U.ctypes.data, is32, int(y0), int(z0),
                                   out.ctypes.data_as(_dp)), "c2r_line")
    return out
