"""Pins of the CPU FP64 oracle against facts it does not compute itself.

The transform is the 3D DFT taken as three 1D stages (Sec. 2, Fig. 2) with the
X stage real-to-complex and the half spectrum of (Nx+2)/2 modes kept
(Sec. 3.2, Table 1); the backward transform returns the input times a scale
factor (Sec. 4.1).  Each test below fixes the oracle's output by something
other than the oracle: brute-force sums on tiny grids, closed-form spectra,
invariants (Parseval, Hermitian planes, shift theorem, round trip) and an
independent library (numpy's pocketfft).  Together they catch a dropped term,
a wrong sign, a wrong index or a transposed axis anywhere in it.
"""
import cmath
import math

import numpy as np
import pytest

import oracle
import synth

TINY = [(5, 6, 8), (4, 9, 7), (2, 3, 5), (1, 1, 1), (2, 2, 2), (3, 1, 4), (1, 5, 3), (7, 2, 1)]
SMALL = [(8, 12, 16), (9, 10, 15), (7, 11, 13), (16, 6, 5), (12, 14, 32)]


def brute_r2c(u):
    """Literal triple sum of the definition, pure Python (tiny grids only)."""
    nz, ny, nx = u.shape
    nxh = nx // 2 + 1
    out = np.zeros((nz, ny, nxh), dtype=np.complex128)
    for kz in range(nz):
        for ky in range(ny):
            for kx in range(nxh):
                s = 0j
                for z in range(nz):
                    for y in range(ny):
                        for x in range(nx):
                            ph = -2 * math.pi * (kx * x / nx + ky * y / ny + kz * z / nz)
                            s += u[z, y, x] * cmath.exp(1j * ph)
                out[kz, ky, kx] = s
    return out


def brute_c2r(U, nx):
    """Staged backward by pure-Python sums: inverse Z and Y sums, then the 1D C2R formula."""
    nz, ny, nxh = U.shape
    T = np.zeros_like(U)
    for z in range(nz):
        for y in range(ny):
            for kx in range(nxh):
                s = 0j
                for kz in range(nz):
                    for ky in range(ny):
                        s += U[kz, ky, kx] * cmath.exp(2j * math.pi * (ky * y / ny + kz * z / nz))
                T[z, y, kx] = s
    u = np.zeros((nz, ny, nx))
    for z in range(nz):
        for y in range(ny):
            c = T[z, y]
            for x in range(nx):
                v = c[0].real
                for k in range(1, (nx - 1) // 2 + 1):
                    v += 2 * (c[k] * cmath.exp(2j * math.pi * k * x / nx)).real
                if nx % 2 == 0:
                    v += c[nx // 2].real * (-1) ** x
                u[z, y, x] = v
    return u


def rel(a, b):
    b = np.asarray(b)
    d = np.linalg.norm(np.asarray(a) - b)
    n = np.linalg.norm(b)
    return d / n if n > 0 else d


@pytest.mark.parametrize("shape", TINY)
def test_forward_matches_brute_force(shape):
    u = synth.uniform(11, shape)
    ref = brute_r2c(u)
    assert rel(oracle.r2c3d(u), ref) < 1e-13
    assert rel(oracle.r2c3d(u, engine="direct"), ref) < 1e-13


@pytest.mark.parametrize("shape", TINY)
def test_backward_matches_brute_force(shape):
    nz, ny, nx = shape
    U = synth.complex_half(12, (nz, ny, nx // 2 + 1))
    ref = brute_c2r(U, nx)
    assert rel(oracle.c2r3d(U, nx), ref) < 1e-13
    assert rel(oracle.c2r3d(U, nx, engine="direct"), ref) < 1e-13


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7, 8, 11, 12, 13, 16, 30, 49, 64, 97, 120, 210, 243, 1024])
def test_1d_engines_vs_pocketfft(n):
    x = synth.complex_half(n, (n,))
    for sign, lib in ((-1, np.fft.fft), (1, lambda v: np.fft.ifft(v) * n)):
        ref = lib(x)
        assert rel(oracle.fft1d(x, sign), ref) < 1e-13
        assert rel(oracle.dft1d(x, sign), ref) < 1e-13


@pytest.mark.parametrize("shape", SMALL + [(32, 32, 32), (25, 36, 48)])
def test_forward_vs_numpy_rfftn(shape):
    u = synth.uniform(13, shape)
    assert rel(oracle.r2c3d(u), np.fft.rfftn(u)) < 1e-13


@pytest.mark.parametrize("shape", SMALL + [(32, 32, 32)])
def test_backward_vs_numpy_irfftn(shape):
    """numpy's irfftn is C2C over (z, y) then C2R along x dropping Im of modes 0 and nx/2."""
    nz, ny, nx = shape
    U = synth.complex_half(14, (nz, ny, nx // 2 + 1))
    ref = np.fft.irfftn(U, s=shape, axes=(0, 1, 2)) * (nx * ny * nz)
    assert rel(oracle.c2r3d(U, nx), ref) < 1e-13


@pytest.mark.parametrize("shape", SMALL + [(6, 20, 15)])
def test_empty_third_transform_vs_numpy_2d(shape):
    """Empty third transform (Sec. 3.1): every z plane gets the 2D R2C over (y, x)
    and, backward, numpy's 2D inverse (C2C along y, C2R along x); z is untouched."""
    nz, ny, nx = shape
    u = synth.uniform(15, shape)
    assert rel(oracle.r2c3d_third_empty(u), np.fft.rfftn(u, axes=(1, 2))) < 1e-13
    U = synth.complex_half(16, (nz, ny, nx // 2 + 1))
    ref = np.fft.irfftn(U, s=(ny, nx), axes=(1, 2)) * (nx * ny)
    assert rel(oracle.c2r3d_third_empty(U, nx), ref) < 1e-13
    # a z-dependent input stays z-dependent in the same way: no mixing across planes
    v = np.zeros(shape)
    v[nz // 2, 0, 0] = 1.0
    V = oracle.r2c3d_third_empty(v)
    assert np.max(np.abs(V[nz // 2] - 1.0)) < 1e-14
    assert np.max(np.abs(np.delete(V, nz // 2, axis=0))) == 0.0


@pytest.mark.parametrize("nz", [2, 3, 5, 17, 33, 40])
def test_dct1_along_z_pins(nz):
    """Chebyshev third transform: scipy's type-1 DCT as an independent library;
    its own inverse up to 2 (nz - 1); a constant gives a single spike 2 (nz - 1)
    at k = 0; a point at the last Gauss-Lobatto node gives (-1)^k."""
    import scipy.fft as sf

    ny, nxh = 3, 4
    U = synth.complex_half(31 + nz, (nz, ny, nxh))
    V = oracle.stage_dct1_z(U, 2 * (nxh - 1))
    ref = sf.dct(U.real, type=1, axis=0) + 1j * sf.dct(U.imag, type=1, axis=0)
    assert rel(V, ref) < 1e-13
    assert rel(oracle.stage_dct1_z(V, 2 * (nxh - 1)), 2 * (nz - 1) * U) < 1e-13
    C = np.ones((nz, ny, nxh), dtype=np.complex128)
    D = oracle.stage_dct1_z(C, 2 * (nxh - 1))
    assert np.max(np.abs(D[0] - 2 * (nz - 1))) < 1e-12 and np.max(np.abs(D[1:])) < 1e-12
    E = np.zeros((nz, ny, nxh), dtype=np.complex128)
    E[nz - 1] = 1.0
    F = oracle.stage_dct1_z(E, 2 * (nxh - 1))
    assert np.max(np.abs(F - ((-1.0) ** np.arange(nz))[:, None, None])) < 1e-13


def test_cheb_transforms_compose_the_stages():
    """The Chebyshev-third 3D transforms are the X and Y stages followed / preceded by the DCT."""
    nz, ny, nx = 9, 6, 10
    u = synth.uniform(41, (nz, ny, nx))
    import scipy.fft as sf

    W = np.fft.rfftn(u, axes=(1, 2))
    ref = sf.dct(W.real, type=1, axis=0) + 1j * sf.dct(W.imag, type=1, axis=0)
    assert rel(oracle.r2c3d_cheb(u), ref) < 1e-13
    back = oracle.c2r3d_cheb(oracle.r2c3d_cheb(u), nx)
    assert rel(back, u * nx * ny * 2 * (nz - 1)) < 1e-13


@pytest.mark.parametrize("shape", SMALL)
def test_delta_at_origin_gives_constant_spectrum(shape):
    u = np.zeros(shape)
    u[0, 0, 0] = 1.0
    U = oracle.r2c3d(u)
    assert np.max(np.abs(U - 1.0)) < 1e-14


@pytest.mark.parametrize("shape,pos", [((8, 12, 16), (3, 5, 7)), ((9, 10, 15), (8, 1, 14)), ((7, 11, 13), (2, 10, 0))])
def test_shifted_delta_gives_pure_phase(shape, pos):
    nz, ny, nx = shape
    z0, y0, x0 = pos
    u = np.zeros(shape)
    u[z0, y0, x0] = 1.0
    U = oracle.r2c3d(u)
    kz, ky, kx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx // 2 + 1), indexing="ij")
    ph = np.exp(-2j * np.pi * (kx * x0 / nx + ky * y0 / ny + kz * z0 / nz))
    assert np.max(np.abs(U - ph)) < 1e-13


@pytest.mark.parametrize("shape", SMALL)
def test_constant_gives_single_mean_mode(shape):
    u = np.full(shape, 0.375)
    U = oracle.r2c3d(u)
    N = u.size
    assert abs(U[0, 0, 0] - 0.375 * N) < 1e-12 * N
    V = U.copy()
    V[0, 0, 0] = 0
    assert np.max(np.abs(V)) < 1e-12 * N


def _mode_field(shape, a, b, c, fn):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return fn(2 * np.pi * (a * x / nx + b * y / ny + c * z / nz))


@pytest.mark.parametrize("shape,mode", [
    ((8, 12, 16), (3, 2, 1)),   # interior kx: one spike visible in half storage
    ((9, 10, 15), (4, 3, 5)),   # odd nx, odd nz
    ((16, 6, 5), (2, 1, 7)),    # odd nx, non-cubic
    ((8, 12, 16), (0, 2, 3)),   # kx = 0: both spikes in the stored plane
    ((8, 12, 16), (8, 5, 1)),   # kx = nx/2 (Nyquist plane): both spikes stored
])
def test_cosine_and_sine_modes_give_two_spikes(shape, mode):
    nz, ny, nx = shape
    a, b, c = mode
    N = nx * ny * nz
    for fn, amp in ((np.cos, 0.5 * N), (np.sin, -0.5j * N)):
        u = _mode_field(shape, a, b, c, fn)
        U = oracle.r2c3d(u)
        E = np.zeros_like(U)
        E[c % nz, b % ny, a] += amp
        ma, mb, mc = (-a) % nx, (-b) % ny, (-c) % nz
        if ma < nx // 2 + 1:  # mirror spike also lives in the stored half
            E[mc, mb, ma] += np.conj(amp)
        assert np.max(np.abs(U - E)) < 1e-11 * N, (fn.__name__, mode)


@pytest.mark.parametrize("shape", SMALL)
def test_shift_theorem(shape):
    nz, ny, nx = shape
    u = synth.uniform(15, shape)
    s = (2, 3, 1)  # shift in (z, y, x)
    v = np.roll(u, s, axis=(0, 1, 2))
    kz, ky, kx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx // 2 + 1), indexing="ij")
    ph = np.exp(-2j * np.pi * (kx * s[2] / nx + ky * s[1] / ny + kz * s[0] / nz))
    assert rel(oracle.r2c3d(v), oracle.r2c3d(u) * ph) < 1e-13


@pytest.mark.parametrize("shape", SMALL)
def test_linearity(shape):
    a = synth.uniform(16, shape)
    b = synth.uniform(17, shape)
    lhs = oracle.r2c3d(2.5 * a - 0.75 * b)
    rhs = 2.5 * oracle.r2c3d(a) - 0.75 * oracle.r2c3d(b)
    assert rel(lhs, rhs) < 1e-14


@pytest.mark.parametrize("shape", SMALL + [(32, 32, 32)])
def test_parseval_half_spectrum(shape):
    """sum |u|^2 = (1/N) [ |U(kx=0)|^2 + 2 |U(0<kx<nx/2)|^2 + |U(kx=nx/2, even)|^2 ]."""
    nz, ny, nx = shape
    u = synth.uniform(18, shape)
    U = oracle.r2c3d(u)
    w = np.full(nx // 2 + 1, 2.0)
    w[0] = 1.0
    if nx % 2 == 0:
        w[-1] = 1.0
    e_spec = np.sum(w * np.abs(U) ** 2) / u.size
    assert abs(e_spec - np.sum(u ** 2)) < 1e-12 * np.sum(u ** 2)


@pytest.mark.parametrize("shape", SMALL + [(32, 32, 32), (1, 1, 1), (3, 1, 4)])
def test_round_trip_is_n_times_input(shape):
    u = synth.uniform(19, shape)
    back = oracle.c2r3d(oracle.r2c3d(u), shape[2])
    assert rel(back, u.size * u) < 1e-14


@pytest.mark.parametrize("shape", SMALL)
def test_hermitian_planes(shape):
    """kx = 0 and (even nx) kx = nx/2 planes satisfy U[kz,ky] = conj(U[-kz,-ky])."""
    nz, ny, nx = shape
    U = oracle.r2c3d(synth.uniform(20, shape))
    planes = [0] + ([nx // 2] if nx % 2 == 0 else [])
    iz = (-np.arange(nz)) % nz
    iy = (-np.arange(ny)) % ny
    for p in planes:
        P = U[:, :, p]
        assert np.max(np.abs(P - np.conj(P[iz][:, iy]))) < 1e-12 * np.max(np.abs(P))
    # self-conjugate points are real
    for kz in {0, nz // 2} if nz % 2 == 0 else {0}:
        for ky in {0, ny // 2} if ny % 2 == 0 else {0}:
            for p in planes:
                assert abs(U[kz, ky, p].imag) < 1e-12 * np.max(np.abs(U))


def test_backward_of_single_mode_is_cosine():
    shape = (8, 12, 16)
    nz, ny, nx = shape
    a, b, c = 3, 2, 5
    U = np.zeros((nz, ny, nx // 2 + 1), dtype=np.complex128)
    U[c, b, a] = 1.0
    u = oracle.c2r3d(U, nx)
    assert np.max(np.abs(u - 2 * _mode_field(shape, a, b, c, np.cos))) < 1e-13


def test_backward_drops_imaginary_of_real_modes():
    """Staged C2R along X uses only Re of modes 0 and nx/2 of each line."""
    nz, ny, nx = 4, 6, 8
    U = np.zeros((nz, ny, nx // 2 + 1), dtype=np.complex128)
    U[0, 0, 0] = 1.0 + 5.0j
    U[0, 0, nx // 2] = 2.0 - 3.0j
    u = oracle.c2r3d(U, nx)
    x = np.arange(nx)
    expect = (1.0 + 2.0 * (-1.0) ** x)[None, None, :] * np.ones((nz, ny, 1))
    assert np.max(np.abs(u - expect)) < 1e-14


def test_stride1_permutation_is_table1_zyx():
    U = oracle.r2c3d(synth.uniform(21, (5, 6, 8)))
    Z = oracle.to_stride1(U)
    assert Z.shape == (5, 6, 5)
    assert Z[3, 4, 2] == U[2, 4, 3]
    assert np.array_equal(oracle.from_stride1(Z), U)


@pytest.mark.parametrize("shape", [(12, 10, 16), (9, 14, 15)])
def test_sampled_points_and_lines_match_whole_transform(shape):
    nz, ny, nx = shape
    u = synth.uniform(22, shape).astype(np.float32)
    U = oracle.r2c3d(u)
    ky = np.array([0, 1, ny - 1, ny // 2])
    kz = np.array([0, nz - 1, 2, nz // 2])
    for kx in (0, 1, nx // 2):
        pts = oracle.r2c_points(u, kx, ky, kz)
        assert rel(pts, U[kz, ky, kx]) < 1e-13
    V = synth.complex_half(23, (nz, ny, nx // 2 + 1)).astype(np.complex64)
    full = oracle.c2r3d(V, nx)
    for (y0, z0) in ((0, 0), (ny - 1, nz - 1), (3, 5)):
        assert rel(oracle.c2r_line(V, nx, y0, z0), full[z0, y0]) < 1e-13


def test_float32_input_is_promoted_exactly():
    u = synth.uniform(24, (6, 7, 10)).astype(np.float32)
    assert np.array_equal(oracle.r2c3d(u), oracle.r2c3d(u.astype(np.float64)))


@pytest.mark.parametrize("shape", [(5, 6, 8), (4, 9, 7)])
def test_stages_compose_to_the_whole_transform(shape):
    """X stage, then Y, then Z (Sec. 2) equals the brute-force 3D sum; the backward stages likewise."""
    nz, ny, nx = shape
    u = synth.uniform(25, shape)
    A = oracle.stage_x_r2c(u)
    assert rel(A, np.fft.rfft(u, axis=2)) < 1e-13
    A = oracle.stage_c2c(A, nx, "y", -1)
    A = oracle.stage_c2c(A, nx, "z", -1)
    assert rel(A, brute_r2c(u)) < 1e-13
    U = synth.complex_half(26, (nz, ny, nx // 2 + 1))
    B = oracle.stage_c2c(oracle.stage_c2c(U, nx, "z", +1), nx, "y", +1)
    assert rel(oracle.stage_x_c2r(B, nx), brute_c2r(U, nx)) < 1e-13


def test_cheb_composition_with_the_spectral_multiplier_has_the_closed_form():
    """The reference the spectral-step tests build from the oracle (Chebyshev
    forward, the multiplier m = i kx' (-1/|k'|^2) / (nx ny 2 (nz - 1)), Chebyshev
    backward) reproduces the analytic result on a single mode:
    cos(2 pi k0 x / nx) cos(pi q0 z / (nz - 1)) maps to
    kx' / (kx'^2 + kz'^2) sin(2 pi k0 x / nx) cos(pi q0 z / (nz - 1))."""
    for (nz, ny, nx), k0, q0 in (((17, 8, 16), 3, 5), ((9, 6, 10), 2, 0), ((12, 4, 15), 7, 11)):
        kxs = 2 * np.pi * np.arange(nx // 2 + 1) / nx
        kys = 2 * np.pi * np.fft.fftfreq(ny, 1.0 / ny) / ny
        kzs = np.pi * np.arange(nz) / (nz - 1)
        k2 = kxs[None, None, :] ** 2 + kys[None, :, None] ** 2 + kzs[:, None, None] ** 2
        with np.errstate(divide="ignore", invalid="ignore"):
            m = 1j * np.where(k2 > 0, -kxs[None, None, :] / k2, 0.0) / (nx * ny * 2.0 * (nz - 1))
        x = np.arange(nx)[None, None, :]
        z = np.arange(nz)[:, None, None]
        u = np.cos(2 * np.pi * k0 * x / nx) * np.cos(np.pi * q0 * z / (nz - 1)) * np.ones((1, ny, 1))
        kx, kz = 2 * np.pi * k0 / nx, np.pi * q0 / (nz - 1)
        want = kx / (kx * kx + kz * kz) * np.sin(2 * np.pi * k0 * x / nx) * np.cos(np.pi * q0 * z / (nz - 1)) \
            * np.ones((1, ny, 1))
        got = oracle.c2r3d_cheb(oracle.r2c3d_cheb(u) * m, nx)
        assert rel(got, want) < 1e-13, ((nz, ny, nx), k0, q0)
