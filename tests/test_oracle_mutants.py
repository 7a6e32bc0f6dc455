"""The oracle's pins catch plausible mistakes planted in a copy of the oracle.

Each mutant is oracle.c with one textual change (a dropped term, a flipped
sign, a wrong index, a swapped axis, a lost Nyquist mode), compiled with gcc
into a temporary directory and bound in place of the real library for the
duration of one check.  The pin checks here are the closed forms and
brute-force sums of test_oracle_pins.py in compact form; every mutant must
fail at least one of them, and the unmutated source must pass them all.
CPU only.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
import synth
from tests.test_oracle_pins import brute_c2r, brute_r2c, rel

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTANTS = {
    "combine_sign": ("sr += a.re * w[r].re - a.im * w[r].im;\n                si += a.re * w[r].im + a.im * w[r].re;\n            }\n            scratch",
                     "sr += a.re * w[r].re + a.im * w[r].im;\n                si += -a.re * w[r].im + a.im * w[r].re;\n            }\n            scratch"),
    "dropped_term": ("for (int q = 0; q < p; ++q) {\n                long r", "for (int q = 0; q < p - (n > 4); ++q) {\n                long r"),
    "wrong_twiddle_index": ("long r = (((long)q * kk) % n) * step;", "long r = (((long)q * k) % n) * step;"),
    "roots_off_by_one": ("double a = TWO_PI * (double)r / (double)n;", "double a = TWO_PI * (double)r / (double)(n + (n > 2));"),
    "y_pass_wrong_stride": ("for (int y = 0; y < ny; ++y) a[y] = base[(long)y * nc];",
                            "for (int y = 0; y < ny; ++y) a[y] = base[(long)y * (nc > 1 ? nc - 1 : 1)];"),
    "z_pass_skipped_sign": ("return pass_z(engine, nxh, ny, nz, U, -1);", "return pass_z(engine, nxh, ny, nz, U, +1);"),
    "c2r_conj_missing": ("F[nx - k].im = -c[k].im;", "F[nx - k].im = c[k].im;"),
    "c2r_nyquist_lost": ("if (nx % 2 == 0) F[nx / 2].re = c[nx / 2].re;", "if (nx % 2 == 0) F[nx / 2].re = 0.0;"),
    "c2r_dc_counted_twice": ("F[0].re = c[0].re;", "F[0].re = 2.0 * c[0].re;"),
    "forward_keeps_too_few": ("memcpy(U + L * nxh, b, sizeof(cplx) * (size_t)nxh);",
                              "memcpy(U + L * nxh, b, sizeof(cplx) * (size_t)(nxh - 1));"),
    "backward_y_sign": ("if (!err) err = pass_y(engine, nxh, ny, nz, T, +1);", "if (!err) err = pass_y(engine, nxh, ny, nz, T, -1);"),
    "dct_end_node_sign": ("const double sg = (k % 2 == 0) ? 1.0 : -1.0;", "const double sg = 1.0;"),
    "dct_interior_weight": ("const double w = 2.0 * c[((long)j * k) % L];", "const double w = c[((long)j * k) % L];"),
}


def pins_pass() -> bool:
    """Compact pin suite: brute force, closed forms, Parseval, round trip."""
    try:
        for shape in ((5, 6, 8), (4, 9, 7), (3, 5, 6)):
            nz, ny, nx = shape
            u = synth.uniform(31, shape)
            if rel(oracle.r2c3d(u), brute_r2c(u)) > 1e-12:
                return False
            U = synth.complex_half(32, (nz, ny, nx // 2 + 1))
            if rel(oracle.c2r3d(U, nx), brute_c2r(U, nx)) > 1e-12:
                return False
        shape = (8, 12, 16)
        u = np.zeros(shape)
        u[0, 0, 0] = 1.0
        if np.max(np.abs(oracle.r2c3d(u) - 1.0)) > 1e-12:
            return False
        u = synth.uniform(33, (12, 10, 16))
        if rel(oracle.c2r3d(oracle.r2c3d(u), 16), u.size * u) > 1e-12:
            return False
        # Chebyshev third transform: its own inverse up to 2 (nz - 1); constant -> one spike
        U = synth.complex_half(34, (9, 3, 4))
        if rel(oracle.stage_dct1_z(oracle.stage_dct1_z(U, 6), 6), 16 * U) > 1e-12:
            return False
        D = oracle.stage_dct1_z(np.ones((9, 3, 4), dtype=np.complex128), 6)
        if np.max(np.abs(D[0] - 16)) > 1e-12 or np.max(np.abs(D[1:])) > 1e-12:
            return False
    except Exception:
        return False
    return True


def _build_mutant(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(old, new, 1))
    so = tmp_path / f"lib{name}.so"
    subprocess.run(["gcc", "-O1", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", str(so), str(path), "-lm"],
                   check=True)
    return oracle.bind(ctypes.CDLL(str(so)))


def test_unmutated_oracle_passes_compact_pins():
    assert pins_pass()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, monkeypatch, name):
    old, new = MUTANTS[name]
    lib = _build_mutant(tmp_path, name, old, new)
    monkeypatch.setattr(oracle, "_lib", lib)
    assert not pins_pass(), f"planted mistake {name} went unnoticed"
