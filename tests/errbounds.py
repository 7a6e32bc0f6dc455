"""Error bounds for parts of a transform's output (test helpers, no GPU).

The rounding error of a floating-point FFT is spread evenly over its outputs:
every butterfly stage adds errors of the size of the unit roundoff times the
magnitudes it combines, and the later stages mix them over all frequencies, so
the error of a 3D transform is close to white noise of total norm
tol * ||U|| (the whole-result bound of the precision).  A subset S of n_S of
the n outputs then carries an error of norm about tol * ||U|| * sqrt(n_S / n),
and relative to the subset's own norm

    ||e_S|| / ||U_S||  <=  tol * sqrt(n_S / n) * ||U|| / ||U_S||.

This is the bound asserted for a rank's block of a share-only transform and
for each |k| shell of a power-law field, whose energy falls off with |k| while
the rounding error does not.
"""
import math

import numpy as np


def white_floor_bound(tol, n_part, n_whole, norm_whole, norm_part):
    """Largest relative L2 error of a subset of n_part of n_whole outputs under a white error floor."""
    return tol * math.sqrt(n_part / n_whole) * norm_whole / norm_part


def rel_l2(got, ref):
    got = np.asarray(got)
    ref = np.asarray(ref)
    return float(np.linalg.norm((got - ref).ravel()) / np.linalg.norm(ref.ravel()))


def shell_edges(n):
    """|k| shell edges 0, 1, 2, 4, ..., n/2, inf for a grid of edge about n."""
    return [0.0] + [2.0 ** j for j in range(0, max(1, int(math.log2(max(n, 2)))))] + [math.inf]


def shell_errors(got, ref, nx, ny, nz):
    """Per-|k|-shell error of a STRIDE1 half spectrum [kx][ky][kz] (got, ref) of an nx x ny x nz grid.

    Returns a list of (k_lo, k_hi, modes, err_norm, ref_norm) and the whole (err_norm, ref_norm, modes).
    |k| uses integer wavenumbers (ky, kz signed).  Computed plane by plane in FP64.
    """
    edges = shell_edges(max(nx, ny, nz))
    ky = np.fft.fftfreq(ny, 1.0 / ny)
    kz = np.fft.fftfreq(nz, 1.0 / nz)
    k2 = ky[:, None] ** 2 + kz[None, :] ** 2
    nb = len(edges) - 1
    num = np.zeros(nb)
    den = np.zeros(nb)
    cnt = np.zeros(nb)
    for kx in range(got.shape[0]):
        e2 = np.abs(got[kx].astype(np.complex128) - ref[kx]) ** 2
        r2 = np.abs(ref[kx]) ** 2
        b = (np.digitize(np.sqrt(kx * kx + k2), edges) - 1).ravel()
        num += np.bincount(b, weights=e2.ravel(), minlength=nb)[:nb]
        den += np.bincount(b, weights=r2.ravel(), minlength=nb)[:nb]
        cnt += np.bincount(b, minlength=nb)[:nb]
    shells = [(edges[i], edges[i + 1], int(cnt[i]), math.sqrt(num[i]), math.sqrt(den[i])) for i in range(nb)]
    return shells, (math.sqrt(num.sum()), math.sqrt(den.sum()), int(cnt.sum()))


def check_shells(got, ref, nx, ny, nz, tol):
    """Assert every |k| shell's relative error against the white-floor bound; returns the table."""
    shells, (_, whole, n) = shell_errors(got, ref, nx, ny, nz)
    rows = []
    for lo, hi, m, e, r in shells:
        if m == 0 or r == 0.0:
            continue
        bound = white_floor_bound(tol, m, n, whole, r)
        rows.append((lo, hi, m, e / r, bound))
        assert e / r <= bound, (lo, hi, m, e / r, bound)
    return rows
