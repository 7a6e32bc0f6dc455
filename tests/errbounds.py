"""Error bounds for parts of a transform's output (test helpers, no GPU).

A staged 3D transform (three passes of 1D transforms, Sec. 2) rounds in each
pass.  A pass's rounding errors on one line are of the size of the unit
roundoff times that line's norm and are spread evenly over the outputs of the
line, and the outputs of the last pass carry one more rounding relative to
their own size.  With the passes along axes a1, a2, a3 (in order) and n
outputs, the expected squared error of output k is therefore about eps^2
times

    M(k) = ||A||^2 / n                               (first pass, spread over everything)
         + ||A[k_a1 = k_a1(k)]||^2 / (n_a2 n_a3)     (second pass, spread over the a1-slice)
         + ||A[k_a1, k_a2 = ...]||^2 / n_a3          (last pass, spread over the line)
         + |A(k)|^2                                  (the last rounding of the output itself)

where the bracketed norms are over the slice of the result that shares the
indices named.  Summed over all outputs the four terms give 4 ||A||^2, so with
eps = tol / 2 the bound for a subset S of the outputs,

    ||e_S||  <=  (tol / 2) sqrt(sum_{k in S} M(k)),

is consistent with the whole-result bound ||e|| <= tol ||A|| of the precision.
It is asserted for each |k| shell of a power-law field (whose energy falls
off with |k|, so a single whole-result norm would hide the weak shells) and
for the block of one rank of a share-only transform.
"""
import math

import numpy as np


def staged_floor(A, axes):
    """M(k) of the module docstring for a whole result A whose passes ran along axes (a1, a2, a3)."""
    a1, a2, a3 = axes
    r2 = np.abs(np.asarray(A)).astype(np.float64) ** 2
    n = r2.size
    total = r2.sum()
    plane = r2.sum(axis=(a2, a3), keepdims=True) / (r2.shape[a2] * r2.shape[a3])
    line = r2.sum(axis=a3, keepdims=True) / r2.shape[a3]
    return (total / n + plane + line + r2) / 4.0


def check_subset(err_sq, floor_sum, tol):
    """Assert sqrt(err_sq) <= tol sqrt(floor_sum) (floor_sum = sum of M over the subset, already / 4)."""
    bound = tol * math.sqrt(floor_sum)
    e = math.sqrt(err_sq)
    assert e <= bound, (e, bound)
    return e, bound


def shell_edges(n):
    """|k| shell edges 0, 1, 2, 4, ..., n/2, inf for a grid of edge about n (the first shell is mode 0)."""
    return [0.0] + [2.0 ** j for j in range(0, max(1, int(math.log2(max(n, 2)))))] + [math.inf]


def check_shells(got, ref, nx, ny, nz, tol):
    """Every |k| shell of a STRIDE1 forward result [kx][ky][kz] (passes X, Y, Z) within its staged bound.

    Computed plane by plane in FP64.  Returns rows (k_lo, k_hi, modes, rel L2 error, rel bound).
    """
    edges = shell_edges(max(nx, ny, nz))
    nb = len(edges) - 1
    ky = np.fft.fftfreq(ny, 1.0 / ny)
    kz = np.fft.fftfreq(nz, 1.0 / nz)
    k2 = ky[:, None] ** 2 + kz[None, :] ** 2
    nxh = got.shape[0]
    n = nxh * ny * nz
    total = sum(float((np.abs(ref[kx]) ** 2).sum()) for kx in range(nxh))
    num, den, flo, cnt = (np.zeros(nb) for _ in range(4))
    for kx in range(nxh):
        r2 = np.abs(ref[kx]) ** 2
        e2 = np.abs(got[kx].astype(np.complex128) - ref[kx]) ** 2
        m = (total / n + r2.sum() / (ny * nz) + r2.sum(axis=1, keepdims=True) / nz + r2) / 4.0
        b = (np.digitize(np.sqrt(kx * kx + k2), edges) - 1).ravel()
        num += np.bincount(b, weights=e2.ravel(), minlength=nb)[:nb]
        den += np.bincount(b, weights=r2.ravel(), minlength=nb)[:nb]
        flo += np.bincount(b, weights=m.ravel(), minlength=nb)[:nb]
        cnt += np.bincount(b, minlength=nb)[:nb]
    rows = []
    for i in range(nb):
        if cnt[i] == 0:
            continue
        e, bound = check_subset(num[i], flo[i], tol)
        r = math.sqrt(den[i]) if den[i] > 0 else float("nan")
        rows.append((edges[i], edges[i + 1], int(cnt[i]), e / r, bound / r))
    return rows
