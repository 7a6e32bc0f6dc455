"""Share-only plans: one rank's local stages at its Table 1 shapes (Sec. 2, 3.2).

Rank (r1, r2) of an m1 x m2 grid transforms its own X-pencil block along X,
its own Y-pencil block along Y and its own Z-pencil block along Z; each
exchange keeps only what the rank sends to itself and the other ranks' blocks
count as zero.  The forward result is therefore the 3D transform of the input
with every element outside the rank's X-pencil set to zero, restricted to the
rank's Z-pencil block; the backward result is the staged C2R of the half
spectrum with every mode outside the rank's Z-pencil block set to zero,
restricted to its X-pencil block.  Both are checked against the oracle on
exactly those masked inputs.  A 1 x 1 share is the whole transform and must
equal the ordinary plan bit for bit.
"""
import numpy as np
import pytest

from tests import errbounds
import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1905_02803_amd as pf  # noqa: E402


def rel(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


def ranges(nx, ny, nz, lay):
    """(x-pencil z, y ranges) and (z-pencil kx, ky ranges) of rank (r1, r2) as slices."""
    stx, szx, _ = pf.pf_query_dims(nx, ny, nz, lay, pf.PF_PENCIL_X, lay.r1, lay.r2)
    stz, szz, _ = pf.pf_query_dims(nx, ny, nz, lay, pf.PF_PENCIL_Z, lay.r1, lay.r2)
    xz = slice(stx[2], stx[2] + szx[2])
    xy = slice(stx[1], stx[1] + szx[1])
    zkx = slice(stz[0], stz[0] + szz[0])
    zky = slice(stz[1], stz[1] + szz[1])
    return xz, xy, zkx, zky


def check_block(got, ref, whole, tol, floor_block=None):
    """A rank's block against the masked oracle: the error over the norm of the
    whole masked transform (the scale of the rounding error, by Parseval) within
    tol, and the block's own error within the staged rounding bound of
    errbounds.py, tol / 2 sqrt(sum of M over the block), when floor_block (M of
    the whole result cut to the block, in the block's layout) is given."""
    got, ref, whole = np.asarray(got), np.asarray(ref), np.asarray(whole)
    e = float(np.linalg.norm((got - ref).ravel()))
    nw, nb = float(np.linalg.norm(whole.ravel())), float(np.linalg.norm(ref.ravel()))
    assert e / nw < tol, (e / nw, tol)
    if floor_block is not None:
        errbounds.check_subset(e * e, float(np.sum(floor_block)), tol)
    return e / nw, (e / nb if nb > 0 else 0.0)


# passes of the forward transform along x, y, z: axes 2, 1, 0 of a [kz][ky][kx]
# result; of the backward transform along z, y, x: axes 0, 1, 2 of [z][y][x]
FWD_AXES = (2, 1, 0)
BWD_AXES = (0, 1, 2)


def z_block(U, zkx, zky, stride1):
    """Rank's Z-pencil block of a half spectrum U[kz][ky][kx], in Table 1 order."""
    b = U[:, zky, zkx]
    return np.ascontiguousarray(b.transpose(2, 1, 0) if stride1 else b)


CASES = [
    # (nz, ny, nx), (m1, m2), (r1, r2)
    ((12, 10, 16), (2, 3), (1, 2)),
    ((18, 20, 30), (3, 4), (2, 1)),
    ((9, 7, 15), (2, 2), (0, 1)),
    ((16, 32, 1024), (2, 4), (1, 3)),    # power-of-two X stage, modes 513 over 2 ranks
    ((64, 64, 512), (4, 2), (3, 0)),     # power-of-two Y and Z passes, 16-column blocks cut by the split
    ((32, 64, 64), (1, 8), (0, 5)),      # slab: 1 x P
    ((32, 48, 64), (5, 1), (4, 0)),      # m2 = 1
]


@pytest.mark.parametrize("stride1", [1, 0])
@pytest.mark.parametrize("prec", [pf.PF_F32, pf.PF_F64])
@pytest.mark.parametrize("shape,grid,rank", CASES, ids=lambda v: "x".join(map(str, v)))
def test_share_only_matches_masked_oracle(shape, grid, rank, prec, stride1):
    nz, ny, nx = shape
    print(f"case shape={shape} grid={grid} rank={rank} prec={prec} stride1={stride1}", flush=True)
    lay = pf.Layout(m1=grid[0], m2=grid[1], share_only=1, r1=rank[0], r2=rank[1], precision=prec,
                    stride1=stride1)
    tol = 1e-12 if prec == pf.PF_F64 else 1e-6
    rdt = np.float64 if prec == pf.PF_F64 else np.float32
    cdt = np.complex128 if prec == pf.PF_F64 else np.complex64
    xz, xy, zkx, zky = ranges(nx, ny, nz, lay)
    u = synth.uniform(700 + nx + ny + nz, shape).astype(rdt)
    um = np.zeros_like(u)
    um[xz, xy, :] = u[xz, xy, :]
    V = synth.complex_half(800 + nx, (nz, ny, nx // 2 + 1)).astype(cdt)
    Vm = np.zeros_like(V)
    Vm[:, zky, zkx] = V[:, zky, zkx]
    with pf.Plan(nx, ny, nz, lay) as plan:
        assert plan.real_shape == u[xz, xy, :].shape
        got = plan.ftran(torch.from_numpy(np.ascontiguousarray(u[xz, xy, :])).cuda())
        torch.cuda.synchronize()
        whole = oracle.r2c3d(um)
        ref = z_block(whole, zkx, zky, stride1)
        assert got.shape == ref.shape
        assert rel(got.cpu().numpy(), ref) < tol
        check_block(got.cpu().numpy(), ref, whole, tol,
                    z_block(errbounds.staged_floor(whole, FWD_AXES), zkx, zky, stride1))
        vin = torch.from_numpy(z_block(V, zkx, zky, stride1)).cuda()
        back = plan.btran(vin)
        torch.cuda.synchronize()
        wholeb = oracle.c2r3d(Vm, nx)
        refb = wholeb[xz, xy, :]
        assert rel(back.cpu().numpy(), refb) < tol
        check_block(back.cpu().numpy(), refb, wholeb, tol, errbounds.staged_floor(wholeb, BWD_AXES)[xz, xy, :])
        # a second call reuses the workspace: the zero fills must not depend on the first
        got2 = plan.ftran(torch.from_numpy(np.ascontiguousarray(u[xz, xy, :])).cuda())
        torch.cuda.synchronize()
        assert torch.equal(got2, got)


@pytest.mark.parametrize("shape", [(12, 10, 16), (16, 16, 1024)])
def test_one_by_one_share_is_the_whole_transform(shape):
    nz, ny, nx = shape
    u = torch.from_numpy(synth.uniform(31, shape).astype(np.float32)).cuda()
    with pf.Plan(nx, ny, nz) as full, pf.Plan(nx, ny, nz, pf.Layout(share_only=1)) as share:
        assert share.num_passes(pf.PF_DIR_FORWARD) == 5 and share.num_passes(pf.PF_DIR_BACKWARD) == 6
        a = full.ftran(u)
        b = share.ftran(u)
        torch.cuda.synchronize()
        assert torch.equal(a, b)
        assert torch.equal(full.btran(a), share.btran(a))


def test_share_only_at_512_cubed_on_1x8():
    """A slab rank's share of a 512^3 grid: X-pencil [64][512][512] -> Z-pencil [257][64][512].

    The rank's ky range (320..383, i.e. |ky| 129..192) of a |k|^-5/3 field
    holds a small part of the energy, while the FP32 rounding error of a
    transform scales with the norm of the whole result (Parseval); the error
    in the block is therefore measured against the norm of the whole masked
    transform, at the FP32 bound 1e-6.
    """
    nx = ny = nz = 512
    lay = pf.Layout(m1=1, m2=8, share_only=1, r1=0, r2=5)
    xz, xy, zkx, zky = ranges(nx, ny, nz, lay)
    u = synth.grf(2, (nz, ny, nx))
    print("case 512^3 share 1x8 rank (0, 5)", flush=True)
    with pf.Plan(nx, ny, nz, lay) as plan:
        assert plan.real_shape == (64, 512, 512) and plan.complex_shape == (257, 64, 512)
        got = plan.ftran(torch.from_numpy(np.ascontiguousarray(u[xz, xy, :])).cuda()).cpu().numpy()
    um = np.zeros_like(u)
    um[xz, xy, :] = u[xz, xy, :]
    full = oracle.r2c3d(um)
    ref = z_block(full, zkx, zky, 1)
    floor = z_block(errbounds.staged_floor(full, FWD_AXES), zkx, zky, 1)
    err, err_block = check_block(got, ref, full, 1e-6, floor)
    print(f"block error / whole-transform norm {err:.3e}, block-relative {err_block:.3e} (staged bound "
          f"{0.5e-6 * np.sqrt(floor.sum()) / np.linalg.norm(ref):.3e})", flush=True)


@pytest.mark.parametrize("math,bound", [(pf.PF_MFMA_FP16X2, 1e-6), (pf.PF_MFMA_BF16X2, 1e-5)])
def test_share_only_with_matrix_core_stages(math, bound):
    """A share whose X (nx = 1024) and Y (ny = 512) stages run on the matrix
    cores: the forward result against the masked oracle at the variant's bound,
    normalised by the whole masked transform (as for the FP32 shares)."""
    nz, ny, nx = 16, 512, 1024
    lay = pf.Layout(m1=2, m2=4, share_only=1, r1=1, r2=3, math=math)
    print(f"case share mfma math={math}", flush=True)
    xz, xy, zkx, zky = ranges(nx, ny, nz, lay)
    u = synth.uniform(901, (nz, ny, nx)).astype(np.float32)
    um = np.zeros_like(u)
    um[xz, xy, :] = u[xz, xy, :]
    with pf.Plan(nx, ny, nz, lay) as plan:
        got = plan.ftran(torch.from_numpy(np.ascontiguousarray(u[xz, xy, :])).cuda()).cpu().numpy()
    want = oracle.r2c3d(um)
    check_block(got, z_block(want, zkx, zky, 1), want, bound,
                z_block(errbounds.staged_floor(want, FWD_AXES), zkx, zky, 1))
