"""Layout options off the measured configuration: the empty third transform
(Sec. 3.1), USEEVEN (Sec. 3.4) and their combination with the m1 x m2 blocks.

* third = PF_THIRD_EMPTY: the forward result is the X-then-Y transform of
  every z plane, written as the Z-pencil with z untransformed; the backward
  transform inverts Y then takes the staged C2R along X.  Checked against the
  oracle's composition of its X and Y stages (itself pinned to numpy's 2D
  transforms on the CPU).
* useeven = 1 pads exchange blocks to equal size; on one GPU there are no
  exchange buffers, so the results must be bitwise those of useeven = 0.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1905_02803_amd as pf  # noqa: E402


def rel(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


SHAPES = [(12, 10, 16), (9, 7, 15), (16, 32, 1024), (32, 64, 512), (5, 256, 48),
          (256, 12, 36), (1024, 6, 40), (2048, 3, 10),  # these three: power-of-two Z, reorder-only kernel
          (17, 10, 16), (1021, 3, 8)]                   # nz with prime factors above 7: nothing to factor


@pytest.mark.parametrize("stride1", [1, 0])
@pytest.mark.parametrize("prec", [pf.PF_F32, pf.PF_F64])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda v: "x".join(map(str, v)))
def test_empty_third_transform_matches_oracle(shape, prec, stride1):
    nz, ny, nx = shape
    print(f"case shape={shape} prec={prec} stride1={stride1}", flush=True)
    tol = 1e-12 if prec == pf.PF_F64 else 1e-6
    rdt = np.float64 if prec == pf.PF_F64 else np.float32
    cdt = np.complex128 if prec == pf.PF_F64 else np.complex64
    u = synth.uniform(900 + nx + nz, shape).astype(rdt)
    lay = pf.Layout(precision=prec, stride1=stride1, third=pf.PF_THIRD_EMPTY)
    with pf.Plan(nx, ny, nz, lay) as plan:
        got = plan.ftran(torch.from_numpy(u).cuda()).cpu().numpy()
        ref = oracle.r2c3d_third_empty(u)
        assert rel(got, oracle.to_stride1(ref) if stride1 else ref) < tol
        V = synth.complex_half(901 + nx, (nz, ny, nx // 2 + 1)).astype(cdt)
        back = plan.btran(torch.from_numpy(oracle.to_stride1(V) if stride1 else V).cuda()).cpu().numpy()
        assert rel(back, oracle.c2r3d_third_empty(V, nx)) < tol


def test_empty_third_transform_on_processor_grid_and_share():
    """The m1 x m2 blocks and a share-only rank of the empty-third transform equal
    the matching slices / masked oracle result."""
    nz, ny, nx = 18, 20, 32
    u = synth.uniform(77, (nz, ny, nx)).astype(np.float32)
    base = dict(third=pf.PF_THIRD_EMPTY)
    with pf.Plan(nx, ny, nz, pf.Layout(**base)) as full:
        ref = full.ftran(torch.from_numpy(u).cuda()).cpu().numpy()  # [kx][ky][z]
    lay = pf.Layout(m1=2, m2=3, share_only=1, r1=1, r2=2, **base)
    stx, szx, _ = pf.pf_query_dims(nx, ny, nz, lay, pf.PF_PENCIL_X, 1, 2)
    stz, szz, _ = pf.pf_query_dims(nx, ny, nz, lay, pf.PF_PENCIL_Z, 1, 2)
    xz, xy = slice(stx[2], stx[2] + szx[2]), slice(stx[1], stx[1] + szx[1])
    zkx, zky = slice(stz[0], stz[0] + szz[0]), slice(stz[1], stz[1] + szz[1])
    um = np.zeros_like(u)
    um[xz, xy, :] = u[xz, xy, :]
    with pf.Plan(nx, ny, nz, lay) as share:
        got = share.ftran(torch.from_numpy(np.ascontiguousarray(u[xz, xy, :])).cuda()).cpu().numpy()
    want = oracle.to_stride1(oracle.r2c3d_third_empty(um))[zkx, zky, :]
    assert rel(got, want) < 1e-6
    # the whole-grid result of the masked input, sliced, agrees with the oracle too
    assert rel(ref, oracle.to_stride1(oracle.r2c3d_third_empty(u))) < 1e-6


@pytest.mark.parametrize("grid", [(1, 1), (2, 3), (4, 2)])
def test_useeven_changes_no_result(grid):
    nz, ny, nx = 12, 10, 16
    u = torch.from_numpy(synth.uniform(5, (nz, ny, nx)).astype(np.float32)).cuda().reshape(-1)
    outs = []
    for ue in (0, 1):
        lay = pf.Layout(m1=grid[0], m2=grid[1], useeven=ue)
        with pf.Plan(nx, ny, nz, lay) as plan:
            U = torch.empty((nx // 2 + 1) * ny * nz, dtype=torch.complex64, device="cuda")
            pf.pf_ftran_r2c(plan.handle, u.data_ptr(), U.data_ptr(), 0)
            r = torch.empty(nx * ny * nz, dtype=torch.float32, device="cuda")
            pf.pf_btran_c2r(plan.handle, U.data_ptr(), r.data_ptr(), 0)
            torch.cuda.synchronize()
            outs.append((U.clone(), r.clone()))
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])


@pytest.mark.parametrize("nz", [17, 257])  # extension 32 (mixed-radix kernel) and 512 (power-of-two kernel)
def test_cheb_third_transform_on_processor_grid_and_share(nz):
    """The Chebyshev third transform (type-I DCT along z) on the m1 x m2 blocks
    (bitwise slices of the 1 x 1 result) and on one share-only rank (the
    masked oracle composition, restricted to the rank's Z-pencil block)."""
    ny, nx = 20, 32
    print(f"case cheb grid/share nz={nz}", flush=True)
    u = synth.uniform(78, (nz, ny, nx)).astype(np.float32)
    base = dict(third=pf.PF_THIRD_CHEB)
    with pf.Plan(nx, ny, nz, pf.Layout(**base)) as full:
        ref = full.ftran(torch.from_numpy(u).cuda()).cpu().numpy()  # [kx][ky][kz]
    assert rel(ref, oracle.to_stride1(oracle.r2c3d_cheb(u))) < 1e-6
    # m1 x m2 blocks: the concatenated Z-pencil blocks are the 1 x 1 result, bitwise
    from tests.test_gpu_grid import blocks, unblocks

    nxh = nx // 2 + 1
    lay = pf.Layout(m1=2, m2=3, **base)
    with pf.Plan(nx, ny, nz, lay) as grid:
        ub = torch.from_numpy(blocks(u.transpose(2, 1, 0), nx, ny, nz, lay, pf.PF_PENCIL_X)).cuda()
        out = torch.empty(nxh * ny * nz, dtype=torch.complex64, device="cuda")
        pf.pf_ftran_r2c(grid.handle, ub.data_ptr(), out.data_ptr(), 0)
        torch.cuda.synchronize()
    assert np.array_equal(unblocks(out.cpu().numpy(), (nxh, ny, nz), nx, ny, nz, lay, pf.PF_PENCIL_Z), ref)
    # share-only rank (1, 2) of the same grid
    lay = pf.Layout(m1=2, m2=3, share_only=1, r1=1, r2=2, **base)
    stx, szx, _ = pf.pf_query_dims(nx, ny, nz, lay, pf.PF_PENCIL_X, 1, 2)
    stz, szz, _ = pf.pf_query_dims(nx, ny, nz, lay, pf.PF_PENCIL_Z, 1, 2)
    xz, xy = slice(stx[2], stx[2] + szx[2]), slice(stx[1], stx[1] + szx[1])
    zkx, zky = slice(stz[0], stz[0] + szz[0]), slice(stz[1], stz[1] + szz[1])
    um = np.zeros_like(u)
    um[xz, xy, :] = u[xz, xy, :]
    with pf.Plan(nx, ny, nz, lay) as share:
        got = share.ftran(torch.from_numpy(np.ascontiguousarray(u[xz, xy, :])).cuda()).cpu().numpy()
    want = oracle.to_stride1(oracle.r2c3d_cheb(um))
    # normalised by the whole masked transform (FP32 rounding scale), and the
    # block's own error within the staged rounding bound, as for the other share
    # tests (want is [kx][ky][kz]: passes along x, y, z are axes 0, 1, 2)
    from tests import errbounds
    from tests.test_gpu_share import check_block

    check_block(got, want[zkx, zky, :], want, 1e-6, errbounds.staged_floor(want, (0, 1, 2))[zkx, zky, :])
