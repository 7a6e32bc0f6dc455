"""The m1 x m2 local-block layout (Sec. 2, Table 1) on one GPU.

All P ranks' blocks are handled by one plan: the forward input is the
concatenation of the ranks' X-pencils, the output the concatenation of their
Z-pencils, each block in its Table 1 storage order (rank order r2 m1 + r1).
Each rank's block of the result must equal the matching slice of the 1 x 1
transform bit for bit (same kernels, same arithmetic), and the 1 x 1
transform matches the oracle (test_gpu_parity.py).  Grids include uneven
splits such as the paper's 128^3-on-6-tasks case (Sec. 3.4) at reduced size.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1905_02803_amd as pf  # noqa: E402


def blocks(glob_xyz, nx, ny, nz, lay, pencil):
    """Concatenate the ranks' Table 1 blocks of a global array indexed [x][y][z]."""
    parts = []
    for r2 in range(lay.m2):
        for r1 in range(lay.m1):
            st, sz, od = pf.pf_query_dims(nx, ny, nz, lay, pencil, r1, r2)
            b = glob_xyz[st[0]:st[0] + sz[0], st[1]:st[1] + sz[1], st[2]:st[2] + sz[2]]
            # memory order: od[0] fastest -> C array with axes (od[2], od[1], od[0])
            parts.append(np.ascontiguousarray(np.transpose(b, (od[2], od[1], od[0]))).ravel())
    return np.concatenate(parts)


def unblocks(flat, shape_xyz, nx, ny, nz, lay, pencil):
    out = np.empty(shape_xyz, dtype=flat.dtype)
    off = 0
    for r2 in range(lay.m2):
        for r1 in range(lay.m1):
            st, sz, od = pf.pf_query_dims(nx, ny, nz, lay, pencil, r1, r2)
            n = sz[0] * sz[1] * sz[2]
            c = flat[off:off + n].reshape(sz[od[2]], sz[od[1]], sz[od[0]])
            inv = np.argsort([od[2], od[1], od[0]])
            out[st[0]:st[0] + sz[0], st[1]:st[1] + sz[1], st[2]:st[2] + sz[2]] = np.transpose(c, inv)
            off += n
    assert off == flat.size
    return out


CASES = [
    ((12, 10, 16), (2, 3)),     # (nz, ny, nx): 16 / 2 modes 9 over 2 ranks
    ((6, 8, 1024), (4, 2)),     # power-of-two X fast path
    ((18, 20, 32), (3, 4)),
    ((128 // 4, 128 // 4, 128 // 4), (2, 3)),   # 6 tasks, uneven in every pencil
    ((16, 512, 36), (1, 8)),    # slab 1 x P, power-of-two Y
    ((9, 7, 15), (5, 2)),
    ((50, 48, 60), (2, 3)),     # every axis on the compile-time mixed-radix kernels (FP32)
]


@pytest.mark.parametrize("stride1", [1, 0])
@pytest.mark.parametrize("prec", [pf.PF_F32, pf.PF_F64])
@pytest.mark.parametrize("shape,grid", CASES, ids=lambda v: "x".join(map(str, v)))
def test_processor_grid_blocks_equal_whole_grid_slices(shape, grid, prec, stride1):
    nz, ny, nx = shape
    nxh = nx // 2 + 1
    m1, m2 = grid
    print(f"case shape={shape} grid={grid} prec={prec} stride1={stride1}", flush=True)
    rdt = np.float64 if prec == pf.PF_F64 else np.float32
    cdt = np.complex128 if prec == pf.PF_F64 else np.complex64
    u = synth.uniform(500 + nx + ny, shape).astype(rdt)        # [z][y][x]
    lay1 = pf.Layout(precision=prec, stride1=stride1)
    layg = pf.Layout(precision=prec, stride1=stride1, m1=m1, m2=m2)
    with pf.Plan(nx, ny, nz, lay1) as p1, pf.Plan(nx, ny, nz, layg) as pg:
        assert pg.num_passes(pf.PF_DIR_FORWARD) == 5
        ref = p1.ftran(torch.from_numpy(u).cuda())
        ub = torch.from_numpy(blocks(u.transpose(2, 1, 0), nx, ny, nz, layg, pf.PF_PENCIL_X)).cuda()
        out = torch.empty(nxh * ny * nz, dtype=p1.complex_dtype, device="cuda")
        pf.pf_ftran_r2c(pg.handle, ub.data_ptr(), out.data_ptr(), 0)
        torch.cuda.synchronize()
        refc = ref.cpu().numpy()
        ref_xyz = refc.transpose(0, 1, 2) if stride1 else refc.transpose(2, 1, 0)  # -> [kx][ky][kz]
        got_xyz = unblocks(out.cpu().numpy(), (nxh, ny, nz), nx, ny, nz, layg, pf.PF_PENCIL_Z)
        assert np.array_equal(got_xyz, ref_xyz)
        # and against the oracle
        U = oracle.r2c3d(u).transpose(2, 1, 0)
        assert np.linalg.norm(got_xyz - U) / np.linalg.norm(U) < (1e-12 if prec == pf.PF_F64 else 1e-6)
        # backward from blocked Z-pencils of an arbitrary half spectrum
        V = synth.complex_half(600 + nx, (nz, ny, nxh)).astype(cdt)   # [kz][ky][kx]
        Vl = oracle.to_stride1(V) if stride1 else V
        refb = p1.btran(torch.from_numpy(Vl).cuda())
        Vb = torch.from_numpy(blocks(V.transpose(2, 1, 0), nx, ny, nz, layg, pf.PF_PENCIL_Z)).cuda()
        outb = torch.empty(nx * ny * nz, dtype=p1.real_dtype, device="cuda")
        pf.pf_btran_c2r(pg.handle, Vb.data_ptr(), outb.data_ptr(), 0)
        torch.cuda.synchronize()
        gotb = unblocks(outb.cpu().numpy(), (nx, ny, nz), nx, ny, nz, layg, pf.PF_PENCIL_X)
        assert np.array_equal(gotb, refb.cpu().numpy().transpose(2, 1, 0))


def test_processor_grid_inplace():
    nz, ny, nx = 12, 10, 16
    lay = pf.Layout(m1=2, m2=3, inplace=1)
    u = synth.uniform(9, (nz, ny, nx)).astype(np.float32)
    with pf.Plan(nx, ny, nz, pf.Layout(m1=2, m2=3)) as po, pf.Plan(nx, ny, nz, lay) as pi:
        ub = blocks(u.transpose(2, 1, 0), nx, ny, nz, lay, pf.PF_PENCIL_X)
        src = torch.from_numpy(ub).cuda()
        ref = torch.empty((nx // 2 + 1) * ny * nz, dtype=torch.complex64, device="cuda")
        pf.pf_ftran_r2c(po.handle, src.data_ptr(), ref.data_ptr(), 0)
        buf = torch.zeros(ref.numel() * 2, dtype=torch.float32, device="cuda")
        buf[: ub.size] = src
        pf.pf_ftran_r2c(pi.handle, buf.data_ptr(), buf.data_ptr(), 0)
        torch.cuda.synchronize()
        assert torch.equal(buf.view(torch.complex64), ref)
