"""The FP64 power-of-two X stage (nx = 512, 1024): the real line as a complex
line of half the length, its DFT and the split into nx / 2 + 1 modes
(Sec. 3.2), eight lines per tile.  Checked against the oracle's X stage alone
and the whole transform, on tile-ragged line counts (one line, fewer lines
than a tile, more tiles than the resident grid) and in place.  With ny a
multiple of 16 up to 512 the backward X pass (and at nx = 512 the forward one)
uses the transposed workspace [nz][nxh][ny] with 16-line tiles (one 256-byte
row per mode)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1905_02803_amd as pf  # noqa: E402

TOL = 1e-12


def rel(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


SHAPES = [(1, 1, 512), (3, 5, 512), (2, 7, 1024), (9, 8, 512), (4, 300, 512), (35, 40, 1024),
          (5, 16, 512), (3, 32, 1024), (2, 512, 512)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda v: "x".join(map(str, v[::-1])))
def test_f64_power_of_two_x_stage_matches_oracle(shape):
    nz, ny, nx = shape
    print(f"case FP64 X shape={shape}", flush=True)
    u = synth.uniform(900 + nx + ny + nz, shape)
    V = synth.complex_half(901 + nx + ny, (nz, ny, nx // 2 + 1))
    with pf.Plan(nx, ny, nz, pf.Layout(precision=pf.PF_F64, stride1=1)) as plan:
        assert plan.pass_kernel(pf.PF_DIR_FORWARD, 0) == "r2c_pow2"
        assert plan.pass_kernel(pf.PF_DIR_BACKWARD, 2) == "c2r_pow2"
        # the X stage alone, both directions; with ny a multiple of 16 up to 512 the
        # intermediates are the transposed workspace [nz][nxh][ny] (16-line tiles):
        # backward always, forward at nx = 512
        transposed = ny % 16 == 0 and ny <= 512
        ftr = transposed and nx == 512
        assert plan.workspace_layout(pf.PF_DIR_FORWARD) == (pf.PF_WS_TRANSPOSED if ftr else pf.PF_WS_BLOCKED)
        assert plan.workspace_layout(pf.PF_DIR_BACKWARD) == (pf.PF_WS_TRANSPOSED if transposed else pf.PF_WS_BLOCKED)
        viewf = pf.transposed_workspace_to_half_spectrum if ftr else pf.workspace_to_half_spectrum
        ws = torch.zeros(plan.workspace_bytes // 16, dtype=torch.complex128, device="cuda")
        plan.run_pass(pf.PF_DIR_FORWARD, 0, torch.from_numpy(u).cuda(), ws)
        torch.cuda.synchronize()
        assert rel(viewf(ws, nx, ny, nz).cpu().numpy(), oracle.stage_x_r2c(u)) < TOL
        ws.zero_()
        Vd = torch.from_numpy(V).cuda()
        if transposed:
            ws[: V.size].copy_(Vd.permute(0, 2, 1).reshape(-1))
        else:
            pf.half_spectrum_to_workspace(Vd, ws)
        r = plan.empty_real()
        plan.run_pass(pf.PF_DIR_BACKWARD, 2, ws, r)
        torch.cuda.synchronize()
        assert rel(r.cpu().numpy(), oracle.stage_x_c2r(V, nx)) < TOL
        # the whole transform and its round trip
        U = plan.ftran(torch.from_numpy(u).cuda())
        assert rel(U.cpu().numpy(), oracle.to_stride1(oracle.r2c3d(u))) < TOL
        back = plan.btran(torch.from_numpy(oracle.to_stride1(V)).cuda())
        assert rel(back.cpu().numpy(), oracle.c2r3d(V, nx)) < TOL
        rt = plan.btran(U)
        assert rel(rt.cpu().numpy() / (nx * ny * nz), u) < TOL


@pytest.mark.parametrize("shape", [(3, 5, 512), (4, 6, 1024)], ids=lambda v: "x".join(map(str, v[::-1])))
def test_f64_power_of_two_x_inplace_equals_out_of_place(shape):
    nz, ny, nx = shape
    u = synth.uniform(910 + nx, shape)
    lay = dict(precision=pf.PF_F64)
    with pf.Plan(nx, ny, nz, pf.Layout(**lay)) as p_out, pf.Plan(nx, ny, nz, pf.Layout(inplace=1, **lay)) as p_in:
        assert p_in.pass_kernel(pf.PF_DIR_FORWARD, 0) == "r2c_pow2"
        ref = p_out.ftran(torch.from_numpy(u).cuda())
        buf = torch.zeros(p_in.inplace_bytes // 8, dtype=torch.float64, device="cuda")
        buf[: u.size] = torch.from_numpy(u.reshape(-1)).cuda()
        p_in.ftran_inplace(buf)
        torch.cuda.synchronize()
        spec = buf.view(torch.complex128)[: ref.numel()].reshape(ref.shape)
        assert torch.equal(spec, ref)
        back_ref = p_out.btran(ref)
        p_in.btran_inplace(buf)
        torch.cuda.synchronize()
        assert torch.equal(buf[: u.size].reshape(u.shape), back_ref)
