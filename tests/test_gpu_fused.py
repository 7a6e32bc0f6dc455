"""The fused X-Y pass (pf_layout.fused_xy): the slab form of the method,
Sec. 4.3 / Fig. 10 -- the X and Y stages of every z plane in one persistent
kernel, so that a direction takes two passes instead of three.

Its tiles run the same arithmetic as the separate X and Y passes: the
forward result equals the three-pass plan's bit for bit, the backward one to
rounding (the compiler contracts a few multiply-adds of the complex-to-real
split differently in the fused kernel); both are checked against the FP64
oracle (forward, and backward of an arbitrary half spectrum) at the FP32
bound 1e-6.  Plane counts below, equal to and above the number of
work queues (8) are covered, both Z-pencil layouts, in place, repeated calls
(the work counters are reset per launch) and the no-allocation entry point.
No wait may reach its bound (pf_check_status).
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


SHAPES = [  # (nz, ny, nx)
    (24, 1024, 1024),
    (15, 512, 1024),   # 33 Y tiles of 512 points per plane: the last item's second tile is empty
    (9, 512, 2048),
    (5, 1024, 2048),   # fewer planes than queues
    (1, 1024, 1024),
]


@pytest.mark.parametrize("stride1", [1, 0])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s[::-1])))
def test_fused_matches_three_pass_plan_and_oracle(shape, stride1):
    nz, ny, nx = shape
    print(f"case fused shape={shape} stride1={stride1}", flush=True)
    u = synth.uniform(50 + nz, shape).astype(np.float32)
    V = synth.complex_half(60 + nz, (nz, ny, nx // 2 + 1)).astype(np.complex64)
    to_layout = oracle.to_stride1 if stride1 else (lambda a: a)
    with pf.Plan(nx, ny, nz, pf.Layout(stride1=stride1, fused_xy=1)) as fp, \
            pf.Plan(nx, ny, nz, pf.Layout(stride1=stride1)) as pp:
        assert fp.num_passes(pf.PF_DIR_FORWARD) == 2 and fp.num_passes(pf.PF_DIR_BACKWARD) == 2
        assert fp.pass_name(pf.PF_DIR_FORWARD, 0) == "fwd_xy_fused"
        assert fp.pass_name(pf.PF_DIR_BACKWARD, 1) == "bwd_yx_fused"
        ud = torch.from_numpy(u).cuda()
        Vd = torch.from_numpy(np.ascontiguousarray(to_layout(V))).cuda()
        Uf = fp.ftran(ud)
        Uf2 = fp.ftran(ud).clone()
        Up = pp.ftran(ud)
        bf = fp.btran(Vd)
        bp = pp.btran(Vd)
        pf.pf_check_status(fp.handle)
        assert torch.equal(Uf, Uf2)
        assert torch.equal(Uf, Up)
        assert float((bf - bp).norm() / bp.norm()) < 1e-6
        assert rel(Uf.cpu().numpy(), to_layout(oracle.r2c3d(u))) < 1e-6
        assert rel(bf.cpu().numpy(), oracle.c2r3d(V, nx)) < 1e-6


def test_fused_inplace_and_noalloc():
    nz, ny, nx = 12, 512, 1024
    print("case fused in place / no-alloc", flush=True)
    u = torch.from_numpy(synth.uniform(71, (nz, ny, nx)).astype(np.float32)).cuda()
    with pf.Plan(nx, ny, nz, pf.Layout(fused_xy=1, inplace=1)) as pi, pf.Plan(nx, ny, nz) as pp:
        ref = pp.ftran(u)
        buf = torch.zeros(pi.inplace_bytes // 4, dtype=torch.float32, device="cuda")
        buf[: u.numel()] = u.reshape(-1)
        pi.ftran_inplace(buf)
        torch.cuda.synchronize()
        assert torch.equal(buf.view(torch.complex64)[: ref.numel()].reshape(ref.shape), ref)
        back = pp.btran(ref)
        pi.btran_inplace(buf)
        pf.pf_check_status(pi.handle)
        got = buf[: u.numel()].reshape(u.shape)
        assert float((got - back).norm() / back.norm()) < 1e-6
    with pf.Plan(nx, ny, nz, pf.Layout(fused_xy=1)) as fp:
        out = fp.empty_complex()
        pf.pf_exec_noalloc(fp.handle, pf.PF_DIR_FORWARD, u.data_ptr(), out.data_ptr(), 0)
        pf.pf_check_status(fp.handle)
        assert torch.equal(out, ref)


def test_fused_refusals():
    for dims, lay in (((512, 512, 16), pf.Layout(fused_xy=1)),           # nx = 512: no fused kernel
                      ((1024, 256, 16), pf.Layout(fused_xy=1)),          # ny = 256
                      ((1024, 512, 16), pf.Layout(fused_xy=1, precision=pf.PF_F64)),
                      ((1024, 512, 16), pf.Layout(fused_xy=1, math=pf.PF_MFMA_BF16X2)),
                      ((1024, 512, 16), pf.Layout(fused_xy=1, m1=2, m2=2))):
        with pytest.raises(pf.PfError) as e:
            pf.Plan(*dims, lay)
        assert e.value.code == pf.PF_EUNSUPPORTED, (dims, lay)
    with pytest.raises(pf.PfError) as e:
        pf.Batch([(1024, 512, 4)], pf.Layout(fused_xy=1))
    assert e.value.code == pf.PF_EUNSUPPORTED
    with pf.Plan(1024, 512, 9, pf.Layout(fused_xy=1, third=pf.PF_THIRD_CHEB)) as plan:
        u = plan.empty_real().uniform_()
        with pytest.raises(pf.PfError) as e:
            pf.spectral_step(plan, u)
        assert e.value.code == pf.PF_EUNSUPPORTED
        # the transforms themselves run (Chebyshev third transform on the Z pass)
        U = plan.ftran(u)
        pf.pf_check_status(plan.handle)
        assert rel(U.cpu().numpy(), oracle.to_stride1(oracle.r2c3d_cheb(u.cpu().numpy()))) < 1e-6
