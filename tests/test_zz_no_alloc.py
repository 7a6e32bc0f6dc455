"""The no-allocation entry point pf_exec_noalloc: the transform with the
library's static device scratch as its workspace, called through the C ABI.

Its results must equal those of pf_ftran_r2c / pf_btran_c2r on the same plan
(the same kernels run on the same data: bit for bit, which implies the FP32
1e-6 / FP64 1e-12 bars against the oracle, also checked), on consecutive
calls where the second uses a smaller grid than the first (the scratch keeps
the first call's contents), for 1 x 1 and m1 x m2 plans in both precisions.
Plans whose workspace exceeds the scratch, share-only plans and bad
directions are refused before anything is enqueued.
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


def run_both(plan, u, V):
    """(existing forward, no-alloc forward, existing backward, no-alloc backward) on the plan."""
    ref_f = plan.empty_complex()
    got_f = plan.empty_complex().fill_(float("nan"))
    pf.pf_ftran_r2c(plan.handle, u.data_ptr(), ref_f.data_ptr(), 0)
    pf.pf_exec_noalloc(plan.handle, pf.PF_DIR_FORWARD, u.data_ptr(), got_f.data_ptr(), 0)
    ref_b = plan.empty_real()
    got_b = plan.empty_real().fill_(float("nan"))
    pf.pf_btran_c2r(plan.handle, V.data_ptr(), ref_b.data_ptr(), 0)
    pf.pf_exec_noalloc(plan.handle, pf.PF_DIR_BACKWARD, V.data_ptr(), got_b.data_ptr(), 0)
    torch.cuda.synchronize()
    return ref_f, got_f, ref_b, got_b


@pytest.mark.parametrize("prec", [pf.PF_F32, pf.PF_F64])
def test_noalloc_matches_existing_entry_point_large_then_small(prec):
    rdt = np.float64 if prec == pf.PF_F64 else np.float32
    cdt = np.complex128 if prec == pf.PF_F64 else np.complex64
    tol = 1e-12 if prec == pf.PF_F64 else 1e-6
    # first a grid on the power-of-two kernels (FP32), then smaller ones on the
    # compile-time mixed-radix kernels (FP32: lengths 96, 60, 50) and on the
    # runtime-radix kernels (lengths 36, 20, 24)
    for step, shape in enumerate([(64, 256, 512), (50, 60, 96), (24, 20, 36)]):
        nz, ny, nx = shape
        print(f"case no-alloc call {step} shape={shape} prec={prec}", flush=True)
        with pf.Plan(nx, ny, nz, pf.Layout(precision=prec)) as plan:
            assert plan.workspace_bytes <= pf.PF_NOALLOC_MAX_BYTES
            u_h = synth.uniform(11 + step, shape).astype(rdt)
            V_h = synth.complex_half(12 + step, (nz, ny, nx // 2 + 1)).astype(cdt)
            u = torch.from_numpy(u_h).cuda()
            V = torch.from_numpy(oracle.to_stride1(V_h)).cuda()
            ref_f, got_f, ref_b, got_b = run_both(plan, u, V)
            assert torch.equal(got_f, ref_f)
            assert torch.equal(got_b, ref_b)
            assert rel(got_f.cpu().numpy(), oracle.to_stride1(oracle.r2c3d(u_h))) < tol
            assert rel(got_b.cpu().numpy(), oracle.c2r3d(V_h, nx)) < tol
            # the input is left as it was (out-of-place plan)
            assert torch.equal(u, torch.from_numpy(u_h).cuda())


def test_noalloc_processor_grid_plan():
    """An m1 x m2 plan: the scratch holds the workspace and the global-layout array."""
    nz, ny, nx = 12, 10, 16
    lay = pf.Layout(m1=2, m2=3)
    print("case no-alloc 2x3 grid", flush=True)
    with pf.Plan(nx, ny, nz, lay) as plan:
        nreal, ncplx = nx * ny * nz, (nx // 2 + 1) * ny * nz
        u = torch.from_numpy(synth.uniform(21, (nreal,)).astype(np.float32)).cuda()
        V = torch.from_numpy(synth.complex_half(22, (ncplx,)).astype(np.complex64)).cuda()
        ref_f = torch.empty(ncplx, dtype=torch.complex64, device="cuda")
        got_f = torch.full((ncplx,), float("nan"), dtype=torch.complex64, device="cuda")
        pf.pf_ftran_r2c(plan.handle, u.data_ptr(), ref_f.data_ptr(), 0)
        pf.pf_exec_noalloc(plan.handle, pf.PF_DIR_FORWARD, u.data_ptr(), got_f.data_ptr(), 0)
        ref_b = torch.empty(nreal, dtype=torch.float32, device="cuda")
        got_b = torch.full((nreal,), float("nan"), dtype=torch.float32, device="cuda")
        pf.pf_btran_c2r(plan.handle, V.data_ptr(), ref_b.data_ptr(), 0)
        pf.pf_exec_noalloc(plan.handle, pf.PF_DIR_BACKWARD, V.data_ptr(), got_b.data_ptr(), 0)
        torch.cuda.synchronize()
        assert torch.equal(got_f, ref_f)
        assert torch.equal(got_b, ref_b)


def test_noalloc_refusals():
    print("case no-alloc refusals", flush=True)
    with pf.Plan(512, 512, 512) as big:  # workspace 570 MB > 256 MiB
        assert big.workspace_bytes > pf.PF_NOALLOC_MAX_BYTES
        u = big.empty_real()
        U = big.empty_complex()
        with pytest.raises(pf.PfError) as e:
            pf.pf_exec_noalloc(big.handle, pf.PF_DIR_FORWARD, u.data_ptr(), U.data_ptr(), 0)
        assert e.value.code == pf.PF_EWORKSPACE
    with pf.Plan(16, 8, 8) as plan:
        u = plan.empty_real()
        U = plan.empty_complex()
        for d in (-1, 2):
            with pytest.raises(pf.PfError) as e:
                pf.pf_exec_noalloc(plan.handle, d, u.data_ptr(), U.data_ptr(), 0)
            assert e.value.code == pf.PF_EINVAL
        with pytest.raises(pf.PfError) as e:
            pf.pf_exec_noalloc(plan.handle, pf.PF_DIR_FORWARD, u.data_ptr(), u.data_ptr(), 0)
        assert e.value.code == pf.PF_EALIAS
    with pf.Plan(16, 8, 8, pf.Layout(m1=2, m2=2, share_only=1, r1=1, r2=0)) as share:
        u = share.empty_real()
        U = share.empty_complex()
        with pytest.raises(pf.PfError) as e:
            pf.pf_exec_noalloc(share.handle, pf.PF_DIR_FORWARD, u.data_ptr(), U.data_ptr(), 0)
        assert e.value.code == pf.PF_EUNSUPPORTED
    torch.cuda.synchronize()
