"""Compile-time mixed-radix passes (7-smooth lengths 48 .. 320 and 360, 480):
every length of the table in each of the three roles, against the FP64 oracle.

For each length n:
  * (nx, ny, nz) = (n, n, 3): the forward X pass (two real lines per complex
    line, split in LDS) and the Y pass at length n; 3 n lines, odd when n is,
    so the last line pair of the last tile is half empty; nx / 2 + 1 modes
    leave a ragged last column block;
  * (nx, ny, nz) = (6, 5, n): the Z pass at length n with 4 modes (12 of the
    16 columns of the only column block empty).
Forward of a uniform field and backward of an arbitrary half spectrum, both
Z-pencil layouts for the second shape, all within the FP32 bound 1e-6 of the
relative L2 error; the plan must report the mixed-radix kernels for those
passes (pf_pass_kernel), so that the check cannot pass on another kernel.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1905_02803_amd as pf  # noqa: E402

MR_LENGTHS = [48, 49, 50, 54, 56, 60, 63, 64, 70, 72, 75, 80, 81, 84, 90, 96, 98, 100, 105, 108, 112, 120, 125,
              126, 128, 135, 140, 144, 147, 150, 160, 162, 168, 175, 180, 189, 192, 196, 200, 210, 216, 224, 225,
              240, 243, 245, 250, 252, 270, 280, 288, 294, 300, 315, 320, 360, 480]


def rel(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


def kernels(plan):
    return {(d, plan.pass_name(d, i)): plan.pass_kernel(d, i)
            for d in (pf.PF_DIR_FORWARD, pf.PF_DIR_BACKWARD) for i in range(plan.num_passes(d))}


def run_case(nx, ny, nz, stride1, seed, expect):
    print(f"case mixed-radix {nx}x{ny}x{nz} stride1={stride1}", flush=True)
    u = synth.uniform(seed, (nz, ny, nx)).astype(np.float32)
    V = synth.complex_half(seed + 1, (nz, ny, nx // 2 + 1)).astype(np.complex64)
    to_layout = oracle.to_stride1 if stride1 else (lambda a: a)
    with pf.Plan(nx, ny, nz, pf.Layout(stride1=stride1)) as plan:
        got = kernels(plan)
        for key, fam in expect.items():
            assert got[key] == fam, (key, got[key], fam)
        U = plan.ftran(torch.from_numpy(u).cuda())
        b = plan.btran(torch.from_numpy(np.ascontiguousarray(to_layout(V))).cuda())
        torch.cuda.synchronize()
        assert rel(U.cpu().numpy(), to_layout(oracle.r2c3d(u))) < 1e-6
        assert rel(b.cpu().numpy(), oracle.c2r3d(V, nx)) < 1e-6


@pytest.mark.parametrize("n", MR_LENGTHS)
def test_mixed_radix_x_and_y(n):
    F, B = pf.PF_DIR_FORWARD, pf.PF_DIR_BACKWARD
    run_case(n, n, 3, 1, 100 + n, {(F, "fwd_x_r2c"): "r2c_mixed", (F, "fwd_y_c2c"): "c2c_mixed",
                                   (B, "bwd_y_c2c"): "c2c_mixed", (B, "bwd_x_c2r"): "c2r_mixed"})


@pytest.mark.parametrize("n", MR_LENGTHS)
@pytest.mark.parametrize("stride1", [1, 0])
def test_mixed_radix_z(n, stride1):
    F, B = pf.PF_DIR_FORWARD, pf.PF_DIR_BACKWARD
    run_case(6, 5, n, stride1, 300 + n, {(F, "fwd_z_c2c"): "c2c_mixed", (B, "bwd_z_c2c"): "c2c_mixed"})


def test_mixed_radix_grid_480x360x250():
    """The mixed-radix benchmark grid: all six passes on the compile-time kernels."""
    nx, ny, nz = 480, 360, 250
    print("case mixed-radix 480x360x250", flush=True)
    u = synth.uniform(7, (nz, ny, nx)).astype(np.float32)
    with pf.Plan(nx, ny, nz) as plan:
        fams = set(kernels(plan).values())
        assert fams == {"r2c_mixed", "c2c_mixed", "c2r_mixed"}, fams
        U = plan.ftran(torch.from_numpy(u).cuda())
        r = plan.btran(U)
        torch.cuda.synchronize()
        ref = oracle.r2c3d(u)
        assert rel(U.cpu().numpy(), oracle.to_stride1(ref)) < 1e-6
        back = r.cpu().numpy() / (nx * ny * nz)
        assert rel(back, u) < 1e-6


def test_mixed_radix_not_for_cheb_or_f64():
    """The Chebyshev third transform and FP64 keep the runtime-radix kernels."""
    with pf.Plan(60, 60, 61, pf.Layout(third=pf.PF_THIRD_CHEB)) as plan:
        k = kernels(plan)
        assert k[(pf.PF_DIR_FORWARD, "fwd_z_c2c")] == "c2c_generic"
        assert k[(pf.PF_DIR_FORWARD, "fwd_y_c2c")] == "c2c_mixed"
    with pf.Plan(60, 60, 60, pf.Layout(precision=pf.PF_F64)) as plan:
        assert set(kernels(plan).values()) <= {"c2c_generic", "r2c_generic", "c2r_generic"}
