"""Parity at the benchmark's own grid sizes, in the launch configuration bench.py times.

* 1024^3 FP32 Gaussian random field (shell spectrum |k|^-5/3), STRIDE1,
  out-of-place: the forward output against the oracle's whole transform, the
  backward of an arbitrary half spectrum against the oracle's staged C2R, the
  round trip (Sec. 4.1) and Parseval; the forward error of every |k| shell
  against the staged rounding bound (errbounds.py).
  Also the two matrix-core precision variants at their stated bounds
  (FP16 x 2: 1e-6, BF16 x 2: 1e-5).
* 512^3 and 480 x 360 x 250 FP32 random fields: the same checks.
* 32^3 FP64, uniform[-1, 1] from seed 1, and the 512^3 FP64 benchmark grid
  (a random field): forward, backward and round trip at 1e-12.
* 2048^3 FP32 (eight times the benchmark's grid): round trip and Parseval,
  which hold at any size, reduced on the device.
* 1024^3 plane wave: every output of the forward transform and of the C2R of
  a single mode against the closed form.
The oracle runs in FP64 on the host (OpenMP); FP32 inputs are promoted exactly.
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
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def half_weights(nx):
    w = np.full(nx // 2 + 1, 2.0)
    w[0] = 1.0
    if nx % 2 == 0:
        w[-1] = 1.0
    return w


MFMA_BOUND = {pf.PF_MFMA_FP16X2: 1e-6, pf.PF_MFMA_BF16X2: 1e-5}


def check_grid(shape, seed, tol, maths=()):
    nz, ny, nx = shape
    print(f"case shape={shape} seed={seed}", flush=True)
    u = synth.grf(seed, shape)
    with pf.Plan(nx, ny, nz, pf.Layout(precision=pf.PF_F32, stride1=1)) as plan:
        ud = torch.from_numpy(u).cuda()
        Ud = plan.ftran(ud)
        back = plan.btran(Ud)
        torch.cuda.synchronize()
        # round trip and Parseval on the device result (independent of the oracle)
        N = float(nx) * ny * nz
        rt = (torch.linalg.vector_norm(back.double() / N - ud.double()) / torch.linalg.vector_norm(ud.double())).item()
        assert rt < tol, rt
        w = torch.from_numpy(half_weights(nx)).cuda()
        e_spec = (Ud.abs().double() ** 2 * w[:, None, None]).sum().item() / N
        e_real = (ud.double() ** 2).sum().item()
        assert abs(e_spec - e_real) / e_real < tol
        del back
        got = Ud.cpu().numpy()
        del Ud
        ref = oracle.to_stride1(oracle.r2c3d(u))
        err = rel(got, ref)
        print(f"forward rel L2 {err:.3e}, round trip {rt:.3e}", flush=True)
        assert err < tol
        # per |k| shell: the power-law field's energy falls off with |k|, so the
        # whole-result norm hides the weak shells; each shell is held to the
        # staged rounding bound of errbounds.py
        for lo, hi, m, e, bound in errbounds.check_shells(got, ref, nx, ny, nz, tol):
            print(f"  shell [{lo:g}, {hi:g}): {m} modes, rel L2 {e:.3e} (bound {bound:.3e})", flush=True)
        if nx in (1024, 2048) and ny in (512, 1024):  # the fused X-Y plan gives the same bits
            with pf.Plan(nx, ny, nz, pf.Layout(precision=pf.PF_F32, stride1=1, fused_xy=1)) as pfz:
                Uz = pfz.ftran(ud)
                assert np.array_equal(Uz.cpu().numpy(), got)
                bz = pfz.btran(Uz)
                pf.pf_check_status(pfz.handle)
                rtz = (torch.linalg.vector_norm(bz.double() / N - ud.double()) /
                       torch.linalg.vector_norm(ud.double())).item()
                assert abs(rtz - rt) <= 1e-3 * rt, (rtz, rt)
                del Uz, bz
        del got
        for mth in maths:  # the matrix-core variants against the same oracle result
            with pf.Plan(nx, ny, nz, pf.Layout(precision=pf.PF_F32, stride1=1, math=mth)) as pm:
                Um = pm.ftran(ud)
                bm = pm.btran(Um)
                torch.cuda.synchronize()
                rtm = (torch.linalg.vector_norm(bm.double() / N - ud.double()) /
                       torch.linalg.vector_norm(ud.double())).item()
                del bm
                em = rel(Um.cpu().numpy(), ref)
                del Um
            print(f"math {mth}: forward rel L2 {em:.3e}, round trip {rtm:.3e}", flush=True)
            assert em < MFMA_BOUND[mth] and rtm < 2 * MFMA_BOUND[mth]
        del ref
        # backward of an arbitrary half spectrum
        V = synth.complex_half(seed + 1000, (nz, ny, nx // 2 + 1)).astype(np.complex64)
        Vd = torch.from_numpy(oracle.to_stride1(V)).cuda()
        vd = plan.btran(Vd)
        torch.cuda.synchronize()
        del Vd
        err_b = rel(vd.cpu().numpy(), oracle.c2r3d(V, nx))
        print(f"backward rel L2 {err_b:.3e}", flush=True)
        assert err_b < tol


@pytest.mark.timeout(1200)
def test_1024_cubed_grf_matches_oracle():
    check_grid((1024, 1024, 1024), 3, 1e-6, maths=(pf.PF_MFMA_FP16X2, pf.PF_MFMA_BF16X2))


@pytest.mark.timeout(600)
@pytest.mark.parametrize("shape,seed", [((512, 512, 512), 2), ((250, 360, 480), 22)])
def test_512_cubed_and_uneven_grf_match_oracle(shape, seed):
    check_grid(shape, seed, 1e-6)


def test_32_cubed_f64_matches_oracle():
    shape = (32, 32, 32)
    u = synth.uniform(1, shape)
    with pf.Plan(32, 32, 32, pf.Layout(precision=pf.PF_F64)) as plan:
        Ud = plan.ftran(torch.from_numpy(u).cuda())
        back = plan.btran(Ud)
        torch.cuda.synchronize()
        assert rel(Ud.cpu().numpy(), oracle.to_stride1(oracle.r2c3d(u))) < 1e-12
        assert rel(back.cpu().numpy() / u.size, u) < 1e-12
        V = synth.complex_half(2, (32, 32, 17))
        vd = plan.btran(torch.from_numpy(oracle.to_stride1(V)).cuda())
        torch.cuda.synchronize()
        assert rel(vd.cpu().numpy(), oracle.c2r3d(V, 32)) < 1e-12


@pytest.mark.timeout(600)
def test_512_cubed_f64_matches_oracle():
    """The FP64 benchmark grid, in the plan bench.py times (FP64 power-of-two X kernels,
    the transposed backward chain): forward against the oracle, the backward of an
    arbitrary half spectrum against the oracle's staged C2R, and the round trip, at 1e-12."""
    n = 512
    print("case 512^3 FP64", flush=True)
    u = synth.grf(3, (n, n, n)).astype(np.float64)
    with pf.Plan(n, n, n, pf.Layout(precision=pf.PF_F64)) as plan:
        assert plan.pass_kernel(pf.PF_DIR_FORWARD, 0) == "r2c_pow2"
        assert plan.pass_kernel(pf.PF_DIR_BACKWARD, 2) == "c2r_pow2"
        assert plan.workspace_layout(pf.PF_DIR_BACKWARD) == pf.PF_WS_TRANSPOSED
        Ud = plan.ftran(torch.from_numpy(u).cuda())
        assert rel(Ud.cpu().numpy(), oracle.to_stride1(oracle.r2c3d(u))) < 1e-12
        back = plan.btran(Ud)
        del Ud
        assert rel(back.cpu().numpy() / u.size, u) < 1e-12
        del back
        V = synth.complex_half(6, (n, n, n // 2 + 1))
        vd = plan.btran(torch.from_numpy(oracle.to_stride1(V)).cuda())
        assert rel(vd.cpu().numpy(), oracle.c2r3d(V, n)) < 1e-12


@pytest.mark.timeout(600)
def test_2048_cubed_round_trip_and_parseval():
    """A grid eight times the benchmark's (2048^3 FP32, 34 GB per array; the
    power-of-two kernels with 8-column Y / Z tiles and the 1024-point X
    kernel): properties that hold at any size, reduced on the device in FP64
    chunks -- the round trip returns N u, and Parseval holds with the
    half-spectrum weights (1 for kx = 0 and nx/2, 2 otherwise)."""
    n = 2048
    print("case 2048^3 round trip and Parseval", flush=True)
    g = torch.Generator(device="cuda")
    g.manual_seed(7)
    u = torch.empty((n, n, n), device="cuda", dtype=torch.float32).uniform_(-1.0, 1.0, generator=g)
    with pf.Plan(n, n, n) as plan:
        U = plan.ftran(u)                     # STRIDE1 [kx][ky][kz]
        back = plan.btran(U)
        torch.cuda.synchronize()
        su = sd = se = 0.0
        for z in range(0, n, 64):
            uc = u[z:z + 64].double()
            su += float((uc * uc).sum())
            d = back[z:z + 64].double() / float(n) ** 3 - uc
            sd += float((d * d).sum())
        w = torch.full((n // 2 + 1,), 2.0, dtype=torch.float64, device="cuda")
        w[0] = w[-1] = 1.0
        for kx in range(0, n // 2 + 1, 64):
            Uc = U[kx:kx + 64]
            se += float((Uc.real.double() ** 2 + Uc.imag.double() ** 2).sum(dim=(1, 2)).mul(w[kx:kx + 64]).sum())
    assert (sd / su) ** 0.5 < 1e-6
    assert abs(se / float(n) ** 3 - su) <= 1e-6 * su


@pytest.mark.timeout(600)
def test_1024_cubed_single_mode_every_output():
    """Every output at the benchmark's size against a closed form: the plane wave
    cos(2 pi (3x + 5y + 7z) / 1024) has the single half-spectrum entry N/2 at
    (kx, ky, kz) = (3, 5, 7) and zeros elsewhere, and the C2R of that single
    entry is N times the wave.  Reduced on the device in FP64 chunks."""
    n = 1024
    N = float(n) ** 3
    print("case 1024^3 single mode", flush=True)
    u = torch.empty((n, n, n), device="cuda", dtype=torch.float32)
    x = torch.arange(n, device="cuda", dtype=torch.float64)
    for z in range(0, n, 64):
        zz = torch.arange(z, z + 64, device="cuda", dtype=torch.float64)[:, None, None]
        u[z:z + 64] = torch.cos(2 * np.pi * (3 * x[None, None, :] + 5 * x[None, :, None] + 7 * zz) / n).float()
    with pf.Plan(n, n, n) as plan:
        U = plan.ftran(u)                              # STRIDE1 [kx][ky][kz]
        torch.cuda.synchronize()
        peak = complex(U[3, 5, 7].item())
        U[3, 5, 7] = 0
        rest = sum(float(U[k:k + 64].abs().double().pow(2).sum()) for k in range(0, n // 2 + 1, 64)) ** 0.5
        assert abs(peak - N / 2) <= 1e-6 * N / 2
        assert rest <= 1e-6 * N / 2
        U.zero_()
        U[3, 5, 7] = N / 2
        back = plan.btran(U)
        torch.cuda.synchronize()
        num = den = 0.0
        for z in range(0, n, 64):
            b = back[z:z + 64].double()
            ref = N * u[z:z + 64].double()
            num += float((b - ref).pow(2).sum())
            den += float(ref.pow(2).sum())
        assert (num / den) ** 0.5 < 1e-6
