"""GPU parity of the HIP transform against the CPU FP64 oracle, through the C ABI.

Sizes are small enough for the oracle to finish in seconds but span several
tiles, ragged column blocks (nx/2+1 not a multiple of the 16- or 8-wide
workspace blocks), an odd number of real lines (an unpaired last line in the
two-for-one X stage), every radix (2, 3, 4, 5, 7, 8, 16) and degenerate axes
of length 1.  Tolerances (relative L2 over all stored outputs): FP64 1e-12,
FP32 1e-6.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1905_02803_amd as pf  # noqa: E402

TOL = {pf.PF_F32: 1e-6, pf.PF_F64: 1e-12}

# (nz, ny, nx)
SHAPES = [
    (32, 32, 32),     # the 32^3 grid
    (24, 20, 36),     # nxh = 19: ragged second column block
    (9, 7, 15),       # all odd, odd line count
    (5, 3, 250),      # radix 2 x 5 x 5 x 5 along X
    (12, 360, 8),     # 360 = 8 x 3 x 3 x 5 along Y
    (250, 4, 6),      # long Z
    (6, 10, 480),     # 480 = 16 x 2 x 3 x 5
    (20, 14, 112),    # 112 = 16 x 7
    (49, 21, 10),     # 7 x 7 and 3 x 7
    (2, 3, 1024),     # 1024 = 16 x 16 x 4 along X
    (3, 1024, 2),     # along Y
    (1024, 2, 4),     # along Z
    (64, 64, 64),
    (256, 12, 36),    # power-of-two Z (compile-time radix path), ragged column blocks
    (16, 512, 36),    # power-of-two Y
    (1024, 6, 40),
    (3, 2048, 10),
    (4096, 2, 6),
    (5, 7, 512),      # even power-of-two X (half-length path): 35 lines, tiles cross z planes
    (3, 5, 2048),
    (40, 24, 1024),
    # transposed workspace (STRIDE1, ny a multiple of 16 up to 512): both chains in FP32,
    # FP64 backward (and forward at nx = 512); tiles of 16 lines cross z planes at ny = 16
    (4, 48, 512), (5, 32, 1024), (3, 16, 2048), (2, 512, 512), (1, 16, 512), (7, 64, 1024),
    (1, 1, 1), (1, 1, 2), (2, 1, 1), (1, 5, 3), (3, 1, 4),
]


def rel(a, b):
    a = np.asarray(a, dtype=np.complex128 if np.iscomplexobj(a) else np.float64)
    b = np.asarray(b)
    n = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (n if n > 0 else 1.0)


def np_real(prec):
    return np.float64 if prec == pf.PF_F64 else np.float32


def np_cplx(prec):
    return np.complex128 if prec == pf.PF_F64 else np.complex64


def to_layout(U, stride1):
    return oracle.to_stride1(U) if stride1 else U


def ids(shape):
    return "x".join(map(str, shape[::-1]))


@pytest.fixture(scope="module", autouse=True)
def gpu_available():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")


@pytest.mark.parametrize("stride1", [1, 0])
@pytest.mark.parametrize("prec", [pf.PF_F32, pf.PF_F64])
@pytest.mark.parametrize("shape", SHAPES, ids=ids)
def test_forward_and_backward_match_oracle(shape, prec, stride1):
    nz, ny, nx = shape
    print(f"case shape={shape} prec={prec} stride1={stride1}", flush=True)
    u = synth.uniform(100 + nx + 3 * ny + 7 * nz, shape).astype(np_real(prec))
    with pf.Plan(nx, ny, nz, pf.Layout(precision=prec, stride1=stride1)) as plan:
        ud = torch.from_numpy(u).cuda()
        Ud = plan.ftran(ud)
        torch.cuda.synchronize()
        ref = to_layout(oracle.r2c3d(u), stride1)
        assert rel(Ud.cpu().numpy(), ref) < TOL[prec]
        # input preserved (out-of-place)
        assert np.array_equal(ud.cpu().numpy(), u)
        # backward of an arbitrary half spectrum: the staged C2R
        V = synth.complex_half(200 + nx, (nz, ny, nx // 2 + 1)).astype(np_cplx(prec))
        Vd = torch.from_numpy(to_layout(V, stride1)).cuda()
        vd = plan.btran(Vd)
        torch.cuda.synchronize()
        assert rel(vd.cpu().numpy(), oracle.c2r3d(V, nx)) < TOL[prec]
        assert np.array_equal(Vd.cpu().numpy(), to_layout(V, stride1))
        # round trip returns N u
        back = plan.btran(Ud)
        torch.cuda.synchronize()
        assert rel(back.cpu().numpy() / (nx * ny * nz), u) < TOL[prec]


# the longest lines each precision accepts on every axis (FP32 8192, FP64 4096), and
# 4096 / 8192 where the power-of-two kernels stop (X above 2048, Y and Z above 4096)
MAX_CASES = [((2, 3, 8192), pf.PF_F32), ((3, 8192, 2), pf.PF_F32), ((8192, 2, 3), pf.PF_F32),
             ((2, 3, 4096), pf.PF_F32), ((3, 4096, 2), pf.PF_F32),
             ((2, 3, 4096), pf.PF_F64), ((3, 4096, 2), pf.PF_F64), ((4096, 2, 3), pf.PF_F64)]


@pytest.mark.parametrize("stride1", [1, 0])
@pytest.mark.parametrize("shape,prec", MAX_CASES, ids=lambda v: ids(v) if isinstance(v, tuple) else str(v))
def test_maximum_lengths_match_oracle(shape, prec, stride1):
    nz, ny, nx = shape
    print(f"case max shape={shape} prec={prec} stride1={stride1}", flush=True)
    u = synth.uniform(200 + nx + ny, shape).astype(np_real(prec))
    with pf.Plan(nx, ny, nz, pf.Layout(precision=prec, stride1=stride1)) as plan:
        got = plan.ftran(torch.from_numpy(u).cuda()).cpu().numpy()
        assert rel(got, to_layout(oracle.r2c3d(u), stride1)) < TOL[prec]
        V = synth.complex_half(201 + nx, (nz, ny, nx // 2 + 1)).astype(np_cplx(prec))
        back = plan.btran(torch.from_numpy(to_layout(V, stride1)).cuda()).cpu().numpy()
        assert rel(back, oracle.c2r3d(V, nx)) < TOL[prec]


@pytest.mark.parametrize("prec", [pf.PF_F32, pf.PF_F64])
@pytest.mark.parametrize("shape", [(24, 20, 36), (9, 7, 15), (6, 10, 480), (3, 1024, 2), (16, 512, 36), (1024, 6, 40),
                                   (5, 7, 512), (40, 24, 1024), (6, 32, 512), (3, 48, 1024)], ids=ids)
def test_each_pass_matches_oracle_stage(shape, prec):
    """Every kernel alone against the oracle's own stage (forward X, Y, Z; backward Z, Y, X).
    The intermediates are read in the layout the plan reports for each direction (plans
    with a power-of-two X pass and ny a multiple of 16 up to 512 use the transposed one;
    forward, FP64 plans only at nx = 512)."""
    nz, ny, nx = shape
    print(f"case shape={shape} prec={prec}", flush=True)
    tol = TOL[prec]
    u = synth.uniform(300 + nx, shape).astype(np_real(prec))
    with pf.Plan(nx, ny, nz, pf.Layout(precision=prec, stride1=1)) as plan:
        csz = 16 if prec == pf.PF_F64 else 8
        nws = plan.workspace_bytes // csz
        ws = torch.zeros(nws, dtype=plan.complex_dtype, device="cuda")
        ws2 = torch.zeros_like(ws)
        ud = torch.from_numpy(u).cuda()
        # the intermediates are transposed for plans that take the transposed chains
        # (the forward one for FP64 at nx = 512 only)
        transposed = ny % 16 == 0 and ny <= 512 and nx in ((512, 1024, 2048) if prec == pf.PF_F32 else (512, 1024))
        layout_f = plan.workspace_layout(pf.PF_DIR_FORWARD)
        ftr = transposed and (prec == pf.PF_F32 or nx == 512)
        assert layout_f == (pf.PF_WS_TRANSPOSED if ftr else pf.PF_WS_BLOCKED)
        viewf = pf.transposed_workspace_to_half_spectrum if layout_f == pf.PF_WS_TRANSPOSED \
            else pf.workspace_to_half_spectrum
        plan.run_pass(pf.PF_DIR_FORWARD, 0, ud, ws)
        torch.cuda.synchronize()
        A = oracle.stage_x_r2c(u)
        got = viewf(ws, nx, ny, nz).cpu().numpy()
        assert rel(got, A) < tol
        plan.run_pass(pf.PF_DIR_FORWARD, 1, ws, ws)
        torch.cuda.synchronize()
        A = oracle.stage_c2c(A, nx, "y", -1)
        assert rel(viewf(ws, nx, ny, nz).cpu().numpy(), A) < tol
        out = plan.empty_complex()
        plan.run_pass(pf.PF_DIR_FORWARD, 2, ws, out)
        torch.cuda.synchronize()
        A = oracle.stage_c2c(A, nx, "z", -1)
        assert rel(out.cpu().numpy(), oracle.to_stride1(A)) < tol
        # backward stages on an arbitrary half spectrum
        layout = plan.workspace_layout(pf.PF_DIR_BACKWARD)
        assert layout == (pf.PF_WS_TRANSPOSED if transposed else pf.PF_WS_BLOCKED)
        view = pf.transposed_workspace_to_half_spectrum if transposed else pf.workspace_to_half_spectrum
        V = synth.complex_half(400 + nx, (nz, ny, nx // 2 + 1)).astype(np_cplx(prec))
        Vd = torch.from_numpy(oracle.to_stride1(V)).cuda()
        plan.run_pass(pf.PF_DIR_BACKWARD, 0, Vd, ws2)
        torch.cuda.synchronize()
        B = oracle.stage_c2c(V, nx, "z", +1)
        assert rel(view(ws2, nx, ny, nz).cpu().numpy(), B) < tol
        plan.run_pass(pf.PF_DIR_BACKWARD, 1, ws2, ws2)
        torch.cuda.synchronize()
        B = oracle.stage_c2c(B, nx, "y", +1)
        assert rel(view(ws2, nx, ny, nz).cpu().numpy(), B) < tol
        r = plan.empty_real()
        plan.run_pass(pf.PF_DIR_BACKWARD, 2, ws2, r)
        torch.cuda.synchronize()
        assert rel(r.cpu().numpy(), oracle.stage_x_c2r(B, nx)) < tol


@pytest.mark.parametrize("shape", [(24, 20, 36), (64, 64, 64), (16, 512, 36), (1024, 6, 40), (40, 24, 1024)],
                         ids=ids)
def test_repeat_runs_are_bitwise_identical(shape):
    """Same input, same kernels: results must not depend on timing (catches missing barriers)."""
    nz, ny, nx = shape
    u = synth.uniform(7, shape).astype(np.float32)
    with pf.Plan(nx, ny, nz) as plan:
        ud = torch.from_numpy(u).cuda()
        a = plan.ftran(ud).clone()
        b = plan.ftran(ud).clone()
        ra = plan.btran(a).clone()
        rb = plan.btran(b).clone()
        torch.cuda.synchronize()
        assert torch.equal(a, b)
        assert torch.equal(ra, rb)


@pytest.mark.parametrize("prec", [pf.PF_F32, pf.PF_F64])
@pytest.mark.parametrize("shape", [(24, 20, 36), (9, 7, 15), (4, 32, 512)], ids=ids)
def test_inplace_matches_out_of_place(shape, prec):
    nz, ny, nx = shape
    u = synth.uniform(8, shape).astype(np_real(prec))
    with pf.Plan(nx, ny, nz, pf.Layout(precision=prec)) as p_out, \
            pf.Plan(nx, ny, nz, pf.Layout(precision=prec, inplace=1)) as p_in:
        ref = p_out.ftran(torch.from_numpy(u).cuda())
        nbytes = max(u.nbytes, ref.numel() * ref.element_size())
        buf = torch.zeros(nbytes // u.itemsize, dtype=p_in.real_dtype, device="cuda")
        buf[: u.size] = torch.from_numpy(u.reshape(-1)).cuda()
        p_in.ftran_inplace(buf)
        torch.cuda.synchronize()
        spec = buf.view(p_in.complex_dtype)[: ref.numel()].reshape(ref.shape)
        assert torch.equal(spec, ref)
        back_ref = p_out.btran(ref)
        p_in.btran_inplace(buf)
        torch.cuda.synchronize()
        assert torch.equal(buf[: u.size].reshape(u.shape), back_ref)


def test_inplace_buffer_is_checked_before_the_call():
    """The binding's in-place calls refuse a buffer that is too small, not
    16-byte aligned, not contiguous or not on the device, before anything runs."""
    nz, ny, nx = 6, 10, 16
    with pf.Plan(nx, ny, nz, pf.Layout(inplace=1)) as p_in:
        need = p_in.inplace_bytes
        assert need == max(nx * ny * nz * 4, (nx // 2 + 1) * ny * nz * 8)
        ok = torch.zeros(need // 4, dtype=torch.float32, device="cuda")
        p_in.ftran_inplace(ok)
        p_in.btran_inplace(ok)
        torch.cuda.synchronize()
        for bad in (torch.zeros(need // 4 - 4, dtype=torch.float32, device="cuda"),  # 16 bytes short
                    ok.view(torch.uint8)[4:],                                         # misaligned
                    torch.zeros(2 * need // 4, dtype=torch.float32, device="cuda")[::2],  # strided
                    torch.zeros(need // 4, dtype=torch.float32)):                     # host memory
            with pytest.raises(ValueError):
                p_in.ftran_inplace(bad)
            with pytest.raises(ValueError):
                p_in.btran_inplace(bad)
        # a view that starts inside a large enough storage but leaves too little after it
        with pytest.raises(ValueError):
            p_in.ftran_inplace(ok[4:])


@pytest.mark.parametrize("nbytes", [16, 4096, (1 << 20) + 48, 3 * 131072 + 16])
def test_probes_move_the_bytes(nbytes):
    """The bandwidth probes copy exactly the bytes asked for (partial last tile included); the in-place
    probe leaves the data as it was; nothing beyond the range is touched."""
    src = torch.randint(0, 2 ** 31 - 1, (nbytes // 4 + 64,), dtype=torch.int32, device="cuda")
    for kind in (pf.PF_PROBE_COPY, pf.PF_PROBE_TILES):
        dst = torch.full_like(src, -1)
        pf.pf_probe(kind, dst.data_ptr(), src.data_ptr(), nbytes, 0)
        torch.cuda.synchronize()
        n = nbytes // 4
        assert torch.equal(dst[:n], src[:n]), kind
        assert bool((dst[n:] == -1).all()), kind
    keep = src.clone()
    pf.pf_probe(pf.PF_PROBE_TILES_INPLACE, src.data_ptr(), src.data_ptr(), nbytes, 0)
    torch.cuda.synchronize()
    assert torch.equal(src, keep)


def test_call_errors_are_reported():
    with pf.Plan(16, 8, 4) as plan:
        u = plan.empty_real()
        U = plan.empty_complex()
        raw = u.view(torch.uint8)
        with pytest.raises(pf.PfError) as e:
            pf.pf_ftran_r2c(plan.handle, raw.data_ptr() + 4, U.data_ptr(), 0)
        assert e.value.code == pf.PF_EALIGN
        with pytest.raises(pf.PfError) as e:
            pf.pf_ftran_r2c(plan.handle, U.data_ptr(), U.data_ptr(), 0)
        assert e.value.code == pf.PF_EALIAS
        with pytest.raises(pf.PfError) as e:
            pf.pf_ftran_r2c(plan.handle, 0, U.data_ptr(), 0)
        assert e.value.code == pf.PF_EINVAL
        with pytest.raises(pf.PfError) as e:
            pf.pf_set_workspace(plan.handle, U.data_ptr(), 16)
        assert e.value.code == pf.PF_EWORKSPACE


def test_user_workspace_gives_identical_results():
    shape = (24, 20, 36)
    nz, ny, nx = shape
    u = torch.from_numpy(synth.uniform(9, shape).astype(np.float32)).cuda()
    with pf.Plan(nx, ny, nz) as a, pf.Plan(nx, ny, nz) as b:
        ws = torch.empty(b.workspace_bytes, dtype=torch.uint8, device="cuda")
        pf.pf_set_workspace(b.handle, ws.data_ptr(), ws.numel())
        ra = a.ftran(u)
        rb = b.ftran(u)
        torch.cuda.synchronize()
        assert torch.equal(ra, rb)
