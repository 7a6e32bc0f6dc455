"""The matrix-core precision variant: the middle radix-16 stage of the
power-of-two passes as DFT-matrix products with split half-precision operands
(hi + lo, FP32 accumulation), FP16 (per-butterfly power-of-two scale) and
BF16.  Checked against the FP64 oracle at the stated bounds: FP16 x 2 within
1e-6 relative L2 (FP32 class), BF16 x 2 within 1e-5.  The variant must run
(results differ from the plain FP32 path by rounding) and be deterministic.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1905_02803_amd as pf  # noqa: E402

BOUND = {pf.PF_MFMA_FP16X2: 1e-6, pf.PF_MFMA_BF16X2: 1e-5}

SHAPES = [
    (8, 1024, 40),    # (nz, ny, nx): Y = 1024 on the matrix cores
    (1024, 6, 40),    # Z = 1024
    (6, 10, 1024),    # X: nx = 1024, half-length 512 on the matrix cores
    (12, 512, 2048),  # Y = 512, X half-length 1024
    (16, 24, 1024),   # tiles crossing z planes in the X stage
]


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.mark.parametrize("stride1", [1, 0])
@pytest.mark.parametrize("math", [pf.PF_MFMA_FP16X2, pf.PF_MFMA_BF16X2])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s[::-1])))
def test_mfma_variant_matches_oracle(shape, math, stride1):
    """Forward, backward and round trip at the variant's bound, for both Z-pencil
    layouts: stride1 = 0 runs the Z passes on the unaligned [nz][ny][nxh] rows
    (column-at-a-time accesses traded between lanes) around the matrix-core stages."""
    nz, ny, nx = shape
    print(f"case shape={shape} math={math} stride1={stride1}", flush=True)
    u = synth.grf(31, shape) if nx * ny * nz > 1 << 16 else synth.uniform(31, shape).astype(np.float32)
    ud = torch.from_numpy(u).cuda()
    to_layout = oracle.to_stride1 if stride1 else (lambda a: a)
    with pf.Plan(nx, ny, nz, pf.Layout(math=math, stride1=stride1)) as pm, \
            pf.Plan(nx, ny, nz, pf.Layout(stride1=stride1)) as pp:
        Um = pm.ftran(ud).clone()
        Um2 = pm.ftran(ud).clone()
        Up = pp.ftran(ud)
        bm = pm.btran(Um)
        torch.cuda.synchronize()
        assert torch.equal(Um, Um2)
        assert not torch.equal(Um, Up)  # the matrix-core stage really ran
        ref = to_layout(oracle.r2c3d(u))
        ef = rel(Um.cpu().numpy(), ref)
        rt = rel(bm.cpu().numpy() / u.size, u)
        V = synth.complex_half(32, (nz, ny, nx // 2 + 1)).astype(np.complex64)
        vb = pm.btran(torch.from_numpy(np.ascontiguousarray(to_layout(V))).cuda())
        torch.cuda.synchronize()
        eb = rel(vb.cpu().numpy(), oracle.c2r3d(V, nx))
        print(f"forward {ef:.3e} backward {eb:.3e} round trip {rt:.3e}", flush=True)
        assert ef < BOUND[math] and eb < BOUND[math] and rt < 2 * BOUND[math]


def test_mfma_option_requires_f32():
    with pytest.raises(pf.PfError) as e:
        pf.Plan(32, 32, 32, pf.Layout(math=pf.PF_MFMA_FP16X2, precision=pf.PF_F64))
    assert e.value.code == pf.PF_EUNSUPPORTED


@pytest.mark.parametrize("math", [pf.PF_MFMA_FP16X2, pf.PF_MFMA_BF16X2])
def test_mfma_with_chebyshev_third_transform(math):
    """Matrix-core X and Y stages (nx = 1024, ny = 512) with the type-I DCT along
    z (plain arithmetic, extension 512 on the power-of-two kernel): forward and
    backward against the oracle's composition at the variant's bound."""
    nz, ny, nx = 257, 512, 1024
    print(f"case mfma + cheb math={math}", flush=True)
    u = synth.uniform(33, (nz, ny, nx)).astype(np.float32)
    with pf.Plan(nx, ny, nz, pf.Layout(math=math, third=pf.PF_THIRD_CHEB)) as plan:
        got = plan.ftran(torch.from_numpy(u).cuda()).cpu().numpy()
        assert rel(got, oracle.to_stride1(oracle.r2c3d_cheb(u))) < BOUND[math]
        V = synth.complex_half(34, (nz, ny, nx // 2 + 1)).astype(np.complex64)
        back = plan.btran(torch.from_numpy(oracle.to_stride1(V)).cuda()).cpu().numpy()
        assert rel(back, oracle.c2r3d_cheb(V, nx)) < BOUND[math]
