"""Batched transforms of many uneven grids (each dimension a 7-smooth length
in [48, 320], odd ones included; the paper's arbitrary grid sizes, Sec. 3.1).

Every transform of a batch must match the oracle (FP32 1e-6, FP64 1e-12),
in every execution mode (one transform at a time, one fused launch per pass,
both replayed from a captured hipGraph, and both spread over the batch's own
streams) and with tuned radix orders and tile widths; the modes run the same
arithmetic and must agree bit for bit.
Graph replays are checked one by one, with eager work between them.
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


def small_dims(count, seed, cap=96):
    """count triples from the batch generator, each length folded below cap (still 7-smooth)."""
    out = []
    for d in synth.batch_sizes(seed, count):
        t = []
        for v in d:
            while v > cap:
                v //= 2 if v % 2 == 0 else (3 if v % 3 == 0 else (5 if v % 5 == 0 else 7))
            t.append(max(v, 1))
        out.append(tuple(t))
    return out


def fill(batch, buf, which, seed, dt):
    for i, (nx, ny, nz) in enumerate(batch.dims):
        v = batch.view(buf, which, i)
        if which == 0:
            v.copy_(torch.from_numpy(synth.uniform(seed + i, (nz, ny, nx)).astype(dt)))
        else:
            V = synth.complex_half(seed + i, (nz, ny, nx // 2 + 1)).astype(dt)
            v.copy_(torch.from_numpy(oracle.to_stride1(V) if batch.layout.stride1 else V))


def check_batch(batch, tol, seed=40):
    rdt = np.float64 if batch.layout.precision == pf.PF_F64 else np.float32
    cdt = np.complex128 if batch.layout.precision == pf.PF_F64 else np.complex64
    # buffers start zeroed so that the padding between transforms compares equal
    R = batch.empty(0).zero_()
    C = batch.empty(1).zero_()
    fill(batch, R, 0, seed, rdt)
    batch.ftran(R, C)
    Cin = batch.empty(1).zero_()
    fill(batch, Cin, 1, seed + 500, cdt)
    Rout = batch.empty(0).zero_()
    batch.btran(Cin, Rout)
    torch.cuda.synchronize()
    for i, (nx, ny, nz) in enumerate(batch.dims):
        u = batch.view(R, 0, i).cpu().numpy()
        ref = oracle.r2c3d(u)
        got = batch.view(C, 1, i).cpu().numpy()
        assert rel(got, oracle.to_stride1(ref) if batch.layout.stride1 else ref) < tol, (i, (nx, ny, nz))
        V = batch.view(Cin, 1, i).cpu().numpy()
        V = oracle.from_stride1(V) if batch.layout.stride1 else V
        assert rel(batch.view(Rout, 0, i).cpu().numpy(), oracle.c2r3d(V, nx)) < tol, (i, (nx, ny, nz))
    return R, C, Cin, Rout


@pytest.mark.parametrize("stride1", [1, 0])
@pytest.mark.parametrize("prec", [pf.PF_F32, pf.PF_F64])
def test_fused_batch_matches_oracle(prec, stride1):
    dims = small_dims(12, 4)
    print(f"case batch dims={dims} prec={prec} stride1={stride1}", flush=True)
    with pf.Batch(dims, pf.Layout(precision=prec, stride1=stride1)) as b:
        check_batch(b, 1e-12 if prec == pf.PF_F64 else 1e-6)


def test_all_modes_agree_bitwise_and_graph_replays():
    dims = small_dims(10, 7)
    print(f"case batch dims={dims}", flush=True)
    with pf.Batch(dims, mode=pf.PF_BATCH_FUSED) as b:
        R, C, Cin, Rout = check_batch(b, 1e-6)
        ref_c, ref_r = C.clone(), Rout.clone()
        for mode in (pf.PF_BATCH_SERIAL, pf.PF_BATCH_SERIAL | pf.PF_BATCH_GRAPH,
                     pf.PF_BATCH_FUSED | pf.PF_BATCH_GRAPH, pf.PF_BATCH_SERIAL | pf.PF_BATCH_STREAMS,
                     pf.PF_BATCH_FUSED | pf.PF_BATCH_STREAMS):
            b.set_mode(mode)
            for rep in range(3):  # replays of the captured graph, eager work in between
                C2 = torch.zeros_like(C)
                R2 = torch.zeros_like(Rout)
                b.ftran(R, C2)
                b.btran(Cin, R2)
                junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
                torch.cuda.synchronize()
                assert junk.isfinite()
                assert torch.equal(C2, ref_c), (mode, rep)
                assert torch.equal(R2, ref_r), (mode, rep)
        # a graph captured in one mode is not replayed in another: fused launches after serial ones
        b.set_mode(pf.PF_BATCH_SERIAL | pf.PF_BATCH_GRAPH)
        b.ftran(R, C2)
        b.set_mode(pf.PF_BATCH_FUSED | pf.PF_BATCH_GRAPH)
        b.ftran(R, C2)
        torch.cuda.synchronize()
        assert torch.equal(C2, ref_c)
        # new buffers: the graph is captured again
        b.set_mode(pf.PF_BATCH_FUSED | pf.PF_BATCH_GRAPH)
        R3 = R.clone()
        C3 = torch.zeros_like(C)
        b.ftran(R3, C3)
        torch.cuda.synchronize()
        assert torch.equal(C3, ref_c)


def test_tuned_plans_match_oracle():
    """Every radix order and a spread of tile widths, drawn per transform."""
    dims = small_dims(12, 11)
    rng = np.random.default_rng(5)
    tune = [(tuple(int(v) for v in rng.integers(0, 4, 3)), tuple(int(v) for v in rng.choice([0, 1, 2, 4, 8, 16], 3)))
            for _ in dims]
    print(f"case batch dims={dims} tune={tune}", flush=True)
    with pf.Batch(dims, tune=tune) as b:
        R, C, Cin, Rout = check_batch(b, 1e-6)
        # the fused passes split into one launch per block size here; serial
        # per-transform chains must give the same bits
        b.set_mode(pf.PF_BATCH_SERIAL)
        C2, R2 = torch.zeros_like(C), torch.zeros_like(Rout)
        b.ftran(R, C2)
        b.btran(Cin, R2)
        torch.cuda.synchronize()
        assert torch.equal(C2, C) and torch.equal(R2, Rout)
    with pf.Batch(dims, pf.Layout(precision=pf.PF_F64), tune=tune) as b:
        check_batch(b, 1e-12)


def test_batch_argument_errors():
    with pytest.raises(pf.PfError) as e:
        pf.Batch([(16, 8, 8)], pf.Layout(inplace=1))
    assert e.value.code == pf.PF_EUNSUPPORTED
    with pf.Batch([(16, 8, 8), (12, 10, 6)]) as b:
        R = b.empty(0)
        with pytest.raises(pf.PfError) as e:
            b.ftran(R, R)
        assert e.value.code == pf.PF_EALIAS
        with pytest.raises(pf.PfError) as e:
            b.set_mode(9)
        assert e.value.code == pf.PF_EINVAL
        with pytest.raises(pf.PfError) as e:
            b.set_mode(pf.PF_BATCH_GRAPH | pf.PF_BATCH_STREAMS)
        assert e.value.code == pf.PF_EUNSUPPORTED


@pytest.mark.timeout(900)
def test_full_batch_workload():
    """The benchmark's batch (synth.batch_sizes(4, 64): 64 transforms, 285.8 M points)
    in the configurations it times: fused and graph-replayed with the tuned fused
    plans, and the serial chains with the tuned serial plans.  In both, every
    transform's forward output matches the FP64 oracle at 1e-6, every
    transform's backward of an arbitrary (non-Hermitian) half spectrum matches
    the oracle's staged C2R at 1e-6, and every transform round-trips to N u;
    fused and serial results agree to rounding (their tuned radix orders
    differ)."""
    from paper_1905_02803_amd import autotune

    dims = synth.batch_sizes(4, 64)
    print(f"case full batch: {len(dims)} transforms", flush=True)
    refs_f, refs_b = {}, {}
    outs = {}
    for mode, tune in ((pf.PF_BATCH_FUSED | pf.PF_BATCH_GRAPH, autotune.tune_for(dims, mode="fused")),
                       (pf.PF_BATCH_SERIAL, autotune.tune_for(dims, mode="serial"))):
        print(f"mode {mode}", flush=True)
        with pf.Batch(dims, mode=mode, tune=tune) as b:
            R = b.empty(0).zero_()
            C = b.empty(1).zero_()
            R2 = b.empty(0).zero_()
            g = torch.Generator(device="cuda")
            g.manual_seed(4)
            for i in range(len(dims)):
                v = b.view(R, 0, i)
                v.copy_(torch.rand(v.shape, generator=g, device="cuda") * 2 - 1)
            for _ in range(2):  # the second call replays the captured graph
                b.ftran(R, C)
            b.btran(C, R2)
            Cin = b.empty(1).zero_()
            fill(b, Cin, 1, 900, np.complex64)
            Rb = b.empty(0).zero_()
            b.btran(Cin, Rb)
            torch.cuda.synchronize()
            for i, (nx, ny, nz) in enumerate(dims):
                u, back = b.view(R, 0, i), b.view(R2, 0, i)
                err = float((back / (nx * ny * nz) - u).norm() / u.norm())
                assert err < 1e-6, (i, dims[i], err)
                un = u.cpu().numpy()
                if i not in refs_f:
                    refs_f[i] = oracle.to_stride1(oracle.r2c3d(un))
                ef = rel(b.view(C, 1, i).cpu().numpy(), refs_f[i])
                assert ef < 1e-6, (mode, i, dims[i], ef)
                if i not in refs_b:
                    refs_b[i] = oracle.c2r3d(oracle.from_stride1(b.view(Cin, 1, i).cpu().numpy()), nx)
                eb = rel(b.view(Rb, 0, i).cpu().numpy(), refs_b[i])
                assert eb < 1e-6, (mode, i, dims[i], eb)
            outs[mode] = (R.clone(), C.clone())
    (Rf, Cf), (Rs, Cs) = outs[pf.PF_BATCH_FUSED | pf.PF_BATCH_GRAPH], outs[pf.PF_BATCH_SERIAL]
    assert torch.equal(Rf, Rs)
    # tuned radix orders differ between the two plan sets, so compare per transform to rounding
    with pf.Batch(dims) as b:
        for i in range(len(dims)):
            cf, cs = b.view(Cf, 1, i), b.view(Cs, 1, i)
            assert float((cf - cs).norm() / cs.norm()) < 1e-6, (i, dims[i])


@pytest.mark.parametrize("third", [pf.PF_THIRD_EMPTY, pf.PF_THIRD_CHEB], ids=["empty", "cheb"])
def test_batch_with_other_third_transforms(third):
    """The batch takes the layout's third transform too: every transform matches
    the oracle's composition (X and Y stages, then nothing or the type-I DCT
    along z), forward and backward, fused and serial bitwise equal."""
    dims = [(36, 20, 17), (48, 30, 9), (40, 16, 33)]  # nz - 1 = 16, 8, 32 for the DCT
    print(f"case batch third={third}", flush=True)
    fwd = oracle.r2c3d_third_empty if third == pf.PF_THIRD_EMPTY else oracle.r2c3d_cheb
    bwd = oracle.c2r3d_third_empty if third == pf.PF_THIRD_EMPTY else oracle.c2r3d_cheb
    outs = []
    for mode in (pf.PF_BATCH_FUSED, pf.PF_BATCH_SERIAL):
        with pf.Batch(dims, pf.Layout(third=third), mode=mode) as b:
            R = b.empty(0).zero_()
            C = b.empty(1).zero_()
            fill(b, R, 0, 60, np.float32)
            b.ftran(R, C)
            Cin = b.empty(1).zero_()
            fill(b, Cin, 1, 70, np.complex64)
            Rout = b.empty(0).zero_()
            b.btran(Cin, Rout)
            torch.cuda.synchronize()
            for i, (nx, ny, nz) in enumerate(dims):
                u = b.view(R, 0, i).cpu().numpy()
                assert rel(b.view(C, 1, i).cpu().numpy(), oracle.to_stride1(fwd(u))) < 1e-6, (i, dims[i])
                V = oracle.from_stride1(b.view(Cin, 1, i).cpu().numpy())
                assert rel(b.view(Rout, 0, i).cpu().numpy(), bwd(V, nx)) < 1e-6, (i, dims[i])
            outs.append((C.clone(), Rout.clone()))
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])
