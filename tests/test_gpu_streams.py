"""The entry points enqueue on the stream they are given.

Each case prepares its input on a side stream (default priority) behind a queue
of copies, runs the transform on that stream and synchronises only that stream:
the results must equal, bitwise, the same calls on the default stream.  A call
that ran on another stream would race the copies that produce its input.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1905_02803_amd as pf  # noqa: E402


def _queued_copy(src, s, n=20):
    """src copied n times on stream s (the last copy is the input)."""
    with torch.cuda.stream(s):
        u = torch.empty_like(src)
        for _ in range(n):
            u.copy_(src)
    return u


@pytest.mark.parametrize("shape", [(64, 256, 512), (24, 20, 36)])  # power-of-two and mixed-radix paths
def test_plan_runs_on_the_given_stream(shape):
    nz, ny, nx = shape
    src = torch.from_numpy(synth.uniform(3, shape).astype(np.float32)).cuda()
    with pf.Plan(nx, ny, nz) as plan:
        ref = plan.ftran(src)
        ref_back = plan.btran(ref)
        torch.cuda.synchronize()
        s = torch.cuda.Stream()
        u = _queued_copy(src, s)
        with torch.cuda.stream(s):
            U = plan.empty_complex()
            plan.ftran(u, U, stream=s)
            back = plan.btran(U, stream=s)
        s.synchronize()
        assert torch.equal(U, ref) and torch.equal(back, ref_back)


def test_batch_and_graph_run_on_the_given_stream():
    dims = [(36, 20, 24), (48, 30, 10), (64, 16, 12)]
    with pf.Batch(dims, mode=pf.PF_BATCH_FUSED | pf.PF_BATCH_GRAPH) as b:
        R = b.empty(0).zero_()
        for i, (nx, ny, nz) in enumerate(dims):
            b.view(R, 0, i).copy_(torch.from_numpy(synth.uniform(10 + i, (nz, ny, nx)).astype(np.float32)))
        C_ref = b.empty(1).zero_()
        b.ftran(R, C_ref)
        torch.cuda.synchronize()
        s = torch.cuda.Stream()
        for rep in range(2):  # capture, then replay
            Rq = _queued_copy(R, s)
            with torch.cuda.stream(s):
                C = torch.zeros_like(C_ref)
                b.ftran(Rq, C, stream=s)
            s.synchronize()
            assert torch.equal(C, C_ref), rep


def test_spectral_step_runs_on_the_given_stream():
    nz, ny, nx = 129, 16, 32  # fused z pass (extension 256)
    src = torch.from_numpy(synth.uniform(12, (nz, ny, nx)).astype(np.float32)).cuda()
    with pf.Plan(nx, ny, nz, pf.Layout(third=pf.PF_THIRD_CHEB)) as plan:
        ref = pf.spectral_step(plan, src)
        ref_t = pf.spectral_step(plan, src, adjoint=True)
        torch.cuda.synchronize()
        s = torch.cuda.Stream()
        u = _queued_copy(src, s)
        with torch.cuda.stream(s):
            y = pf.spectral_step(plan, u, stream=s)
            yt = pf.spectral_step(plan, u, adjoint=True, stream=s)
        s.synchronize()
        assert torch.equal(y, ref) and torch.equal(yt, ref_t)
