"""mpc_solve_noalloc (no plan, no device allocation, scratch in a library-held
device array) against mpc_solve on the same inputs, through the C ABI.

Three calls in a row share the one scratch array: 480 humanoid agents at
N = 10 (the iteration kernel with one wavefront per stage), then a smaller
batch of 96 quadruped agents at N = 14 (the streaming kernel), then the same
quadruped batch warm-started from the iterate the second call left in the
caller's buffers.  Each must equal a plan's solve of the same batch: the same
kernels run on the same inputs, so every output is compared bit for bit; the
oracle checks u_0 of a few agents at the FP32 tolerance.  A batch beyond the
scratch limit is rejected before anything is launched.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2510_12717_amd import mpc, synth

pytestmark = pytest.mark.gpu

TOL_FP32 = 1e-5
KEYS = ("u0", "x", "u", "z", "y", "objective", "residuals", "status")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    mpc.lib()


def _plan_solution(plan, prob, warm):
    plan.solve(prob, warm_start=warm)
    return plan.get_solution()


def _compare(got, ref, what):
    torch.cuda.synchronize()
    for k in KEYS:
        assert torch.equal(got[k], ref[k]), f"{what}: {k} differs from mpc_solve " \
            f"(max |diff| {(got[k].double() - ref[k].double()).abs().max().item():.3e})"
    assert bool((got["status"] == 0).all()), f"{what}: status {got['status'].unique()}"


def _u0_vs_oracle(got, batch, ids, nu, warm=None):
    sub_ref = oracle.solve_batch(batch, iters=50, warm=warm)
    u0 = got["u0"].view(batch.n_agents, nu).double().cpu().numpy()[ids]
    uo = sub_ref["u"].reshape(batch.n_agents, -1)[ids, :nu]
    err = (np.abs(u0 - uo).max(1) / np.abs(uo).max(1)).max()
    assert err < TOL_FP32, err
    return sub_ref


def test_noalloc_matches_plan_on_consecutive_calls():
    # call 1: humanoid, N = 10
    hb = synth.make_batch([synth.humanoid(10)] * 480, stream_id=1, dtype=np.float32)
    hp = mpc.to_device(hb, "fp32")
    plan_h = mpc.Plan(hb.shapes, precision="fp32", kernel="fused")
    ref_h = _plan_solution(plan_h, hp, False)
    out_h = mpc.solution_buffers(hb.shapes)
    mpc.solve_noalloc(hb.shapes, hp, out_h)
    _compare(out_h, ref_h, "humanoid N=10")

    # call 2: a smaller batch of another shape and the streaming kernel
    qb = synth.make_batch([synth.quadruped(14)] * 96, stream_id=7, dtype=np.float32)
    qp = mpc.to_device(qb, "fp32")
    plan_q = mpc.Plan(qb.shapes, precision="fp32", kernel="fused")
    ref_q = _plan_solution(plan_q, qp, False)
    out_q = mpc.solution_buffers(qb.shapes)
    mpc.solve_noalloc(qb.shapes, qp, out_q)
    _compare(out_q, ref_q, "quadruped N=14")

    # call 3: warm start from the caller's buffers (the second call's iterate)
    ref_w = _plan_solution(plan_q, qp, True)
    mpc.solve_noalloc(qb.shapes, qp, out_q, warm_start=True)
    _compare(out_q, ref_w, "quadruped N=14 warm")

    # the oracle on a few agents of each call
    q64 = synth.make_batch([synth.quadruped(14)] * 96, stream_id=7)
    ids = np.arange(0, 96, 12)
    cold = _u0_vs_oracle(ref_q, q64, ids, 24)
    _u0_vs_oracle(out_q, q64, ids, 24, warm={k: ref_q[k].double().cpu().numpy() for k in ("u", "z", "y")})
    del cold
    h64 = synth.make_batch([synth.humanoid(10)] * 480, stream_id=1)
    _u0_vs_oracle(out_h, h64, np.arange(0, 480, 60), 30)
    plan_h.close()
    plan_q.close()


def test_noalloc_rejects_batches_beyond_scratch():
    sh = synth.humanoid(20)
    n = 2000  # 2000 humanoid agents at N = 20 need far more than the scratch
    shapes = [sh] * n
    hb = synth.make_batch([sh] * 2, stream_id=1, dtype=np.float32)
    prob = mpc.to_device(hb, "fp32")
    out = mpc.solution_buffers(hb.shapes)
    with pytest.raises(mpc.MPCError) as ei:
        mpc.solve_noalloc(shapes, prob, out)
    assert ei.value.code == mpc.MPC_ERR_UNSUPPORTED_SHAPE
    assert "scratch" in str(ei.value)
    # a mixed-shape batch and another precision are refused as well
    with pytest.raises(mpc.MPCError):
        mpc.solve_noalloc([synth.humanoid(10), synth.humanoid(11)], prob, out)
