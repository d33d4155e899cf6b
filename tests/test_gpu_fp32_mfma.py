"""GPU: MPC_FP32_MFMA, the register-resident kernels with the Riccati factor's
block products on the FP32 matrix cores.

The factor's products P B_k, P A_k, B_k'P B_k, B_k'P A_k and the closed-loop
update take FP32 operands (rounded to nearest from the FP64 values the
recursion keeps in LDS) with FP32 accumulation (v_mfma_f32_16x16x4f32); the
stage-Hessian inverse, K_k = -H_k^{-1} G_k and everything after the factor are
the MPC_FP32 plan's.  A product over K <= 48 terms carries a relative error of
about sqrt(K) u_32 (u_32 = 2^-24 = 6e-8), and the 50 fixed iterations magnify an
operator error about 60-fold, which leaves the iterate near the FP32 path's own
error; the mode therefore runs without refinement and meets the FP32 tolerance
(1e-5) against the FP64 oracle: every agent of a small and an uneven batch,
every 16th agent of the 4096-agent humanoid batch, agents that fail stay
local, the persistent launch and the served loop give the plan's results bit
for bit, and the solution differs from the FP64-product plan's (so the FP32
products did run) by no more than the tolerance.  The GPU's own warm-started
100-step loop is checked in tests/test_gpu_warm_closed_loop.py.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2510_12717_amd import mpc, synth

from test_gpu_parity import TOL, agent_errors

pytestmark = pytest.mark.gpu

KEYS = ("u", "x", "z", "y", "status", "residuals", "objective")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    mpc.lib()


def _solve(b, precision="fp32mfma", kernel="auto", steps=1):
    plan = mpc.Plan(b.shapes, precision=precision, iters=50, kernel=kernel)
    prob = mpc.to_device(b, "fp32")
    for k in range(steps):
        plan.solve(prob, warm_start=k > 0)
    return plan, prob


def _np(plan):
    return {k: v.cpu().numpy() for k, v in plan.get_solution().items()}


@pytest.mark.parametrize("which", ["small", "uneven"])
def test_every_agent_matches_oracle(which):
    b = synth.small_humanoid_batch(64) if which == "small" else synth.uneven_batch(128)
    b = b.astype(np.float32)
    plan, _ = _solve(b)
    assert plan.config()["kernel"] == "fused"
    g = _np(plan)
    assert np.all(g["status"] == 0)
    e = agent_errors(b, g, oracle.solve_batch(b, iters=50))
    print(which, "fp32 matrix-core products: max u0/traj", e[:, :2].max(axis=0))
    assert e[:, :2].max() < TOL["fp32"]


def test_humanoid_4096_sampled():
    b = synth.humanoid_batch(4096, dtype=np.float32)
    plan, _ = _solve(b)
    g = _np(plan)
    assert np.all(g["status"] == 0)
    ids = np.arange(0, 4096, 16)
    sub = synth.humanoid_batch(agent_ids=ids)
    o = oracle.solve_batch(sub, iters=50)
    o["_off"] = sub.offsets()
    e = agent_errors(b, g, o, agents=ids, go=np.arange(len(ids)))
    print("humanoid_batch sampled, fp32 products: max u0/traj", e[:, :2].max(axis=0))
    assert e[:, :2].max() < TOL["fp32"]


def test_differs_from_fp64_products_within_tolerance():
    b = synth.uneven_batch(96).astype(np.float32)
    pm, _ = _solve(b)
    pd, _ = _solve(b, precision="fp32")
    gm, gd = _np(pm), _np(pd)
    assert not np.array_equal(gm["u"], gd["u"])
    off = b.offsets()
    for a in range(b.n_agents):
        u = slice(off["u"][a], off["u"][a + 1])
        assert np.abs(gm["u"][u] - gd["u"][u]).max() <= 2 * TOL["fp32"] * np.abs(gd["u"][u]).max(), a


def test_failures_stay_local():
    b = synth.small_humanoid_batch(6)
    o_ = b.offsets()
    b.A[o_["A"][2] + 17] = np.nan
    b.r[o_["r"][4]:o_["r"][5]] = -5.0
    b = b.astype(np.float32)
    plan, _ = _solve(b)
    g = _np(plan)
    o = oracle.solve_batch(b, iters=50)
    assert g["status"].tolist() == o["status"].tolist() == [0, 0, 3, 0, 2, 0]
    assert agent_errors(b, g, o, agents=[0, 1, 3, 5])[:, :2].max() < TOL["fp32"]


def test_persistent_launch_bit_for_bit():
    b = synth.uneven_batch(160).astype(np.float32)
    pf, _ = _solve(b, kernel="fused", steps=3)
    pp, _ = _solve(b, kernel="persistent", steps=3)
    sf, sp = pf.get_solution(), pp.get_solution()
    for k in KEYS:
        assert torch.equal(sf[k], sp[k]), k


def test_served_loop_matches_plan():
    b = synth.uneven_batch(48).astype(np.float32)
    prob = mpc.to_device(b, "fp32")
    plan = mpc.Plan(b.shapes, precision="fp32mfma", iters=50)
    off = b.offsets()
    srv = mpc.Server(precision="fp32mfma", max_batch=16, max_inflight=2)
    reqs = mpc.agent_problems(prob, b)
    bufs = [torch.full((s.nu,), float("nan"), device="cuda") for s in b.shapes]
    st = torch.full((b.n_agents,), -1, dtype=torch.int32, device="cuda")
    for step in range(2):
        plan.solve(prob, warm_start=step > 0)
        u = plan.get_solution()["u"].cpu()
        for a, s in enumerate(b.shapes):
            srv.submit(a, s, reqs[a], bufs[a], warm=True, status_out=st[a:a + 1])
        srv.drain()
        torch.cuda.synchronize()
        for a, s in enumerate(b.shapes):
            assert torch.equal(bufs[a].cpu(), u[off["u"][a]:off["u"][a] + s.nu]), (step, a)
        assert (st == 0).all()
    long = synth.make_batch([synth.humanoid(30)], seed=1, stream_id=60).astype(np.float32)
    pl = mpc.to_device(long, "fp32")
    with pytest.raises(mpc.MPCError) as ei:
        srv.submit(99, long.shapes[0], mpc.agent_problems(pl, long)[0], bufs[0])
    assert ei.value.code == mpc.MPC_ERR_UNSUPPORTED_SHAPE
    srv.drain()


def test_rejections():
    with pytest.raises(mpc.MPCError) as ei:   # no register-resident instantiation beyond N = 20
        mpc.Plan([synth.humanoid(10), synth.humanoid(30)], precision="fp32mfma")
    assert ei.value.code == mpc.MPC_ERR_UNSUPPORTED_SHAPE
    for kw in (dict(kernel="generic"), dict(joint_limits=1), dict(no_slip=1), dict(inner_solve=1),
               dict(riccati_scan=1)):
        with pytest.raises(mpc.MPCError) as ei:
            mpc.Plan([synth.humanoid(10)], precision="fp32mfma", **kw)
        assert ei.value.code == mpc.MPC_ERR_INVALID_ARG, kw
