"""GPU: joint limits of Eq. (mpc_formulation) (state rows x_lo <= x_k <= x_hi,
k = 1..N) against the oracle, through the C ABI.

Plans created with joint_limits = 1 run the generic kernels (FP64 and FP32);
compared per agent with the oracle's solve on the same data and limits (FP32
data widened exactly): u_0 and the trajectory at 1e-10 (FP64) / 1e-5 (FP32),
z, y and the state rows' z_x, y_x at the same bars for FP64, the residual
report, cold and warm-started from the GPU's own first solve.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2510_12717_amd import mpc, synth

from test_gpu_parity import agent_errors

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    mpc.lib()


def _batch(kind, precision):
    dt = np.float64 if precision == "fp64" else np.float32
    if kind == "humanoid":
        return synth.humanoid_batch(agent_ids=np.arange(0, 4096, 256), dtype=dt)
    return synth.uneven_batch(agent_ids=np.arange(0, 8192, 512), dtype=dt)


def _rel_blocks(b, got, want, scale, key_scale):
    """Per-agent max |got - want| over the agent's state rows, relative to the
    largest of |want| and of the agent's ``scale`` block (an agent whose limits
    never bind has y_x at rounding level: it is measured against the
    multipliers y of the same problem, z_x against its z)."""
    off = b.offsets()
    e = []
    for a in range(b.n_agents):
        g = got[off["c"][a]:off["c"][a + 1]].astype(np.float64)
        w = want[off["c"][a]:off["c"][a + 1]]
        sc = scale[off[key_scale][a]:off[key_scale][a + 1]]
        e.append(np.abs(g - w).max() / max(np.abs(w).max(), np.abs(sc).max(), 1e-300))
    return np.array(e)


@pytest.mark.parametrize("precision,kind", [("fp64", "humanoid"), ("fp32", "humanoid"),
                                            ("fp64", "uneven"), ("fp32", "uneven")])
def test_joint_limits_match_oracle_cold_and_warm(precision, kind):
    b = _batch(kind, precision)
    lo, hi = synth.joint_limits(b)
    plan = mpc.Plan(b.shapes, precision=precision, iters=50, joint_limits=1)
    assert plan.config()["kernel"] == "generic"
    prob = mpc.to_device(b, precision)
    td = prob["A"].dtype
    prob["x_lo"] = torch.from_numpy(lo).to(td).cuda()
    prob["x_hi"] = torch.from_numpy(hi).to(td).cuda()
    plan.solve(prob)
    g = {k: v.cpu().numpy() for k, v in plan.get_solution().items()}
    assert np.all(g["status"] == 0)
    o = oracle.solve_batch(b, iters=50, x_lo=lo, x_hi=hi)
    e = agent_errors(b, g, o)
    ezx = _rel_blocks(b, g["zx"], o["zx"], o["x"], "x")
    eyx = _rel_blocks(b, g["yx"], o["yx"], o["y"], "z")
    print(f"{precision} {kind} cold: max u0/traj/z/y {e.max(axis=0)} zx {ezx.max():.2e} yx {eyx.max():.2e}")
    assert np.count_nonzero(np.abs(o["yx"]) > 1e-3) > 0  # limits are active on these problems
    assert e[:, :2].max() < TOL[precision]
    if precision == "fp64":
        assert max(e.max(), ezx.max(), eyx.max()) < TOL["fp64"]
        assert np.allclose(g["residuals"], o["res"], rtol=1e-7, atol=1e-12)
    else:
        assert ezx.max() < 10 * TOL["fp32"]
    # warm: the next control step from the GPU's own iterate
    x0n = (b.x0 + 0.01 * np.random.default_rng(3).standard_normal(b.x0.shape)).astype(b.x0.dtype)
    prob["x0"] = torch.from_numpy(x0n).cuda()
    plan.solve(prob, warm_start=True)
    g2 = {k: v.cpu().numpy() for k, v in plan.get_solution().items()}
    warm = {k: g[k].astype(np.float64) for k in ("u", "z", "y", "zx", "yx")}
    o2 = oracle.solve_batch(b, iters=50, warm=warm, x0=x0n, x_lo=lo, x_hi=hi)
    e2 = agent_errors(b, g2, o2)
    print(f"{precision} {kind} warm: max u0/traj/z/y {e2.max(axis=0)}")
    assert np.all(g2["status"] == 0) and e2[:, :2].max() < TOL[precision]


def test_set_warm_limits_resumes_the_state_rows():
    b = _batch("humanoid", "fp64")
    lo, hi = synth.joint_limits(b)
    o = oracle.solve_batch(b, iters=30, x_lo=lo, x_hi=hi)
    plan = mpc.Plan(b.shapes, precision="fp64", iters=20, joint_limits=1)
    prob = mpc.to_device(b, "fp64")
    prob["x_lo"], prob["x_hi"] = torch.from_numpy(lo).cuda(), torch.from_numpy(hi).cuda()
    plan.set_warm_state(*(torch.from_numpy(o[k]).cuda() for k in ("u", "z", "y")))
    plan.set_warm_limits(torch.from_numpy(o["zx"]).cuda(), torch.from_numpy(o["yx"]).cuda())
    plan.solve(prob, warm_start=True)
    g = {k: v.cpu().numpy() for k, v in plan.get_solution().items()}
    whole = oracle.solve_batch(b, iters=50, x_lo=lo, x_hi=hi)
    e = agent_errors(b, g, whole)
    assert e.max() < 1e-9


def test_joint_limit_plans_check_their_inputs():
    b = _batch("humanoid", "fp32")
    lo, hi = synth.joint_limits(b)
    prob = mpc.to_device(b, "fp32")
    plan = mpc.Plan(b.shapes, precision="fp32", joint_limits=1)
    with pytest.raises(mpc.MPCError) as ei:
        plan.solve(prob)  # limits required
    assert ei.value.code == mpc.MPC_ERR_INVALID_ARG
    plain = mpc.Plan(b.shapes, precision="fp32")
    prob["x_lo"], prob["x_hi"] = torch.from_numpy(lo).cuda(), torch.from_numpy(hi).cuda()
    with pytest.raises(mpc.MPCError):
        plain.solve(prob)  # a plan without limits refuses them
    for bad in (dict(precision="bf16"), dict(precision="fp32", scaling_iters=5),
                dict(precision="fp32", kernel="fused")):
        with pytest.raises(mpc.MPCError):
            mpc.Plan(b.shapes, joint_limits=1, **bad)
    # a box that excludes every point marks the agent, not the batch
    bad_lo = lo.copy()
    bad_lo[5] = 1.0
    bad_hi = hi.copy()
    bad_hi[5] = 0.0
    prob["x_lo"], prob["x_hi"] = torch.from_numpy(bad_lo).cuda(), torch.from_numpy(bad_hi).cuda()
    plan.solve(prob)
    st = plan.get_solution()["status"].cpu().numpy()
    assert st[0] == mpc.AGENT_NONFINITE and np.all(st[1:] == 0)
