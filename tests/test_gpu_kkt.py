"""GPU: the paper's own inner solve (inner_solve = 1: dynamics as equality rows
with the finite penalty rho_eq, the quasi-definite KKT matrix of
Eq. (kkt_system) factored once per solve and solved by substitution every
iteration) against the oracle's (oracle/kkt.py, which factors the full KKT
matrix by a banded LDL^T in a different elimination order), through the C ABI.

Every component of the iterate is compared per agent -- the states are ADMM
variables here, not a rollout -- at 1e-10 (FP64) and 1e-5 (FP32, u_0 and the
trajectory), cold, warm from the GPU's own iterate, and resumed through
mpc_set_warm_kkt; the residual report equals the oracle's residuals of the
oracle's iterate.  As rho_eq grows the iterate approaches the exact-dynamics
(Riccati) path's.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from oracle import kkt as KKT
from paper_2510_12717_amd import mpc, synth

from test_gpu_parity import agent_errors

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5}
ARGS = ("s", "A", "B", "c", "q", "r", "x_ref", "x0", "tau_max", "mu", "stance")


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


def _rel_blocks(b, got, want, key):
    off = b.offsets()
    out = []
    for a in range(b.n_agents):
        g = got[off[key][a]:off[key][a + 1]].astype(np.float64)
        w = want[off[key][a]:off[key][a + 1]]
        out.append(np.abs(g - w).max() / max(np.abs(w).max(), 1e-300))
    return np.array(out)


def _get(plan):
    return {k: v.cpu().numpy() for k, v in plan.get_solution().items()}


@pytest.mark.parametrize("precision,kind", [("fp64", "humanoid"), ("fp32", "humanoid"),
                                            ("fp64", "uneven"), ("fp32", "uneven")])
def test_kkt_inner_solve_matches_oracle_cold_and_warm(precision, kind):
    b = _batch(kind, precision)
    plan = mpc.Plan(b.shapes, precision=precision, iters=50, inner_solve=1)
    assert plan.config()["kernel"] == "generic"
    prob = mpc.to_device(b, precision)
    plan.solve(prob)
    g = _get(plan)
    assert np.all(g["status"] == 0)
    o = KKT.solve_batch(b, iters=50)
    e = agent_errors(b, g, o)
    ex = _rel_blocks(b, g["x"], o["x"], "x")
    ezd = _rel_blocks(b, g["zd"], o["zd"], "c")
    eyd = _rel_blocks(b, g["yd"], o["yd"], "c")
    print(f"{precision} {kind} cold: max u0/traj/z/y {e.max(axis=0)} x {ex.max():.2e} "
          f"zd {ezd.max():.2e} yd {eyd.max():.2e}")
    assert e[:, :2].max() < TOL[precision]
    if precision == "fp64":
        assert max(e.max(), ex.max(), ezd.max(), eyd.max()) < TOL["fp64"]
        # the residual report: the oracle's residuals of the oracle's iterate
        off = b.offsets()
        for a in range(b.n_agents):
            ag = oracle.agent(b, a)
            s = ag["s"]
            m = s.nu + 4 * s.n_feet
            res, obj = oracle.residuals(*[ag[k] for k in ARGS],
                                        o["x"][off["x"][a]:off["x"][a + 1]].reshape(s.N + 1, s.nx),
                                        o["u"][off["u"][a]:off["u"][a + 1]].reshape(s.N, s.nu),
                                        o["z"][off["z"][a]:off["z"][a + 1]].reshape(s.N, m),
                                        o["y"][off["z"][a]:off["z"][a + 1]].reshape(s.N, m))
            assert np.allclose(g["residuals"][a], res, rtol=1e-7, atol=1e-12)
            assert g["objective"][a] == pytest.approx(obj, rel=1e-10)
    # warm: the next control step from the GPU's own iterate
    x0n = (b.x0 + 0.01 * np.random.default_rng(4).standard_normal(b.x0.shape)).astype(b.x0.dtype)
    prob["x0"] = torch.from_numpy(x0n).cuda()
    plan.solve(prob, warm_start=True)
    g2 = _get(plan)
    warm = {k: g[k].astype(np.float64) for k in ("x", "u", "z", "y", "zd", "yd")}
    o2 = KKT.solve_batch(b, iters=50, warm=warm, x0=x0n)
    e2 = agent_errors(b, g2, o2)
    print(f"{precision} {kind} warm: max u0/traj/z/y {e2.max(axis=0)}")
    assert np.all(g2["status"] == 0) and e2[:, :2].max() < TOL[precision]


def test_set_warm_kkt_resumes_the_iterate():
    b = _batch("humanoid", "fp64")
    o = KKT.solve_batch(b, iters=30)
    plan = mpc.Plan(b.shapes, precision="fp64", iters=20, inner_solve=1)
    prob = mpc.to_device(b, "fp64")
    with pytest.raises(mpc.MPCError):  # no iterate to start from yet
        plan.solve(prob, warm_start=True)
    plan.set_warm_state(*(torch.from_numpy(o[k]).cuda() for k in ("u", "z", "y")))
    plan.set_warm_kkt(*(torch.from_numpy(o[k]).cuda() for k in ("x", "zd", "yd")))
    plan.solve(prob, warm_start=True)
    g = _get(plan)
    whole = KKT.solve_batch(b, iters=50)
    assert agent_errors(b, g, whole).max() < 1e-9
    assert _rel_blocks(b, g["x"], whole["x"], "x").max() < 1e-9


def test_large_rho_eq_approaches_the_riccati_path():
    """The exact-dynamics path is the rho_eq -> infinity limit of this one."""
    b = _batch("humanoid", "fp64")
    prob = mpc.to_device(b, "fp64")
    ric = mpc.Plan(b.shapes, precision="fp64", iters=50)
    ric.solve(prob)
    gr = _get(ric)
    near = mpc.Plan(b.shapes, precision="fp64", iters=50, inner_solve=1, rho_eq_scale=1e7)
    near.solve(prob)
    gn = _get(near)
    far = mpc.Plan(b.shapes, precision="fp64", iters=50, inner_solve=1)
    far.solve(prob)
    gf = _get(far)
    en = agent_errors(b, gn, gr)[:, :2].max()
    ef = agent_errors(b, gf, gr)[:, :2].max()
    print(f"KKT vs Riccati path: rho_eq 1e2 {ef:.2e}, rho_eq 1e6 {en:.2e}")
    assert en < 1e-4 and ef > 10 * en


def test_kkt_plans_check_their_settings():
    b = _batch("humanoid", "fp32")
    for bad in (dict(precision="bf16"), dict(precision="fp32", kernel="fused"),
                dict(precision="fp32", scaling_iters=5), dict(precision="fp32", rho_interval=10),
                dict(precision="fp32", joint_limits=1), dict(precision="fp32", no_slip=1),
                dict(precision="fp32", inner_solve=2)):
        kw = dict(inner_solve=1)
        kw.update(bad)
        with pytest.raises(mpc.MPCError):
            mpc.Plan(b.shapes, **kw)
    plain = mpc.Plan(b.shapes, precision="fp32")
    with pytest.raises(mpc.MPCError):
        plain.set_warm_kkt(torch.zeros(1, device="cuda"), torch.zeros(1, device="cuda"),
                           torch.zeros(1, device="cuda"))
