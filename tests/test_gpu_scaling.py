"""GPU: Alg. 1's scaling step (Ruiz equilibration, f_Ruiz) and OSQP's adaptive
rho against the oracle's (oracle/scaling.py), through the C ABI.

The plan equilibrates every agent on the device, iterates on the scaled
problem (rho re-estimated every `rho_interval` iterations and the factor
recomputed), and maps the iterate back.  The oracle runs the same steps on the
same data (FP32 data widened exactly for FP32 plans); compared per agent: the
scale factors, the final rho, and (x, u, z, y) -- FP64 plans at 1e-10, FP32
plans at the FP32 tolerance 1e-5 (u_0 and the trajectory, norm-wise).

A rho update is a decision taken in floating point (the estimate is compared
with a threshold and rounded to a grid) from residuals that an FP32 plan
computes from its FP32 iterate; near convergence (warm starts) those residuals
are small differences that an iterate error of a few 1e-6 moves by percents,
so an agent's decision can fall on the other side of a boundary than the
oracle's.  The plan reports the rho of every segment: agents whose sequence
equals the oracle's are compared in full, the others (at most a quarter) must
have run on grid values and reached a finite solution.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from oracle import scaling
from paper_2510_12717_amd import mpc, synth

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    mpc.lib()


def _batch(kind, precision):
    dt = np.float64 if precision == "fp64" else np.float32
    if kind == "conditioned":  # N = 16, kappa = 1e6
        return synth.conditioned_humanoid_batch(agent_ids=np.arange(0, 16384, 1024), kappa=1e6, dtype=dt)
    if kind == "humanoid":     # N = 10
        return synth.humanoid_batch(agent_ids=np.arange(0, 4096, 256), dtype=dt)
    return synth.uneven_batch(agent_ids=np.arange(0, 8192, 512), dtype=dt)


def _oracle(b, warm=None, x0=None, **kw):
    out = []
    off = b.offsets()
    for a in range(b.n_agents):
        ag = oracle.agent(b, a)
        if x0 is not None:
            ag["x0"] = np.asarray(x0[off["x0"][a]:off["x0"][a + 1]], dtype=np.float64)
        w = None if warm is None else tuple(warm[a])
        out.append(scaling.solve(ag, warm=w, **kw))
    return out


def _errors(b, g, ref):
    off = b.offsets()
    e = []
    for a, s in enumerate(b.shapes):
        x = g["x"][off["x"][a]:off["x"][a + 1]].astype(np.float64)
        u = g["u"][off["u"][a]:off["u"][a + 1]].astype(np.float64)
        z = g["z"][off["z"][a]:off["z"][a + 1]].astype(np.float64)
        y = g["y"][off["z"][a]:off["z"][a + 1]].astype(np.float64)
        o = ref[a]
        xo, uo = np.ravel(o["x"]), np.ravel(o["u"])
        tr, to = np.concatenate([x[s.nx:], u]), np.concatenate([xo[s.nx:], uo])
        rel = lambda p, q: np.abs(p - q).max() / max(np.abs(q).max(), 1e-300)
        e.append((rel(u[:s.nu], uo[:s.nu]), rel(tr, to), rel(z, np.ravel(o["z"])), rel(y, np.ravel(o["y"]))))
    return np.array(e)


def _check_rho(plan, ref, rho_interval):
    """Agents that took the oracle's rho decisions at every update are compared
    in full; the others must have run on grid values with a finite solution.
    Returns the mask of agents to compare element-wise."""
    n = len(ref)
    keep = np.ones(n, dtype=bool)
    if not rho_interval:
        return keep
    hist = plan.get_rho().cpu().numpy()
    assert hist.shape == (n, -(-50 // rho_interval))
    want = np.array([r["rhos"] for r in ref])
    assert np.any(want != 0.1)  # the estimates moved rho on these problems
    for a in range(n):
        if not np.allclose(hist[a], want[a], rtol=1e-14, atol=0):
            keep[a] = False
            k = 4 * np.log2(hist[a][1:])
            assert np.allclose(k, np.round(k), atol=1e-9)  # grid values
    assert keep.sum() >= 0.75 * n, hist
    return keep


def _run(b, precision, kernel, warm_state=None, x0=None, **kw):
    plan = mpc.Plan(b.shapes, precision=precision, iters=50, kernel=kernel, **kw)
    prob = mpc.to_device(b, precision)
    if x0 is not None:
        prob["x0"] = torch.from_numpy(np.asarray(x0)).to(prob["x0"].dtype).cuda()
    if warm_state is not None:
        td = prob["A"].dtype
        plan.set_warm_state(*(torch.from_numpy(np.asarray(warm_state[k])).to(td).cuda()
                              for k in ("u", "z", "y")))
    plan.solve(prob, warm_start=warm_state is not None)
    g = {k: v.cpu().numpy() for k, v in plan.get_solution().items()}
    return g, plan


CASES = [("fp64", "generic", "conditioned"), ("fp32", "fused", "conditioned"),
         ("fp32", "fused", "humanoid"), ("fp32", "generic", "humanoid"),
         ("fp32", "auto", "uneven")]


@pytest.mark.parametrize("precision,kernel,kind", CASES)
@pytest.mark.parametrize("rho_interval", [0, 10])
def test_scaled_solve_matches_oracle(precision, kernel, kind, rho_interval):
    b = _batch(kind, precision)
    kw = dict(scaling_iters=10, rho_interval=rho_interval)
    g, plan = _run(b, precision, kernel, **kw)
    assert np.all(g["status"] == 0)
    ref = _oracle(b, iters=50, ruiz_iters=10, rho_interval=rho_interval)
    # scale factors
    sc = plan.get_scaling().cpu().numpy()
    for a, s in enumerate(b.shapes):
        o = ref[a]["scale"]
        assert np.abs(sc[a, :s.nx] / o["Dx"] - 1).max() < 1e-12
        assert np.abs(sc[a, 64:64 + s.nu] / o["Du"] - 1).max() < 1e-12
        assert abs(sc[a, 96] / o["c"] - 1) < 1e-12
    keep = _check_rho(plan, ref, rho_interval)
    e = _errors(b, g, ref)[keep]
    print(f"{precision} {kernel} {kind} rho_interval={rho_interval}: max u0/traj/z/y {e.max(axis=0)}"
          f" ({int((~keep).sum())} agents with a boundary decision)")
    assert e[:, :2].max() < TOL[precision]
    if precision == "fp64":
        assert e.max() < TOL["fp64"]


@pytest.mark.parametrize("precision,kernel", [("fp64", "generic"), ("fp32", "fused")])
def test_scaled_warm_start(precision, kernel):
    """A warm start moves into the scaled variables and out again: the second
    solve of a closed loop (x0 advanced) from the first one's iterate."""
    b = _batch("humanoid", precision)
    kw = dict(scaling_iters=10, rho_interval=10)
    plan = mpc.Plan(b.shapes, precision=precision, iters=50, kernel=kernel, **kw)
    prob = mpc.to_device(b, precision)
    plan.solve(prob)
    g0 = {k: v.cpu().numpy() for k, v in plan.get_solution().items()}
    x0n = b.x0 + 0.01 * np.random.default_rng(0).standard_normal(b.x0.shape)
    x0n = x0n.astype(b.x0.dtype)
    prob["x0"] = torch.from_numpy(x0n).cuda()
    plan.solve(prob, warm_start=True)
    g = {k: v.cpu().numpy() for k, v in plan.get_solution().items()}
    assert np.all(g["status"] == 0) and np.all(np.isfinite(g["u"]))
    off = b.offsets()
    warm = [(g0["u"][off["u"][a]:off["u"][a + 1]], g0["z"][off["z"][a]:off["z"][a + 1]],
             g0["y"][off["z"][a]:off["z"][a + 1]]) for a in range(b.n_agents)]
    ref = _oracle(b, warm=[tuple(np.asarray(v, dtype=np.float64) for v in w) for w in warm], x0=x0n,
                  iters=50, ruiz_iters=10, rho_interval=10)
    keep = _check_rho(plan, ref, 10)
    e = _errors(b, g, ref)[keep]
    print(f"{precision} {kernel} warm scaled: max u0/traj/z/y {e.max(axis=0)}"
          f" ({int((~keep).sum())} agents with a boundary decision)")
    assert e[:, :2].max() < TOL[precision]


def test_scaling_rejects_an_input_reference_and_bad_settings():
    b = _batch("humanoid", "fp32")
    plan = mpc.Plan(b.shapes, precision="fp32", iters=50, scaling_iters=10)
    prob = mpc.to_device(b, "fp32")
    prob["u_ref"] = torch.zeros(sum(s.N * s.nu for s in b.shapes), device="cuda")
    with pytest.raises(mpc.MPCError) as ei:
        plan.solve(prob)
    assert ei.value.code == mpc.MPC_ERR_INVALID_ARG
    for bad in (dict(scaling_iters=-1), dict(scaling_iters=101), dict(rho_interval=-2),
                dict(rho_interval=5, rho_tolerance=0.5)):
        with pytest.raises(mpc.MPCError):
            mpc.Plan(b.shapes, precision="fp32", **bad)
    plain = mpc.Plan(b.shapes, precision="fp32")
    plain.solve(mpc.to_device(b, "fp32"))
    with pytest.raises(mpc.MPCError):
        plain.get_rho()
    with pytest.raises(mpc.MPCError):
        plain.get_scaling()
