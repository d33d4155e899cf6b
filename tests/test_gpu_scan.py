"""GPU: the parallel-in-time Riccati factor (plan riccati_scan = 1).

The scan composes the stages' maps P -> J + A'P(I + CP)^{-1}A in
ceil(log2(N + 1)) doubling rounds and forms every stage's operators from its
P_{k+1}; it must give the serial recursion's operators up to rounding.  Checked
against the oracle's factor (K_k, s_k and H_k^{-1} = (L_k L_k')^{-1}) at FP64,
horizons 1 to 40 (one round to six; the generic iteration kernel's LDS holds
a humanoid agent up to N = 42); the solves of scan plans against the
oracle's iterate (FP64 1e-10, FP32 1e-5), mixed shapes in one plan, and a
non-finite agent that stays local.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2510_12717_amd import mpc, synth

from test_gpu_parity import TOL, agent_errors

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    mpc.lib()


def rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("N", [1, 2, 7, 31, 40])
def test_scan_factor_matches_oracle_factor(N):
    shapes = [synth.humanoid(N), synth.quadruped(N), synth.humanoid(max(1, N // 2))]
    b = synth.make_batch(shapes, seed=3, stream_id=1)
    plan = mpc.Plan(b.shapes, precision="fp64", iters=1, riccati_scan=1)
    assert all(g["family"] == "generic" for g in plan.groups())
    plan.solve(mpc.to_device(b, "fp64"))
    sol = plan.get_solution()
    assert np.all(sol["status"].cpu().numpy() == 0)
    for a in range(len(shapes)):
        s = b.shapes[a]
        ag = oracle.agent(b, a)
        _, _, rho = oracle.stage_bounds(s, ag["tau_max"], ag["stance"])
        st, Ko, Lo, svo, _ = oracle.factor(s, ag["A"], ag["B"], ag["c"], ag["q"], ag["r"], rho, ag["mu"])
        assert st == oracle.OK
        K, Acl, Hi, sv = (t.cpu().numpy() for t in plan.export_factor(a))
        Hio = np.stack([np.linalg.inv(Lo[k] @ Lo[k].T) for k in range(s.N)])
        Aclo = ag["A"] + np.einsum("kij,kjl->kil", ag["B"], Ko)
        e = (rel(K, Ko), rel(Acl, Aclo), rel(Hi, Hio), rel(sv, svo))
        print("N", s.N, "nx", s.nx, "K/Acl/Hinv/s rel err", e)
        assert max(e) < 1e-10


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_scan_solves_match_oracle(precision):
    shapes = [synth.humanoid(40), synth.quadruped(25), synth.humanoid(9), synth.quadruped(33)]
    b = synth.make_batch(shapes, seed=5, stream_id=2)
    dt = np.float64 if precision == "fp64" else np.float32
    b = b.astype(dt)
    plan = mpc.Plan(b.shapes, precision=precision, iters=50, riccati_scan=1)
    plan.solve(mpc.to_device(b, precision))
    g = {k: v.cpu().numpy() for k, v in plan.get_solution().items()}
    assert np.all(g["status"] == 0)
    e = agent_errors(b, g, oracle.solve_batch(b, iters=50))
    print(precision, "scan max u0/traj/z/y", e.max(axis=0))
    assert e[:, :2].max() < TOL[precision]


def test_scan_equals_serial_generic_factor_closely():
    """Same solve with the serial generic factor: the two factors differ only
    in rounding order."""
    shapes = [synth.humanoid(40)] * 3
    b = synth.make_batch(shapes, seed=9, stream_id=1)
    prob = mpc.to_device(b, "fp64")
    ps = mpc.Plan(b.shapes, precision="fp64", iters=50, riccati_scan=1)
    pg = mpc.Plan(b.shapes, precision="fp64", iters=50, kernel="generic")
    ps.solve(prob)
    pg.solve(prob)
    ss, sg = ps.get_solution(), pg.get_solution()
    for k in ("u", "x", "z", "y"):
        a_, b_ = ss[k].cpu().numpy(), sg[k].cpu().numpy()
        assert rel(a_, b_) < 1e-10, k


def test_scan_nonfinite_agent_stays_local():
    shapes = [synth.humanoid(20)] * 4
    b = synth.make_batch(shapes, seed=2, stream_id=1)
    off = b.offsets()
    b.A[off["A"][2] + 5] = np.nan
    plan = mpc.Plan(b.shapes, precision="fp64", iters=50, riccati_scan=1)
    plan.solve(mpc.to_device(b, "fp64"))
    g = {k: v.cpu().numpy() for k, v in plan.get_solution().items()}
    assert g["status"].tolist() == [0, 0, mpc.AGENT_NONFINITE, 0]
    ok = [0, 1, 3]
    sub = b.subset(ok)
    o = oracle.solve_batch(sub, iters=50)
    o["_off"] = sub.offsets()
    e = agent_errors(b, g, o, agents=ok, go=[0, 1, 2])
    assert e[:, :2].max() < TOL["fp64"]


def test_scan_rejections():
    s = [synth.humanoid(10)]
    with pytest.raises(mpc.MPCError):
        mpc.Plan(s, precision="fp32", riccati_scan=1, inner_solve=1)
    with pytest.raises(mpc.MPCError):
        mpc.Plan(s, precision="bf16", riccati_scan=1)
