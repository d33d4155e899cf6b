"""GPU: launch groups of uneven batches, the autotuner and captured-step replay.

Uneven batches (horizons N ~ U{5..20}, half humanoid nx=48 nu=30, half
quadruped nx=36 nu=24) split into register-resident launch groups per shape
class and horizon bucket (N <= 6, 7..11, 12..20; the last on the streaming
iteration kernel).
Every configuration is checked against the FP64 oracle at the FP32 tolerance
(1e-5, norm-wise relative per agent).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2510_12717_amd import mpc, synth

from test_gpu_parity import TOL, agent_errors, run_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    mpc.lib()


def test_groups_of_uneven_batch():
    b = synth.uneven_batch(256)
    g, plan, _ = run_gpu(b, "fp32")
    groups = plan.groups()
    assert sum(x["n_agents"] for x in groups) == 256
    for x in groups:
        assert x["family"] == "fused"
        assert x["N"] <= 20 and (x["nx"], x["nu"]) in ((48, 30), (36, 24))
        if x["N"] <= 11:
            assert x["threads"] == 64 * (x["N"] + 1)  # stage wavefronts + chain
        else:
            assert x["threads"] == 64 * ((x["N"] + 1) // 2 + 2)  # + loader
    assert len(groups) == 6  # two shape classes x three horizon buckets
    assert plan.config()["kernel"] == "fused"
    # the u0 export of an uneven batch (one gather kernel) is each agent's first input
    ou, o0 = 0, 0
    for s in b.shapes:
        np.testing.assert_array_equal(g["u0"][o0:o0 + s.nu], g["u"][ou:ou + s.nu])
        ou += s.N * s.nu
        o0 += s.nu
    assert o0 == g["u0"].size
    o = oracle.solve_batch(b, iters=50)
    assert np.all(g["status"] == 0)
    e = agent_errors(b, g, o)
    print("uneven fp32: %d groups, max u0/traj %s" % (len(groups), e[:, :2].max(axis=0)))
    assert e[:, :2].max() < TOL["fp32"]


@pytest.mark.parametrize("precision,kernel", [("fp32", "auto"), ("fp64", "auto"),
                                              ("fp32", "generic")])
def test_autotune_keeps_parity(precision, kernel):
    b = synth.uneven_batch(128)
    plan = mpc.Plan(b.shapes, precision=precision, iters=50, kernel=kernel)
    prob = mpc.to_device(b, precision)
    groups = plan.autotune(prob, reps=2)
    for x in groups:
        assert x["family"] in (("generic", "fused") if precision == "fp32" and kernel == "auto"
                               else ("generic",))
        if x["family"] == "generic":
            assert x["threads"] in (64, 128, 256)
    with pytest.raises(mpc.MPCError):
        plan.solve(prob, warm_start=True)  # the resident state is dropped by the tuner
    plan.solve(prob)
    sol = {k: v.cpu().numpy() for k, v in plan.get_solution().items()}
    o = oracle.solve_batch(b, iters=50)
    assert np.all(sol["status"] == 0)
    e = agent_errors(b, sol, o)
    print(precision, kernel, "autotuned groups:",
          [(x["family"], x["N"], x["threads"]) for x in groups], "max", e[:, :2].max())
    assert e[:, :2].max() < TOL[precision]


@pytest.mark.parametrize("which", ["uniform", "uneven"])
def test_graph_replay_matches_eager(which):
    """A captured control step (warm solve + plant step) replayed several times,
    with unrelated eager work and synchronisations between replays, gives
    bit-identical results to the same steps issued eagerly."""
    b = synth.humanoid_batch(64) if which == "uniform" else synth.uneven_batch(96)
    nx_tot = sum(s.nx for s in b.shapes)
    pe = mpc.Plan(b.shapes, precision="fp32", iters=50)
    pg = mpc.Plan(b.shapes, precision="fp32", iters=50)
    prob_e = mpc.to_device(b, "fp32")
    prob_g = mpc.to_device(b, "fp32")
    noise_e = torch.empty(nx_tot, dtype=torch.float32, device="cuda")
    noise_g = torch.empty_like(noise_e)
    pe.solve(prob_e)
    pg.solve(prob_g)
    pg.capture(prob_g, warm_start=True, noise=noise_g, x0_next=prob_g["x0"])
    torch.cuda.synchronize()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(7)
    scratch = torch.zeros(1 << 20, device="cuda")
    for step in range(4):
        noise_e.normal_(0.0, 1e-2, generator=gen)
        noise_g.copy_(noise_e)
        pe.solve(prob_e, warm_start=True)
        pe.advance_state(prob_e, noise_e, prob_e["x0"])
        pg.replay()
        scratch.add_(1.0)  # eager work between replays
        torch.cuda.synchronize()
        se = pe.get_solution()
        sg = pg.get_solution()
        torch.cuda.synchronize()
        for k in ("u", "x", "z", "y", "status"):
            assert torch.equal(se[k], sg[k]), (step, k)
        assert torch.equal(prob_e["x0"], prob_g["x0"]), step
    assert float(scratch[0]) == 4.0


def test_replay_without_capture_is_not_ready():
    b = synth.small_humanoid_batch(4)
    plan = mpc.Plan(b.shapes, precision="fp32")
    with pytest.raises(mpc.MPCError) as ei:
        plan.replay()
    assert ei.value.code == mpc.MPC_ERR_NOT_READY


def test_uneven_8192_sampled():
    """The uneven batch at full size (8192 agents) in the benchmark's launch
    configuration: autotuned groups, one captured step replayed; every 64th
    agent is checked against the oracle (cold start)."""
    b = synth.uneven_batch(8192, dtype=np.float32)
    plan = mpc.Plan(b.shapes, precision="fp32", iters=50)
    prob = mpc.to_device(b, "fp32")
    groups = plan.autotune(prob, reps=1)
    assert all(x["family"] == "fused" for x in groups)
    plan.capture(prob, warm_start=False)
    plan.replay()
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in plan.get_solution().items()}
    assert np.all(g["status"] == 0)
    ids = np.arange(0, 8192, 64)
    sub = synth.uneven_batch(agent_ids=ids)
    o = oracle.solve_batch(sub, iters=50)
    o["_off"] = sub.offsets()
    e = agent_errors(b, g, o, agents=ids, go=np.arange(len(ids)))
    print("uneven_batch sampled: max u0/traj", e[:, :2].max(axis=0), "horizons",
          sorted({b.shapes[i].N for i in ids}))
    assert e[:, :2].max() < TOL["fp32"]
