"""GPU: the persistent iteration launch (plan kernel = 3, "persistent").

Each shape class runs its iterations in one persistent launch over every
horizon: as many workgroups as the device holds at once take agents longest
first from a work-queue counter, an agent of horizon N <= 11 on the
register-resident body and a longer one on the streaming body of the same
kernel.  The per-agent arithmetic is that of the per-bucket launches, so the
iterates are compared bit for bit with a plan of launch groups (kernel =
"fused"), cold, over warm control steps and through a captured step replayed
with eager work between replays; the FP32 tolerance against the FP64 oracle
holds as for every other configuration.
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


def _pair(b):
    pb = mpc.Plan(b.shapes, precision="fp32", iters=50, kernel="fused")
    pp = mpc.Plan(b.shapes, precision="fp32", iters=50, kernel="persistent")
    return pb, pp, mpc.to_device(b, "fp32"), mpc.to_device(b, "fp32")


def _same(sa, sb, tag):
    for k in KEYS:
        assert torch.equal(sa[k], sb[k]), (tag, k)


def test_one_launch_per_shape_class():
    b = synth.uneven_batch(256)
    _, pp, _, prob = _pair(b)
    groups = pp.groups()
    assert len(groups) == 2  # humanoid and quadruped, every horizon in one group each
    assert sum(g["n_agents"] for g in groups) == 256
    for g in groups:
        assert g["family"] == "fused"
        # enough wavefronts for the longest register-resident agent (12) and the
        # streaming body's stage + chain + loader wavefronts at N = 20 (12)
        assert g["threads"] == 64 * 12 and g["N"] == max(s.N for s in b.shapes if s.nx == g["nx"])


@pytest.mark.parametrize("which", ["uneven", "uniform"])
def test_matches_launch_groups_bit_for_bit(which):
    b = synth.uneven_batch(200) if which == "uneven" else synth.humanoid_batch(128)
    pb, pp, prob_b, prob_p = _pair(b)
    nx_tot = sum(s.nx for s in b.shapes)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    noise = torch.empty(nx_tot, dtype=torch.float32, device="cuda")
    for step in range(4):
        noise.normal_(0.0, 1e-2, generator=gen)
        pb.solve(prob_b, warm_start=step > 0)
        pp.solve(prob_p, warm_start=step > 0)
        torch.cuda.synchronize()
        _same(pb.get_solution(), pp.get_solution(), step)
        pb.advance_state(prob_b, noise, prob_b["x0"])
        pp.advance_state(prob_p, noise, prob_p["x0"])
    assert torch.equal(prob_b["x0"], prob_p["x0"])


def test_cold_solve_matches_oracle():
    b = synth.uneven_batch(128)
    pp = mpc.Plan(b.shapes, precision="fp32", iters=50, kernel="persistent")
    pp.solve(mpc.to_device(b, "fp32"))
    g = {k: v.cpu().numpy() for k, v in pp.get_solution().items()}
    assert np.all(g["status"] == 0)
    e = agent_errors(b, g, oracle.solve_batch(b, iters=50))
    print("persistent fp32 max u0/traj", e[:, :2].max(axis=0))
    assert e[:, :2].max() < TOL["fp32"]


def test_captured_step_replays_with_the_counter_reset():
    """The work-queue counter is zeroed by a kernel inside the captured step,
    so every replay drains the whole list again."""
    b = synth.uneven_batch(96)
    nx_tot = sum(s.nx for s in b.shapes)
    pe = mpc.Plan(b.shapes, precision="fp32", iters=50, kernel="persistent")
    pg = mpc.Plan(b.shapes, precision="fp32", iters=50, kernel="persistent")
    prob_e, prob_g = mpc.to_device(b, "fp32"), mpc.to_device(b, "fp32")
    noise_e = torch.empty(nx_tot, dtype=torch.float32, device="cuda")
    noise_g = torch.empty_like(noise_e)
    pe.solve(prob_e)
    pg.solve(prob_g)
    pg.capture(prob_g, warm_start=True, noise=noise_g, x0_next=prob_g["x0"])
    torch.cuda.synchronize()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(11)
    scratch = torch.zeros(1 << 16, device="cuda")
    for step in range(4):
        noise_e.normal_(0.0, 1e-2, generator=gen)
        noise_g.copy_(noise_e)
        pe.solve(prob_e, warm_start=True)
        pe.advance_state(prob_e, noise_e, prob_e["x0"])
        pg.replay()
        scratch.add_(1.0)
        torch.cuda.synchronize()
        _same(pe.get_solution(), pg.get_solution(), step)
        assert torch.equal(prob_e["x0"], prob_g["x0"]), step
