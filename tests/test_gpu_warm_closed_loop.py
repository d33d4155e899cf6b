"""GPU parity of the configuration the benchmark times: the 4096-agent humanoid
closed loop, 100 control steps, each solve warm-started from the GPU's OWN
previous iterate (u, z, y resident on the device), 50 ADMM iterations.

The oracle runs its own closed loop on every 16th agent (its own warm starts,
x0 advanced by the agent's own first stage plus the seeded plant noise), and
the sampled agents' x0 on the GPU is taken from that loop, so both sides solve
the same QP sequence from their own iterates.  Every other agent advances by
the GPU's plant step, as in the benchmark.  The gate is the FP32 tolerance on
u_0 and on the trajectory (x_1..N, u_0..N-1) of every checked agent at every
step.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2510_12717_amd import mpc, synth

pytestmark = pytest.mark.gpu

TOL_FP32 = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    mpc.lib()


def _rel(p, q):
    return np.abs(p - q).max(axis=1) / np.abs(q).max(axis=1)


@pytest.mark.parametrize("kernel", ["fused", "generic"])
def test_self_warm_started_closed_loop(kernel):
    n, every, steps, iters = 4096, 16, 100, 50
    sh = synth.humanoid(10)
    nx, nu, N = sh.nx, sh.nu, sh.N
    b = synth.humanoid_batch(n, dtype=np.float32)
    ids = np.arange(0, n, every)
    sub = synth.humanoid_batch(agent_ids=ids)
    plan = mpc.Plan(b.shapes, precision="fp32", iters=iters, kernel=kernel)
    assert plan.config()["kernel"] == kernel
    prob = mpc.to_device(b, "fp32")
    ids_t = torch.from_numpy(ids).cuda()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    noise = torch.empty(n * nx, device="cuda")
    x0_sub = sub.x0.copy()
    state = None
    curve = []
    for step in range(steps):
        o = oracle.solve_batch(sub, iters=iters, warm=state, x0=x0_sub)
        assert np.all(o["status"] == 0)
        prob["x0"].view(n, nx)[ids_t] = torch.from_numpy(x0_sub.reshape(-1, nx)).float().cuda()
        plan.solve(prob, warm_start=step > 0)
        sol = plan.get_solution()
        x = sol["x"].view(n, (N + 1) * nx)[ids_t].double().cpu().numpy()
        u = sol["u"].view(n, N * nu)[ids_t].double().cpu().numpy()
        status = sol["status"].cpu().numpy()
        assert np.all(status == 0), f"step {step}: status {np.unique(status)}"
        xo = o["x"].reshape(len(ids), -1)
        uo = o["u"].reshape(len(ids), -1)
        e_u0 = _rel(u[:, :nu], uo[:, :nu])
        e_tr = _rel(np.concatenate([x[:, nx:], u], 1), np.concatenate([xo[:, nx:], uo], 1))
        curve.append((e_u0.max(), e_tr.max(), np.median(e_tr)))
        # next step: oracle loop for the checked agents, the GPU's own plant step for all
        state = {k: o[k] for k in ("u", "z", "y")}
        x0_sub = oracle.advance_batch(sub, x0_sub, o["u"], synth.step_noise(sub, step))
        noise.normal_(0.0, 1e-2, generator=gen)
        plan.advance_state(prob, noise, prob["x0"])
    curve = np.array(curve)
    for s in (0, 1, 2, 5, 10, 20, 50, 99):
        print(f"{kernel} step {s:3d}: max u0 {curve[s, 0]:.2e} max traj {curve[s, 1]:.2e} "
              f"median traj {curve[s, 2]:.2e}")
    print(f"{kernel}: worst over {steps} steps u0 {curve[:, 0].max():.3e} "
          f"traj {curve[:, 1].max():.3e}")
    assert curve[:, :2].max() < TOL_FP32
