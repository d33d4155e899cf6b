"""How the warm-started closed loop treats a small error in one solve (CPU only).

Each control step warm-starts 50 ADMM iterations from the previous step's
iterate (u, z, y), so an error left in one step's iterate is carried into the
next solve and is contracted only slowly by the iteration.  Two implementations
whose single solves agree to a few 1e-6 therefore drift apart over a long loop
by much more than that.  This test shows it with the FP64 oracle alone: one
loop as is, one whose warm state is perturbed after every step by a seeded
relative 3e-6 (about the FP32 GPU solve's error), every 64th agent of the
4096-agent humanoid batch, 100 steps, the same x0 sequence.  The separation of
u_0 exceeds the single-solve FP32 tolerance by far and stays below the
accumulation bound of 100 steps times that tolerance, the bound the GPU's
independent loop is gated at.
"""
import numpy as np

import oracle
from paper_2510_12717_amd import synth


def test_warm_loop_carries_perturbations():
    n, every, steps, iters, eps = 4096, 64, 100, 50, 3e-6
    ids = np.arange(0, n, every)
    sub = synth.humanoid_batch(agent_ids=ids)
    sh = sub.shapes[0]
    nx, nu, N, m = sh.nx, sh.nu, sh.N, sh.nu + 4 * sh.n_feet
    k = len(ids)
    rng = np.random.default_rng(1)
    x0 = sub.x0.copy()
    sa = sb = None
    e_u0, e_tr = [], []
    for step in range(steps):
        a = oracle.solve_batch(sub, iters=iters, warm=sa, x0=x0)
        b = oracle.solve_batch(sub, iters=iters, warm=sb, x0=x0)
        ua, ub = a["u"].reshape(k, -1), b["u"].reshape(k, -1)
        ta = np.concatenate([a["x"].reshape(k, -1)[:, nx:], ua], 1)
        tb = np.concatenate([b["x"].reshape(k, -1)[:, nx:], ub], 1)
        e_u0.append((np.abs(ua[:, :nu] - ub[:, :nu]).max(1) / np.abs(ua[:, :nu]).max(1)).max())
        e_tr.append((np.abs(ta - tb).max(1) / np.abs(ta).max(1)).max())
        sa = {key: a[key] for key in ("u", "z", "y")}
        sb = {}
        for key, w in (("u", N * nu), ("z", N * m), ("y", N * m)):
            v = b[key].reshape(k, w).copy()
            v += eps * np.abs(v).max(1, keepdims=True) * rng.standard_normal(v.shape)
            sb[key] = v.ravel()
        x0 = oracle.advance_batch(sub, x0, a["u"], synth.step_noise(sub, step))
    e_u0, e_tr = np.array(e_u0), np.array(e_tr)
    print(f"u0 separation: step 1 {e_u0[1]:.2e}, step 10 {e_u0[10]:.2e}, worst {e_u0.max():.2e}; "
          f"trajectory worst {e_tr.max():.2e}")
    assert e_u0[0] == 0.0 and e_tr[0] == 0.0   # the first solve is cold on both sides
    assert e_u0.max() > 10 * 1e-5             # far beyond one solve's tolerance ...
    assert e_u0[50:].max() > 2 * e_u0[1]       # ... because it builds up over steps
    assert max(e_u0.max(), e_tr.max()) < steps * 1e-5  # within the accumulation bound
