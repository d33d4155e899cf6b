"""Pins of the oracle's joint-limit rows (x_lo <= x_k <= x_hi, the joint limits
of Eq. (mpc_formulation)) against things other than the oracle (CPU only):
dense KKT solves of the x-subproblem with the state rows, dense ADMM on the
stacked QP with the state rows, brute-force active-set enumeration over input
and state rows, and the Lagrangian gradient with the state multipliers."""
import numpy as np
import pytest

import dense_ref as D
import oracle
from paper_2510_12717_amd import synth

ARGS = ("s", "A", "B", "c", "q", "r", "x_ref", "x0", "tau_max", "mu", "stance")


def agent(shape, seed):
    b = synth.make_batch([shape], seed=seed, stream_id=88)
    return oracle.agent(b, 0)


def limits(nx, seed, frac=0.7, width=(0.3, 1.5), eq=False):
    """A seeded box with some components unbounded, some one-sided, some two-sided."""
    rng = np.random.default_rng(seed)
    lo = -rng.uniform(*width, nx)
    hi = rng.uniform(*width, nx)
    free = rng.random(nx) > frac
    lo[free], hi[free] = -np.inf, np.inf
    one = rng.random(nx) < 0.2
    hi[one & ~free] = np.inf
    if eq:
        lo[0] = hi[0] = 0.25
    return lo, hi


def rel(a, b):
    a, b = np.asarray(a, dtype=float), np.asarray(b, dtype=float)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("shape,seed", [(synth.Shape(N=3, nx=4, nu=4, n_tau=1, n_feet=1, foot_dim=3), 1),
                                        (synth.quadruped(3), 2), (synth.humanoid(2), 3)])
def test_xupdate_with_state_rows_equals_dense_kkt(shape, seed):
    """Factor with the state penalties in Q~ plus one back-sweep/rollout with the
    state rows' linear terms equals a dense KKT solve of the x-subproblem with
    the state rows."""
    ag = agent(shape, seed)
    s = shape
    lo, hi = limits(s.nx, seed, eq=True)
    rx = oracle.state_penalties(s, lo, hi)
    assert np.array_equal(rx, D.state_rho(lo, hi))
    rng = np.random.default_rng(seed)
    C = D.C_dense(s, ag["mu"])
    l, h = D.bounds_table(s, ag["tau_max"], ag["stance"])
    rr = D.rho_table(l, h)
    m = C.shape[0]
    xj = rng.standard_normal((s.N + 1, s.nx))
    uj = rng.standard_normal((s.N, s.nu))
    z, y = rng.standard_normal((s.N, m)), rng.standard_normal((s.N, m))
    zx, yx = rng.standard_normal((s.N, s.nx)), rng.standard_normal((s.N, s.nx))
    _, rho_rows = oracle.stage_bounds(s, ag["tau_max"], ag["stance"])[1:], oracle.stage_bounds(s, ag["tau_max"], ag["stance"])[2]
    st, K, L, sv, _ = oracle.factor(s, ag["A"], ag["B"], ag["c"], ag["q"], ag["r"], rho_rows, ag["mu"], qx=rx)
    assert st == 0
    sigma = 1e-6
    qt = -ag["q"] * ag["x_ref"] - sigma * xj
    qt[1:] += yx - rx * zx
    rt = -sigma * uj + (y - rr * z) @ C
    xt, ut = oracle.xupdate(s, ag["A"], ag["B"], ag["c"], K, L, sv, ag["x0"], qt, rt)
    H, g = D.x_subproblem(s, ag["q"], ag["r"], ag["x_ref"], C, rr, sigma, xj, uj, z, y)
    for k in range(1, s.N + 1):
        sl = slice((k - 1) * s.nx, k * s.nx)
        H[sl, sl] += np.diag(rx)
        g[sl] += rx * (-zx[k - 1] + yx[k - 1] / rx)
    G, b = D.dynamics_rows(s, ag["A"], ag["B"], ag["c"], ag["x0"])
    v, _ = D.kkt_solve(H, g, G, b)
    xd, ud = D.split(s, v, ag["x0"])
    assert rel(ut, ud) < 1e-9 and rel(xt, xd) < 1e-9


@pytest.mark.parametrize("shape,seed,iters", [(synth.Shape(N=3, nx=4, nu=4, n_tau=1, n_feet=1, foot_dim=3), 4, 9),
                                              (synth.quadruped(3), 5, 6), (synth.humanoid(2), 6, 5)])
def test_fixed_iterates_with_limits_equal_dense_admm(shape, seed, iters):
    ag = agent(shape, seed)
    lo, hi = limits(shape.nx, seed, eq=True)
    o = oracle.solve(*[ag[k] for k in ARGS], iters=iters, x_lo=lo, x_hi=hi)
    x, u, z, y, zx, yx = D.dense_admm_limits(*[ag[k] for k in ARGS], lo, hi, iters)
    assert o["status"] == 0
    for got, want in ((o["x"], x), (o["u"], u), (o["z"], z), (o["y"], y), (o["zx"], zx), (o["yx"], yx)):
        assert rel(got, want) < 1e-9
    # every iterate's z_x lies in the box
    assert np.all(o["zx"] >= lo - 1e-15) and np.all(o["zx"] <= hi + 1e-15)


def test_converged_with_limits_equals_brute_force():
    """Converge mode reaches the exact optimum of the QP with joint limits,
    where some limits are active."""
    s = synth.Shape(N=2, nx=2, nu=2, n_tau=2, n_feet=0, foot_dim=3)
    found = 0
    for seed in range(12):
        ag = agent(s, 100 + seed)
        # inputs strong enough to hold the state inside its limits, references
        # outside them, torque boxes that bind now and then
        ag["B"] = ag["B"] * 100.0
        ag["x_ref"] = ag["x_ref"] * 3.0
        ag["tau_max"] = ag["tau_max"] * 0.05
        lo, hi = limits(s.nx, seed, frac=1.0, width=(0.5, 1.0))
        ref = D.brute_force_qp_limits(*[ag[k] for k in ARGS], lo, hi)
        if ref is None:
            continue
        x, u, y, yx = ref
        o = oracle.solve(*[ag[k] for k in ARGS], iters=0, tol=1e-11, max_iters=400000, x_lo=lo,
                         x_hi=hi)
        assert o["status"] == 1
        assert rel(o["u"], u) < 1e-7 and rel(o["x"], x) < 1e-7
        assert np.abs(o["yx"] - yx).max() < 1e-6 * max(1.0, np.abs(yx).max())
        found += np.count_nonzero(np.abs(yx) > 1e-6)
        assert o["res"].max() < 1e-9
    assert found >= 3  # some limits were active


def test_residuals_with_state_multipliers():
    """The residual report with joint limits equals the stacked QP's: primal
    includes |x_k - z_x,k|, the dual residual is the u-gradient of the
    Lagrangian f + mu'(Gv - b) + y'Cu + y_x'x with mu zeroing the x-gradient."""
    s = synth.quadruped(3)
    ag = agent(s, 7)
    rng = np.random.default_rng(7)
    lo, hi = limits(s.nx, 7)
    C = D.C_dense(s, ag["mu"])
    x = rng.standard_normal((s.N + 1, s.nx))
    x[0] = ag["x0"]
    u = rng.standard_normal((s.N, s.nu))
    z, y = rng.standard_normal((s.N, C.shape[0])), rng.standard_normal((s.N, C.shape[0]))
    # z_x far from x, so that the state rows decide the primal residual
    zx, yx = 10 * rng.standard_normal((s.N, s.nx)), rng.standard_normal((s.N, s.nx))
    res, _ = oracle.residuals(*[ag[k] for k in ARGS], x, u, z, y, x_lo=lo, x_hi=hi, zx=zx, yx=yx)
    G, b = D.dynamics_rows(s, ag["A"], ag["B"], ag["c"], ag["x0"])
    nxv = s.N * s.nx
    grad = np.concatenate([(ag["q"] * (x[1:] - ag["x_ref"][1:]) + yx).ravel(), (ag["r"] * u).ravel()])
    mu_ = np.linalg.solve(G[:, :nxv].T, -grad[:nxv])
    dual = grad[nxv:] + G[:, nxv:].T @ mu_ + (y @ C).ravel()
    prim = max(np.abs(u @ C.T - z).max(), np.abs(x[1:] - zx).max())
    assert np.abs(x[1:] - zx).max() > np.abs(u @ C.T - z).max()
    assert res[0] == pytest.approx(prim, rel=1e-12)
    assert res[1] == pytest.approx(np.abs(dual).max(), rel=1e-9)
    l, h = D.bounds_table(s, ag["tau_max"], ag["stance"])
    comp = max(D.complementarity_natural(l, h, z, y),
               D.complementarity_natural(np.tile(lo, (s.N, 1)), np.tile(hi, (s.N, 1)), zx, yx))
    assert res[3] == pytest.approx(comp, rel=1e-12)


def test_batch_with_limits_equals_single_solves():
    b = synth.uneven_batch(5)
    off = b.offsets()
    rng = np.random.default_rng(9)
    lo = np.concatenate([limits(s.nx, 10 + a)[0] for a, s in enumerate(b.shapes)])
    hi = np.concatenate([limits(s.nx, 10 + a)[1] for a, s in enumerate(b.shapes)])
    o = oracle.solve_batch(b, iters=20, x_lo=lo, x_hi=hi)
    for a, s in enumerate(b.shapes):
        ag = oracle.agent(b, a)
        one = oracle.solve(*[ag[k] for k in ARGS], iters=20, x_lo=lo[off["q"][a]:off["q"][a + 1]],
                           x_hi=hi[off["q"][a]:off["q"][a + 1]])
        assert np.array_equal(o["u"][off["u"][a]:off["u"][a + 1]], one["u"].ravel())
        assert np.array_equal(o["zx"][off["c"][a]:off["c"][a + 1]], one["zx"].ravel())
    del rng
