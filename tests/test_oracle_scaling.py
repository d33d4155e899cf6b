"""Pins of the oracle's Ruiz equilibration and adaptive rho (oracle/scaling.py)
against things other than that module (CPU only): the dense stacked QP built
independently in dense_ref, the definition of the scaled KKT matrix, the
unscaled problem's optimum, the equilibration's own fixed point, and residuals
recomputed from the stacked QP."""
import numpy as np
import pytest

import dense_ref as D
import oracle
from oracle import scaling
from paper_2510_12717_amd import synth


def tiny(N=3, nx=4):
    return synth.Shape(N=N, nx=nx, nu=7, n_tau=1, n_feet=2, foot_dim=3)


def agent(shape, seed=0, kappa=None):
    if kappa is None:
        b = synth.make_batch([shape], seed=seed, stream_id=77)
    else:
        h = 0.5 * np.log10(kappa)
        b = synth.make_batch([shape], seed=seed, stream_id=78, q_log=(-h, h), r_log=(-h, h),
                             r_scale=10 ** -2.5)
    return oracle.agent(b, 0)


def heavy(shape, seed=0):
    """An agent whose cost weights (100 .. 5000) dominate every KKT column."""
    ag = agent(shape, seed)
    rng = np.random.default_rng(seed + 1000)
    ag["q"] = 10 ** rng.uniform(2, 3.7, shape.nx)
    ag["r"] = 10 ** rng.uniform(2, 3.7, shape.nu)
    return ag


def rel(a, b):
    a, b = np.asarray(a, dtype=float), np.asarray(b, dtype=float)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


ARGS = ("s", "A", "B", "c", "q", "r", "x_ref", "x0", "tau_max", "mu", "stance")


def test_stacked_qp_matches_dense_reference():
    s = tiny()
    ag = agent(s, 1)
    P, q, Aeq, Cs = scaling.stacked(ag)
    G, _ = D.dynamics_rows(s, ag["A"], ag["B"], ag["c"], ag["x0"])
    assert np.array_equal(Aeq, G)
    C = D.C_dense(s, ag["mu"])
    m = C.shape[0]
    for k in range(s.N):
        blk = Cs[k * m:(k + 1) * m, s.N * s.nx + k * s.nu:s.N * s.nx + (k + 1) * s.nu]
        assert np.array_equal(blk, C)
    assert np.count_nonzero(Cs) == s.N * np.count_nonzero(C)
    assert np.array_equal(P, np.concatenate([np.tile(ag["q"], s.N), np.tile(ag["r"], s.N)]))
    assert np.array_equal(q[:s.N * s.nx], -(ag["q"] * ag["x_ref"][1:]).ravel())


@pytest.mark.parametrize("shape,cost_heavy", [(tiny(), False), (synth.humanoid(3), False),
                                              (synth.quadruped(2), False), (tiny(), True),
                                              (synth.quadruped(2), True)])
def test_scaled_problem_is_the_scaled_kkt(shape, cost_heavy):
    """The scaled agent's stacked QP equals the definition: P -> c D P D,
    q -> c D q, constraint rows -> E C D (E fixed by the input scales), dynamics
    rows -> (E D)^-1-normalised D-scaled rows, x0 -> D^-1 x0."""
    ag = heavy(shape, 2) if cost_heavy else agent(shape, 2, kappa=1e4)
    sc = scaling.ruiz(ag, 10)
    h = scaling.scale_agent(ag, sc)
    P, q, Aeq, Cs = scaling.stacked(ag)
    Ph, qh, Aeqh, Csh = scaling.stacked(h)
    N, nx = shape.N, shape.nx
    d = np.concatenate([np.tile(sc["Dx"], N), np.tile(sc["Du"], N)])
    e = np.tile(scaling.row_scales(shape, sc["Du"]), N)
    assert rel(Ph, sc["c"] * d * d * P) < 1e-14
    assert rel(qh, sc["c"] * d * q) < 1e-14
    assert rel(Csh, e[:, None] * Cs * d[None, :]) < 1e-14
    # a dynamics row scaled by D on its columns, divided by its x_{k+1} coefficient
    dyn = Aeq * d[None, :] / np.tile(sc["Dx"], N)[:, None]
    assert rel(Aeqh, dyn) < 1e-14
    assert rel(h["x0"], ag["x0"] / sc["Dx"]) < 1e-15
    assert rel(h["c"].ravel(), (ag["c"] / sc["Dx"]).ravel()) < 1e-15


def test_scaling_keeps_the_optimum():
    """The scaled problem's converged solution, unscaled, is the original
    problem's optimum (brute-force active set on a tiny instance, the oracle's
    converge mode on a humanoid agent)."""
    s = synth.Shape(N=2, nx=3, nu=4, n_tau=1, n_feet=1, foot_dim=3)
    ag = agent(s, 5, kappa=1e4)
    ref = D.brute_force_qp(*[ag[k] for k in ARGS])
    o = scaling.solve(ag, iters=0, ruiz_iters=10, tol=1e-12)
    assert rel(o["u"], ref[1]) < 1e-7
    h = agent(synth.humanoid(4), 6, kappa=1e6)
    # (a rho matched to the scaled cost keeps converge mode short)
    o = scaling.solve(h, iters=0, ruiz_iters=10, tol=1e-11, settings=oracle.Settings.default(rho=2e-3))
    p = oracle.solve(*[h[k] for k in ARGS], iters=0, tol=1e-11)
    assert rel(o["u"], p["u"]) < 1e-6 and rel(o["x"], p["x"]) < 1e-6
    assert o["res"][:3].max() < 1e-7


def test_first_step_on_a_cost_dominated_problem():
    """When every KKT column's largest entry is its cost weight p_j (weights
    100 .. 5000 against dynamics and constraint entries of at most 1), the first
    equilibration step scales each variable by 1/sqrt(p_j) of its group (the
    largest weight over the stages and tied components), every scaled cost
    weight of a group's largest member is 1, and the cost factor is
    1/max(mean scaled weight, |scaled q|_inf)."""
    s = tiny()
    ag = heavy(s, 3)
    assert np.abs(ag["A"]).max() < 5 and np.abs(ag["B"]).max() < 1
    sc = scaling.ruiz(ag, 1)
    grp = scaling.input_groups(s)
    pu = np.array([ag["r"][grp == grp[j]].max() for j in range(s.nu)])
    assert np.allclose(sc["Dx"], 1 / np.sqrt(ag["q"]), rtol=1e-14)
    assert np.allclose(sc["Du"], 1 / np.sqrt(pu), rtol=1e-14)
    wx = ag["q"] * sc["Dx"] ** 2
    wu = ag["r"] * sc["Du"] ** 2
    mean_w = (s.N * wx.sum() + s.N * wu.sum()) / (s.N * (s.nx + s.nu))
    qn = np.abs(sc["Dx"] * ag["q"] * ag["x_ref"][1:]).max()
    assert sc["c"] == pytest.approx(1 / max(mean_w, qn), rel=1e-13)


def test_equilibration_reaches_its_fixed_point():
    """At convergence the equilibrated KKT matrix S M S (S = the primal scales,
    the dynamics-row scales and the constraint-row scales fixed by the input
    scales) has every tied column group and every dynamics-row group at
    infinity norm 1, and the cost normalisation at max(mean |P|, |q|) = 1;
    before scaling the column norms spread over orders of magnitude."""
    s = synth.humanoid(3)
    ag = agent(s, 8, kappa=1e6)
    sc = scaling.ruiz(ag, 60)
    P, q, Aeq, Cs = scaling.stacked(ag)
    N, nx, nu = s.N, s.nx, s.nu
    d = np.concatenate([np.tile(sc["Dx"], N), np.tile(sc["Du"], N)])
    ed = np.tile(sc["Ed"], N)
    ec = np.tile(scaling.row_scales(s, sc["Du"]), N)
    Ph = sc["c"] * d * d * P
    Ah = np.abs(Aeq) * ed[:, None] * d[None, :]
    Ch = np.abs(Cs) * ec[:, None] * d[None, :]
    col = np.maximum(np.abs(Ph), np.maximum(Ah.max(0), Ch.max(0)))
    grp = scaling.input_groups(s)
    gx = col[:N * nx].reshape(N, nx).max(0)
    gu = col[N * nx:].reshape(N, nu).max(0)
    gu = np.array([gu[grp == grp[j]].max() for j in range(nu)])
    assert np.abs(gx - 1).max() < 1e-9 and np.abs(gu - 1).max() < 1e-9
    assert np.abs(Ah.max(1).reshape(N, nx).max(0) - 1).max() < 1e-9
    assert abs(max(np.abs(Ph).mean(), np.abs(sc["c"] * d * q).max()) - 1) < 1e-9
    col0 = np.maximum(np.abs(P), np.maximum(np.abs(Aeq).max(0), np.abs(Cs).max(0)))
    assert col0.max() / col0.min() > 10


def test_rho_estimate_from_the_stacked_residuals():
    """The estimate equals OSQP's rule evaluated on residuals recomputed from the
    stacked QP (primal |Cu - z|, dual = u-gradient of the Lagrangian with the
    dynamics multipliers that zero the x-gradient), on the 2^(1/4) grid."""
    s = synth.quadruped(3)
    ag = agent(s, 9)
    o = scaling.solve(ag, iters=7, ruiz_iters=10)
    h = scaling.scale_agent(ag, o["scale"])
    u, z, y = (np.asarray(v) for v in scaling.scale_state(s, o["scale"], o["u"], o["z"], o["y"]))
    x = np.asarray(o["x"]) / o["scale"]["Dx"]
    C = D.C_dense(s, h["mu"])
    G, _ = D.dynamics_rows(s, h["A"], h["B"], h["c"], h["x0"])
    nxv = s.N * s.nx
    grad = np.concatenate([(h["q"] * (x[1:] - h["x_ref"][1:])).ravel(), (h["r"] * u).ravel()])
    lam = np.linalg.solve(G[:, :nxv].T, -grad[:nxv])
    dual = np.abs(grad[nxv:] + G[:, nxv:].T @ lam + (y @ C).ravel()).max()
    prim = np.abs(u @ C.T - z).max()
    pn = max(np.abs(u @ C.T).max(), np.abs(z).max())
    dn = max(np.abs(h["q"] * x[1:]).max(), np.abs(h["r"] * u).max(), np.abs(y @ C).max(),
             np.abs(h["q"] * h["x_ref"][1:]).max())
    raw = 0.3 * np.sqrt((prim / pn) / (dual / dn))
    want = 2.0 ** (np.round(4 * np.log2(raw)) / 4)
    got = scaling.rho_estimate(h, x, u, z, y, 0.3)
    assert got == pytest.approx(want, rel=1e-12)


def test_rho_update_rule():
    """Segments with rho fixed (tolerance never met) equal one uninterrupted
    solve; a rho far from its estimate is replaced after the first segment and
    left alone once within the tolerance; no scaling and fixed rho is the plain
    oracle."""
    ag = agent(synth.humanoid(4), 10, kappa=1e4)
    one = scaling.solve(ag, iters=40, ruiz_iters=10)
    seg = scaling.solve(ag, iters=40, ruiz_iters=10, rho_interval=10, rho_tolerance=1e300)
    assert rel(seg["u"], one["u"]) < 1e-12 and seg["rhos"] == [0.1] * 4
    far = scaling.solve(ag, iters=40, ruiz_iters=10, rho_interval=10,
                        settings=oracle.Settings.default(rho=1e3))
    assert far["rhos"][0] == 1e3 and far["rhos"][1] < 1e3 / 5
    for a, b in zip(far["rhos"][1:], far["rhos"][2:]):
        assert a == b or b > 5 * a or b < a / 5
    plain = scaling.solve(ag, iters=40, ruiz_iters=0)
    p = oracle.solve(*[ag[k] for k in ARGS], iters=40)
    assert np.array_equal(plain["u"], p["u"]) and np.array_equal(plain["y"], p["y"])


def test_warm_start_round_trip():
    """scale_state and unscale_state are inverse changes of variables, and a
    warm-started scaled solve continues a cold one."""
    s = tiny()
    ag = agent(s, 11, kappa=1e4)
    o = scaling.solve(ag, iters=20, ruiz_iters=10)
    sc = o["scale"]
    u, z, y = scaling.scale_state(s, sc, o["u"], o["z"], o["y"])
    _, u2, z2, y2 = scaling.unscale_state(s, sc, o["x"], u, z, y)
    assert rel(u2, o["u"]) < 1e-15 and rel(z2, o["z"]) < 1e-15 and rel(y2, o["y"]) < 1e-15
    whole = scaling.solve(ag, iters=35, ruiz_iters=10)
    cont = scaling.solve(ag, iters=15, ruiz_iters=10, warm=(o["u"], o["z"], o["y"]))
    assert rel(cont["u"], whole["u"]) < 1e-10


def test_decide_and_grid():
    """The update keeps rho within the tolerance band and otherwise takes the
    clipped estimate on the 2^(1/4) grid."""
    assert scaling.decide(0.1, 0.3) == 0.1
    assert scaling.decide(0.1, 0.01) == pytest.approx(2.0 ** -6.75, rel=1e-15)
    assert scaling.decide(0.1, 1e-9) == 1e-6 * 0 + 2.0 ** (np.round(4 * np.log2(1e-6)) / 4)
    assert scaling.grid(2.0 ** -3.1) == 2.0 ** -3.0
