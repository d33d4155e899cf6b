"""Pins of the FP64 oracle against mathematics independent of it (CPU only).

Each test ties one part of the oracle to something other than the oracle:
the problem statement, dense KKT solves of the stacked QP, brute-force
active-set enumeration, the condensed least-squares closed form, SciPy's DARE
solver, exact invariants of the iteration, and the paper's own finite-rho
OSQP form of the KKT system (Eq. (kkt_system)).
"""
import numpy as np
import pytest
import scipy.linalg

import dense_ref as D
import oracle
from paper_2510_12717_amd import synth


def tiny_shape(N=2, nx=3):
    return synth.Shape(N=N, nx=nx, nu=4, n_tau=1, n_feet=1, foot_dim=3)


def one_agent(shape, seed=0, **over):
    b = synth.make_batch([shape], seed=seed, stream_id=99)
    ag = oracle.agent(b, 0)
    ag.update(over)
    return ag


def rel(a, b):
    a, b = np.asarray(a, dtype=float), np.asarray(b, dtype=float)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def args(ag):
    return (ag["s"], ag["A"], ag["B"], ag["c"], ag["q"], ag["r"], ag["x_ref"], ag["x0"],
            ag["tau_max"], ag["mu"], ag["stance"])


# --- problem statement ------------------------------------------------------------------

@pytest.mark.parametrize("shape", [synth.humanoid(4), synth.quadruped(3)])
def test_constraint_rows_and_bounds_match_statement(shape):
    ag = one_agent(shape, seed=3)
    st = ag["stance"].copy()
    st[0, :] = 1
    st[-1, :] = 0
    C = oracle.constraint_matrix(shape, ag["mu"])
    np.testing.assert_array_equal(C, D.C_dense(shape, ag["mu"]))
    l, h, rho = oracle.stage_bounds(shape, ag["tau_max"], st)
    le, he = D.bounds_table(shape, ag["tau_max"], st)
    np.testing.assert_array_equal(l, le)
    np.testing.assert_array_equal(h, he)
    np.testing.assert_array_equal(rho, D.rho_table(le, he))
    # swing foot: wrench rows are equalities at 0, pyramid rows free
    f0 = slice(shape.n_tau, shape.n_tau + shape.foot_dim)
    assert np.all(l[-1, f0] == 0) and np.all(h[-1, f0] == 0)
    assert np.all(np.isinf(l[-1, shape.nu:shape.nu + 4]))


def test_penalised_input_hessian_is_diagonal():
    """The four facets of a foot share one penalty, so C' diag(rho) C is diagonal:
    the f_x f_z cross terms cancel and f_z collects 4 mu^2 rho (plus its own row)."""
    s = synth.humanoid(3)
    ag = one_agent(s, seed=5)
    C = oracle.constraint_matrix(s, ag["mu"])
    _, _, rho = oracle.stage_bounds(s, ag["tau_max"], ag["stance"])
    for k in range(s.N):
        M = C.T @ np.diag(rho[k]) @ C
        assert np.abs(M - np.diag(np.diag(M))).max() < 1e-15
        for f in range(s.n_feet):
            fz = s.n_tau + f * s.foot_dim + 2
            rp = rho[k, s.nu + 4 * f]
            assert M[fz, fz] == pytest.approx(rho[k, fz] + 4 * ag["mu"] ** 2 * rp, rel=1e-14)


def test_x_subproblem_helper_matches_direct_objective():
    """Pins the dense helper itself: its (H, g) reproduce the objective at random points."""
    s = tiny_shape(N=2, nx=3)
    ag = one_agent(s, seed=1)
    rng = np.random.default_rng(0)
    C = D.C_dense(s, ag["mu"])
    l, h = D.bounds_table(s, ag["tau_max"], ag["stance"])
    rho = D.rho_table(l, h)
    xj, uj = rng.standard_normal((s.N + 1, s.nx)), rng.standard_normal((s.N, s.nu))
    z, y = rng.standard_normal((s.N, C.shape[0])), rng.standard_normal((s.N, C.shape[0]))
    H, g = D.x_subproblem(s, ag["q"], ag["r"], ag["x_ref"], C, rho, 1e-6, xj, uj, z, y)
    f = lambda v: D.x_subproblem_objective(s, ag["q"], ag["r"], ag["x_ref"], C, rho, 1e-6, xj,
                                           uj, z, y, v)
    f0 = f(np.zeros(H.shape[0]))
    for _ in range(5):
        v = rng.standard_normal(H.shape[0])
        # f0 is large (y / rho_min terms), so the difference carries its rounding
        assert f(v) - f0 == pytest.approx(0.5 * v @ H @ v + g @ v, rel=1e-10, abs=1e-14 * abs(f0))


# --- Riccati x-update == dense KKT solve -------------------------------------------------

@pytest.mark.parametrize("shape,seed", [(tiny_shape(2, 3), 0), (tiny_shape(5, 4), 1),
                                        (synth.quadruped(4), 2), (synth.humanoid(10), 3)])
def test_xupdate_equals_dense_kkt(shape, seed):
    ag = one_agent(shape, seed=seed)
    s = ag["s"]
    rng = np.random.default_rng(seed)
    C = D.C_dense(s, ag["mu"])
    l, h, rho = oracle.stage_bounds(s, ag["tau_max"], ag["stance"])
    xj, uj = rng.standard_normal((s.N + 1, s.nx)), rng.standard_normal((s.N, s.nu))
    z, y = rng.standard_normal((s.N, C.shape[0])), rng.standard_normal((s.N, C.shape[0]))
    H, g = D.x_subproblem(s, ag["q"], ag["r"], ag["x_ref"], C, rho, 1e-6, xj, uj, z, y)
    G, b = D.dynamics_rows(s, ag["A"], ag["B"], ag["c"], ag["x0"])
    v, _ = D.kkt_solve(H, g, G, b)
    x_ref_, u_ref_ = D.split(s, v, ag["x0"])

    status, K, L, sv, P = oracle.factor(s, ag["A"], ag["B"], ag["c"], ag["q"], ag["r"], rho,
                                        ag["mu"])
    assert status == oracle.OK
    qt = np.vstack([np.zeros((1, s.nx)), g[: s.N * s.nx].reshape(s.N, s.nx)])
    rt = g[s.N * s.nx:].reshape(s.N, s.nu)
    xt, ut = oracle.xupdate(s, ag["A"], ag["B"], ag["c"], K, L, sv, ag["x0"], qt, rt)
    assert rel(ut, u_ref_) < 1e-10
    assert rel(xt, x_ref_) < 1e-10
    # factor by-products: L L' = H_k (SPD), P symmetric
    for k in range(s.N):
        assert np.allclose(np.triu(L[k], 1), 0.0)
        assert np.all(np.diag(L[k]) > 0)
    for k in range(s.N + 1):
        assert np.abs(P[k] - P[k].T).max() <= 1e-12 * np.abs(P[k]).max()


# --- fixed-K iterates == OSQP iterations with dense x-updates ----------------------------

@pytest.mark.parametrize("shape,seed,iters", [(tiny_shape(2, 3), 0, 1), (tiny_shape(3, 3), 4, 7),
                                              (synth.quadruped(3), 5, 5),
                                              (synth.humanoid(4), 6, 12)])
def test_fixed_iterates_equal_dense_admm(shape, seed, iters):
    ag = one_agent(shape, seed=seed)
    out = oracle.solve(*args(ag), iters=iters)
    x, u, z, y = D.dense_admm(*args(ag), iters)
    assert out["status"] == oracle.OK
    assert rel(out["u"], u) < 1e-9
    assert rel(out["x"], x) < 1e-9
    assert rel(out["z"], z) < 1e-9
    assert rel(out["y"], y) < 1e-9


def test_warm_start_continues_the_iteration():
    """j iterations then a warm start with i more == j + i iterations from cold."""
    ag = one_agent(synth.humanoid(5), seed=8)
    a = oracle.solve(*args(ag), iters=6)
    b = oracle.solve(*args(ag), iters=4, warm=(a["u"], a["z"], a["y"]))
    c = oracle.solve(*args(ag), iters=10)
    assert rel(b["u"], c["u"]) < 1e-12
    assert rel(b["y"], c["y"]) < 1e-12


# --- converged optimum ------------------------------------------------------------------

def _active_problem(N, seed):
    s = tiny_shape(N=N, nx=3)
    ag = one_agent(s, seed=seed)
    rng = np.random.default_rng(100 + seed)
    ag["tau_max"] = np.array([0.3])
    ag["B"] = rng.standard_normal(ag["B"].shape) * 0.5
    ag["x_ref"] = rng.standard_normal(ag["x_ref"].shape) * 3.0
    ag["q"] = 10 ** rng.uniform(-1, 1, s.nx)
    ag["r"] = 10 ** rng.uniform(-2, -1, s.nu)
    ag["mu"] = 0.5
    ag["stance"] = rng.integers(0, 2, (N, 1)).astype(np.uint8)
    ag["stance"][0, 0] = 1
    return ag


@pytest.mark.parametrize("N,seed", [(1, 0), (1, 1), (2, 2), (2, 3), (2, 4)])
def test_converged_equals_brute_force_active_set(N, seed):
    ag = _active_problem(N, seed)
    bf = D.brute_force_qp(*args(ag))
    assert bf is not None
    xb, ub, yb = bf
    out = oracle.solve(*args(ag), iters=0, tol=1e-12, max_iters=2_000_000)
    assert out["status"] == oracle.CONVERGED
    assert rel(out["u"], ub) < 1e-8
    assert rel(out["x"], xb) < 1e-8
    # at least one inequality is active somewhere in these instances
    C = D.C_dense(ag["s"], ag["mu"])
    l, h = D.bounds_table(ag["s"], ag["tau_max"], ag["stance"])
    cu = ub @ C.T
    act = (np.isclose(cu, l) | np.isclose(cu, h)) & (l != h)
    assert act.any()
    # multipliers need not be unique (at f = 0 the f_z row and all four facets are
    # active), so check the oracle's y itself: stationarity of the Lagrangian
    # with some dynamics costate, and y in the normal cone of [l, h] at z.
    s = ag["s"]
    G, b = D.dynamics_rows(s, ag["A"], ag["B"], ag["c"], ag["x0"])
    nv = G.shape[1]
    grad = np.zeros(nv)
    grad[: s.N * s.nx] = (ag["q"] * (out["x"][1:] - ag["x_ref"][1:])).ravel()
    grad[s.N * s.nx:] = (ag["r"] * out["u"]).ravel() + (out["y"] @ C).ravel()
    lam, *_ = np.linalg.lstsq(G.T, -grad, rcond=None)
    assert np.abs(grad + G.T @ lam).max() < 1e-8 * max(1.0, np.abs(grad).max())
    yo, zo = out["y"], out["z"]
    assert np.all((yo <= 1e-9) | np.isclose(zo, h, atol=1e-9))
    assert np.all((yo >= -1e-9) | np.isclose(zo, l, atol=1e-9))


def test_no_active_constraint_equals_condensed_lqr():
    """No feet, loose torque box: the QP is an unconstrained LQR; its optimum
    solves the condensed normal equations."""
    s = synth.Shape(N=4, nx=5, nu=3, n_tau=3, n_feet=0, foot_dim=3)
    ag = one_agent(s, seed=11)
    rng = np.random.default_rng(11)
    ag["B"] = rng.standard_normal(ag["B"].shape) * 0.3
    ag["tau_max"] = np.full(3, 1e8)
    ag["stance"] = np.zeros((s.N, 0), dtype=np.uint8)
    out = oracle.solve(*args(ag), iters=0, tol=1e-12, max_iters=500_000)
    assert out["status"] == oracle.CONVERGED
    u = D.unconstrained_optimum(s, ag["A"], ag["B"], ag["c"], ag["q"], ag["r"], ag["x_ref"],
                                ag["x0"])
    assert rel(out["u"], u) < 1e-8
    assert np.abs(out["y"]).max() < 1e-8


def test_factor_gains_equal_condensed_feedback():
    """With sigma = rho = 0 the factor's gains are the finite-horizon LQR
    feedback: u_k = K_k x_k is the condensed optimum of the tail problem from
    stage k (c = 0, r = 0)."""
    s = synth.Shape(N=5, nx=4, nu=3, n_tau=3, n_feet=0, foot_dim=3)
    ag = one_agent(s, seed=12)
    st = oracle.Settings.default(sigma=0.0)
    rho0 = np.zeros((s.N, s.nu))
    status, K, L, sv, P = oracle.factor(s, ag["A"], ag["B"], ag["c"], ag["q"], ag["r"], rho0,
                                        ag["mu"], settings=st)
    assert status == oracle.OK
    for k0 in (0, 2, s.N - 1):
        t = synth.Shape(N=s.N - k0, nx=4, nu=3, n_tau=3, n_feet=0, foot_dim=3)
        A, B = ag["A"][k0:], ag["B"][k0:]
        zc = np.zeros((t.N, t.nx))
        zr = np.zeros((t.N + 1, t.nx))
        Kc = np.zeros((t.nu, t.nx))
        for j in range(t.nx):
            e = np.zeros(t.nx)
            e[j] = 1.0
            Kc[:, j] = D.unconstrained_optimum(t, A, B, zc, ag["q"], ag["r"], zr, e)[0]
        assert rel(K[k0], Kc) < 1e-10


def test_long_horizon_gain_tends_to_dare():
    s = synth.Shape(N=400, nx=4, nu=2, n_tau=2, n_feet=0, foot_dim=3)
    rng = np.random.default_rng(13)
    A1 = np.eye(4) + 0.1 * rng.standard_normal((4, 4)) / 2
    B1 = 0.1 * rng.standard_normal((4, 2))
    q = 10 ** rng.uniform(-1, 1, 4)
    r = 10 ** rng.uniform(-2, 0, 2)
    A = np.repeat(A1[None], s.N, axis=0)
    B = np.repeat(B1[None], s.N, axis=0)
    st = oracle.Settings.default(sigma=0.0)
    status, K, *_ = oracle.factor(s, A, B, np.zeros((s.N, 4)), q, r, np.zeros((s.N, 2)), 0.5,
                                  settings=st)
    Pd = scipy.linalg.solve_discrete_are(A1, B1, np.diag(q), np.diag(r))
    Kd = -np.linalg.solve(np.diag(r) + B1.T @ Pd @ B1, B1.T @ Pd @ A1)
    assert status == oracle.OK
    assert rel(K[0], Kd) < 1e-9


def test_paper_form_osqp_reaches_same_optimum():
    """OSQP on the paper's quasi-definite KKT system with the dynamics as
    finite-penalty rows converges to the same QP optimum as the oracle."""
    ag = _active_problem(2, 7)
    xs, us = D.osqp_dense(*args(ag))
    out = oracle.solve(*args(ag), iters=0, tol=1e-12, max_iters=2_000_000)
    assert out["status"] == oracle.CONVERGED
    assert rel(out["u"], us) < 1e-7


def test_fixed_point_of_the_iteration():
    ag = _active_problem(2, 9)
    out = oracle.solve(*args(ag), iters=0, tol=1e-13, max_iters=2_000_000)
    one = oracle.solve(*args(ag), iters=1, warm=(out["u"], out["z"], out["y"]))
    assert rel(one["u"], out["u"]) < 1e-10
    assert rel(one["z"], out["z"]) < 1e-10
    assert rel(one["y"], out["y"]) < 1e-9


# --- invariants that hold at every iterate ------------------------------------------------

def test_invariants_every_iteration():
    ag = one_agent(synth.humanoid(6), seed=21)
    s = ag["s"]
    C = D.C_dense(s, ag["mu"])
    l, h = D.bounds_table(s, ag["tau_max"], ag["stance"])
    for j in (1, 2, 3, 5, 10, 25, 50):
        o = oracle.solve(*args(ag), iters=j)
        x, u, z, y = o["x"], o["u"], o["z"], o["y"]
        assert np.array_equal(x[0], ag["x0"])
        xr = D.rollout(s, ag["A"], ag["B"], ag["c"], ag["x0"], u)
        assert rel(x, xr) < 1e-12
        assert np.all(z >= l) and np.all(z <= h)
        scale = np.abs(y).max()
        pos, neg = y > 1e-12 * scale, y < -1e-12 * scale
        assert np.array_equal(z[pos], h[pos])
        assert np.array_equal(z[neg], l[neg])
        # the oracle's own residual report agrees with the direct checks
        assert o["res"][2] < 1e-12 * max(1.0, np.abs(x).max())


def test_small_humanoid_agent_converges_to_kkt_tolerance():
    """Converge mode on a full humanoid agent reaches KKT, complementarity and
    dynamics residuals below 1e-9."""
    b = synth.small_humanoid_batch(1)
    ag = oracle.agent(b, 0)
    out = oracle.solve(*args(ag), iters=0, tol=1e-12, max_iters=400_000)
    assert out["status"] == oracle.CONVERGED, out["iters"]
    assert np.all(out["res"] < 1e-9), out["res"]


# --- failure handling and batching ---------------------------------------------------------

def test_batch_equals_single_and_failures_stay_local():
    b = synth.small_humanoid_batch(6)
    b.A[b.offsets()["A"][2] + 17] = np.nan  # agent 2: NaN in A
    o = b.offsets()
    b.r[o["r"][4]:o["r"][5]] = -5.0  # agent 4: indefinite R
    out = oracle.solve_batch(b, iters=20)
    assert out["status"].tolist() == [0, 0, oracle.NONFINITE, 0, oracle.NOT_PD, 0]
    for a in (0, 1, 3, 5):
        single = oracle.solve(*args(oracle.agent(b, a)), iters=20)
        np.testing.assert_array_equal(out["u"][o["u"][a]:o["u"][a + 1]], single["u"].ravel())
    assert np.all(np.isnan(out["u"][o["u"][2]:o["u"][3]]))


def test_subset_reproduces_agents():
    b = synth.small_humanoid_batch(8)
    sub = synth.small_humanoid_batch(agent_ids=[5, 2])
    full = oracle.solve_batch(b, iters=10)
    part = oracle.solve_batch(sub, iters=10)
    o, p = b.offsets(), sub.offsets()
    for j, a in enumerate((5, 2)):
        np.testing.assert_array_equal(full["u"][o["u"][a]:o["u"][a + 1]],
                                      part["u"][p["u"][j]:p["u"][j + 1]])


def test_residuals_match_lagrangian_gradient():
    """The oracle's residual report equals quantities built independently from
    the stacked QP: primal |Cu - z|, dynamics |Gv - b|, the objective, and the
    dual residual = gradient in u of the Lagrangian f + mu'(Gv - b) + y'Cu with
    mu chosen so the gradient in x vanishes."""
    s = synth.quadruped(4)
    ag = one_agent(s, seed=31)
    rng = np.random.default_rng(31)
    C = D.C_dense(s, ag["mu"])
    x = rng.standard_normal((s.N + 1, s.nx))
    x[0] = ag["x0"]
    u = rng.standard_normal((s.N, s.nu))
    z = rng.standard_normal((s.N, C.shape[0]))
    y = rng.standard_normal((s.N, C.shape[0]))
    res, obj = oracle.residuals(s, ag["A"], ag["B"], ag["c"], ag["q"], ag["r"], ag["x_ref"],
                                ag["x0"], ag["tau_max"], ag["mu"], ag["stance"], x, u, z, y)
    G, b = D.dynamics_rows(s, ag["A"], ag["B"], ag["c"], ag["x0"])
    v = np.concatenate([x[1:].ravel(), u.ravel()])
    nxv = s.N * s.nx
    grad = np.concatenate([(ag["q"] * (x[1:] - ag["x_ref"][1:])).ravel(), (ag["r"] * u).ravel()])
    mu_ = np.linalg.solve(G[:, :nxv].T, -grad[:nxv])
    dual = grad[nxv:] + G[:, nxv:].T @ mu_ + (y @ C).ravel()
    f = 0.5 * np.sum(ag["q"] * (x[1:] - ag["x_ref"][1:]) ** 2) + 0.5 * np.sum(ag["r"] * u ** 2)
    assert res[0] == pytest.approx(np.abs(u @ C.T - z).max(), rel=1e-12)
    assert res[1] == pytest.approx(np.abs(dual).max(), rel=1e-9)
    assert res[2] == pytest.approx(np.abs(G @ v - b).max(), rel=1e-9)
    assert obj == pytest.approx(f, rel=1e-12)


def test_complementarity_residual_is_the_projection_residual():
    """res[3] equals the projection residual |z - Pi(z + y)| with the distance of
    z from [l, h] (a formulation of complementarity independent of the oracle's
    per-sign minima): zero at a complementary pair built as z = Pi(v), y = v - z,
    and equal to it once z leaves its bound, crosses it, or y takes the wrong sign."""
    s = synth.quadruped(4)
    ag = one_agent(s, seed=37)
    l, h = D.bounds_table(s, ag["tau_max"], ag["stance"])
    C = D.C_dense(s, ag["mu"])
    rng = np.random.default_rng(37)
    x = rng.standard_normal((s.N + 1, s.nx))
    u = rng.standard_normal((s.N, s.nu))

    def res3(z, y):
        res, _ = oracle.residuals(s, ag["A"], ag["B"], ag["c"], ag["q"], ag["r"], ag["x_ref"],
                                  ag["x0"], ag["tau_max"], ag["mu"], ag["stance"], x, u, z, y)
        return res[3]

    v = rng.standard_normal(l.shape) * 60.0
    z0 = np.clip(v, l, h)
    y0 = v - z0
    assert np.count_nonzero(y0 > 0) > 3 and np.count_nonzero(y0 < 0) > 3
    assert res3(z0, y0) == 0.0 and D.complementarity_natural(l, h, z0, y0) == 0.0
    for trial in range(6):
        z, y = z0.copy(), y0.copy()
        pick = rng.random(l.shape) < 0.3
        if trial % 3 == 0:    # z moved off (or across) its bound
            z[pick] += rng.standard_normal(np.count_nonzero(pick)) * 5.0
        elif trial % 3 == 1:  # multipliers of the wrong sign
            y[pick] = -y[pick] + rng.standard_normal(np.count_nonzero(pick))
        else:                 # both, with z also outside some bounds
            z[pick] += rng.standard_normal(np.count_nonzero(pick)) * 50.0
            y += rng.standard_normal(y.shape)
        want = D.complementarity_natural(l, h, z, y)
        assert want > 0.1
        assert res3(z, y) == pytest.approx(want, rel=1e-12)


def test_plant_step_is_the_solved_first_transition():
    """The closed-loop plant step x0 <- A_0 x0 + B_0 u_0 + c_0 + w: with w = 0 it
    reproduces x_1 of the solved trajectory, which meets the dynamics exactly at
    every iterate (rollout start, affine relaxation), over agents of different
    shapes and horizons; w adds on unchanged."""
    b = synth.uneven_batch(6)
    o = oracle.solve_batch(b, iters=20)
    off = b.offsets()
    x1 = np.concatenate([o["x"][off["x"][a] + s.nx:off["x"][a] + 2 * s.nx]
                         for a, s in enumerate(b.shapes)])
    got = oracle.advance_batch(b, b.x0, o["u"], np.zeros_like(x1))
    assert rel(got, x1) < 1e-12
    w = np.random.default_rng(3).standard_normal(x1.size)
    got_w = oracle.advance_batch(b, b.x0, o["u"], w)
    assert np.abs(got_w - got - w).max() < 1e-12
