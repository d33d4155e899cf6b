"""Pins of the oracle's paper-form inner solve (oracle/kkt.py: OSQP on the
standard form with the quasi-definite KKT matrix of Eq. (kkt_system)
factored once by LDL^T, Eq. (ldl), and solved by Eq. (backsolve_2)) against
things other than itself (CPU only): the factor reproduces the matrix with
the inertia of a quasi-definite matrix, the backsolve equals a dense solve,
fixed iterates equal a dense OSQP iteration written independently, the
iterates approach the exact-dynamics oracle as rho_eq grows, converged
iterates reach the brute-force optimum, and planted mistakes are caught."""
import os
import types

import numpy as np
import pytest

import dense_ref as D
import oracle
from oracle import kkt as KKT
from paper_2510_12717_amd import synth

ARGS = ("s", "A", "B", "c", "q", "r", "x_ref", "x0", "tau_max", "mu", "stance")
TINY = synth.Shape(N=3, nx=4, nu=4, n_tau=1, n_feet=1, foot_dim=3)


def agent(shape, seed):
    b = synth.make_batch([shape], seed=seed, stream_id=91)
    return oracle.agent(b, 0)


def rel(a, b):
    a, b = np.asarray(a, dtype=float), np.asarray(b, dtype=float)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("shape", [TINY, synth.quadruped(3), synth.humanoid(2)])
def test_factor_reproduces_the_kkt_matrix(shape, K=KKT):
    ag = agent(shape, 1)
    prob = K.standard_form(ag)
    fac = K.Factor(prob, 1e-6, shape)
    Kp = fac.K[np.ix_(fac.perm, fac.perm)]
    assert sorted(fac.perm) == list(range(Kp.shape[0]))
    assert np.allclose(np.triu(fac.L, 1), 0) and np.all(np.diag(fac.L) == 1)
    assert rel(fac.L @ np.diag(fac.d) @ fac.L.T, Kp) < 1e-13
    # quasi-definite: as many positive pivots as primal unknowns, the rest negative
    assert (fac.d > 0).sum() == prob["nv"] and (fac.d < 0).sum() == prob["A"].shape[0]
    # the standard form is the statement's: P, q, A, bounds and the penalty rule
    C = D.C_dense(shape, ag["mu"])
    G, b = D.dynamics_rows(shape, ag["A"], ag["B"], ag["c"], ag["x0"])
    N, nx, nu, m = shape.N, shape.nx, shape.nu, C.shape[0]
    assert np.array_equal(prob["A"][:N * nx], G) and np.allclose(prob["l"][:N * nx], b)
    for k in range(N):
        assert np.array_equal(prob["A"][N * nx + k * m:N * nx + (k + 1) * m, N * nx + k * nu:N * nx + (k + 1) * nu], C)
    l, h = D.bounds_table(shape, ag["tau_max"], ag["stance"])
    assert np.array_equal(prob["l"][N * nx:], l.ravel()) and np.array_equal(prob["h"][N * nx:], h.ravel())
    rr = np.concatenate([np.full(N * nx, 100.0), D.rho_table(l, h).ravel()])
    assert np.allclose(prob["rho"], rr, rtol=1e-15)


@pytest.mark.parametrize("shape", [TINY, synth.quadruped(3)])
def test_backsolve_equals_dense_solve(shape, K=KKT):
    ag = agent(shape, 2)
    prob = K.standard_form(ag)
    fac = K.Factor(prob, 1e-6, shape)
    rhs = np.random.default_rng(2).standard_normal(fac.K.shape[0])
    assert rel(fac.solve(rhs), np.linalg.solve(fac.K, rhs)) < 1e-10


@pytest.mark.parametrize("shape,seed,iters", [(TINY, 3, 9), (synth.quadruped(3), 4, 7), (synth.humanoid(2), 5, 5)])
def test_fixed_iterates_equal_dense_osqp(shape, seed, iters, K=KKT):
    ag = agent(shape, seed)
    o = K.solve(ag, iters=iters)
    d = D.osqp_dense_fixed(*[ag[k] for k in ARGS], iters)
    for k in ("x", "u", "z", "y", "zd", "yd"):
        assert rel(o[k], d[k]) < 1e-9, k
    # and warm: the next iterations from the same iterate
    o2 = K.solve(ag, iters=3, warm=(o["v"], o["z_all"], o["y_all"]))
    d2 = D.osqp_dense_fixed(*[ag[k] for k in ARGS], 3, warm=(d["v"], d["z_all"], d["y_all"]))
    assert rel(o2["u"], d2["u"]) < 1e-9 and rel(o2["yd"], d2["yd"]) < 1e-9


@pytest.mark.parametrize("shape", [TINY, synth.humanoid(4)])
def test_large_rho_eq_approaches_the_exact_dynamics_oracle(shape, K=KKT):
    """The exact-dynamics reading is the rho_eq -> infinity limit of this one:
    at rho_eq = 1e6 the 50th iterates agree with the Riccati oracle's to
    1e-5, at the default 1e2 they differ."""
    ag = agent(shape, 6)
    r = oracle.solve(*[ag[k] for k in ARGS], iters=50)
    far = K.solve(ag, iters=50)
    near = K.solve(ag, iters=50, settings=oracle.Settings.default(rho_eq_scale=1e7))
    assert rel(near["u"], r["u"]) < 1e-5 and rel(near["x"], r["x"]) < 1e-5
    assert rel(far["u"], r["u"]) > 10 * rel(near["u"], r["u"])


def test_converged_iterates_reach_the_brute_force_optimum(K=KKT):
    s = synth.Shape(N=2, nx=2, nu=4, n_tau=1, n_feet=1, foot_dim=3)
    found = 0
    for seed in range(6):
        ag = agent(s, 300 + seed)
        ref = D.brute_force_qp(*[ag[k] for k in ARGS])
        if ref is None:
            continue
        x, u = ref[0], ref[1]
        o = K.solve(ag, iters=200000, tol=1e-12)
        assert o["iters"] < 200000
        assert rel(o["u"], u) < 1e-7 and rel(o["x"], x) < 1e-7
        found += 1
    assert found >= 3


def test_batch_equals_single_solves():
    b = synth.uneven_batch(3)
    o = KKT.solve_batch(b, iters=10)
    off = b.offsets()
    for a in range(b.n_agents):
        one = KKT.solve(oracle.agent(b, a), iters=10)
        assert np.array_equal(o["u"][off["u"][a]:off["u"][a + 1]], one["u"].ravel())
        assert np.array_equal(o["yd"][off["c"][a]:off["c"][a + 1]], one["yd"].ravel())


# planted mistakes: each is a textual change of a copy of kkt.py; at least one
# pin above must fail on the copy
SRC = os.path.join(os.path.dirname(KKT.__file__), "kkt.py")
MUTANTS = [
    ("LDL update with the wrong sign", "W[j + 1:e, j + 1:e] -= d[j] * np.outer(col, col)",
     "W[j + 1:e, j + 1:e] += d[j] * np.outer(col, col)"),
    ("backsolve without the diagonal scaling", "    w = w / d\n", "\n"),
    ("dual block with +1/rho", "K[nv:, nv:] = -np.diag(1.0 / prob[\"rho\"])", "K[nv:, nv:] = np.diag(1.0 / prob[\"rho\"])"),
    ("zt from nu alone", "zt = z + (nuk - y) / rho", "zt = z + nuk / rho"),
    ("equality rows with the inequality penalty", "rho = np.where(lo == hi, st.rho_eq_scale * st.rho, st.rho)",
     "rho = np.where(lo == hi, st.rho, st.rho)"),
    ("x_0 term missing from the first dynamics row", "rhs = ag[\"c\"][k] + (ag[\"A\"][0] @ ag[\"x0\"] if k == 0 else 0.0)",
     "rhs = ag[\"c\"][k]"),
    ("no relaxation of v", "v = alpha * xt + (1.0 - alpha) * v", "v = xt"),
    ("cold start with z = 0", "return v, prob[\"A\"] @ v, np.zeros(prob[\"A\"].shape[0])",
     "return v, np.zeros(prob[\"A\"].shape[0]), np.zeros(prob[\"A\"].shape[0])"),
]
CHECKS = [
    lambda K: test_factor_reproduces_the_kkt_matrix(synth.quadruped(3), K=K),
    lambda K: test_backsolve_equals_dense_solve(TINY, K=K),
    lambda K: test_fixed_iterates_equal_dense_osqp(synth.quadruped(3), 4, 7, K=K),
]


def _mutant(text):
    mod = types.ModuleType("oracle._kkt_mutant")
    mod.__package__ = "oracle"
    exec(compile(text, SRC + " (mutant)", "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(name, old, new):
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation site not unique/present: {name}"
    K = _mutant(text.replace(old, new))
    caught = False
    for chk in CHECKS:
        try:
            chk(K)
        except Exception:  # a failing pin (or a crash of the broken copy)
            caught = True
            break
    assert caught, f"no pin failed for mutant: {name}"


def test_unmutated_copy_passes_every_check():
    K = _mutant(open(SRC).read())
    for chk in CHECKS:
        chk(K)
