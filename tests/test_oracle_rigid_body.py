"""Pins of the oracle's rigid-body dynamics (oracle/rigid_body.py: Eq. (rnea),
the mass matrix, forward dynamics, the semi-implicit Euler step of
Eq. (mpc_formulation) and its linearisation, Eq. (mpc_torque)) against
mechanics computed without the spatial recursion (CPU only): potential and
kinetic energy from the bodies' world poses alone, Lagrange's equations, the
feet's Jacobians from their world positions and orientations, and the
inverse/forward dynamics pair."""
import numpy as np
import pytest

from oracle import rigid_body as RB
from paper_2510_12717_amd import synth

MODELS = {k: synth.articulated_model(k, seed=3) for k in ("humanoid", "quadruped")}


def state(kind, i=0):
    m = MODELS[kind]
    s = synth.model_states(m, 4, seed=11)
    return m, s["q"][i], s["qd"][i], s["qdd"][i], s["tau"][i], s["F"][i], s["dt"]


def poses(m, q):
    _, _, R, p = RB.kinematics(m, q)
    return R, p


def potential(m, q):
    R, p = poses(m, q)
    return sum(m["mass"][i] * m["gravity"] * (p[i] + R[i] @ m["com"][i])[2] for i in range(m["n"]))


def kinetic(m, q, qd, h=1e-30):
    """Kinetic energy from the world poses only: centre-of-mass velocities and
    angular velocities (Rdot R' = w x) by complex steps along qd, plus each
    actuator rotor's energy (armature_i qd_i^2 / 2)."""
    R, p = poses(m, q)
    Rc, pc = poses(m, q.astype(complex) + 1j * h * qd)
    T = 0.5 * float(np.sum(m["armature"] * qd * qd))
    for i in range(m["n"]):
        vc = (pc[i] + Rc[i] @ m["com"][i]).imag / h
        W = (Rc[i].imag / h) @ R[i].T
        w = np.array([W[2, 1], W[0, 2], W[1, 0]])
        Iw = R[i] @ np.diag(m["inertia"][i]) @ R[i].T
        T += 0.5 * m["mass"][i] * vc @ vc + 0.5 * w @ Iw @ w
    return T


def mass_from_energy(m, q):
    n = m["n"]
    E = np.eye(n)
    d = np.array([kinetic(m, q, E[i]) for i in range(n)])
    M = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            M[i, j] = 2 * d[i] if i == j else kinetic(m, q, E[i] + E[j]) - d[i] - d[j]
    return M


def rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("kind", ["humanoid", "quadruped"])
def test_gravity_torques_are_the_potential_gradient(kind):
    m, q, *_ = state(kind)
    n = m["n"]
    z = np.zeros(n)
    g = RB.rnea(m, q, z, z)
    grad = np.array([potential(m, q + 1j * 1e-30 * np.eye(n)[j]).imag / 1e-30 for j in range(n)])
    assert rel(g, grad) < 1e-12


@pytest.mark.parametrize("kind", ["humanoid", "quadruped"])
def test_mass_matrix_is_the_kinetic_energy_hessian(kind):
    m, q, *_ = state(kind, 1)
    M = RB.mass_matrix(m, q)
    Me = mass_from_energy(m, q)
    assert rel(M, Me) < 1e-12
    assert rel(M, M.T) < 1e-13 and np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0


@pytest.mark.parametrize("kind", ["humanoid", "quadruped"])
def test_bias_forces_satisfy_lagrange(kind):
    """h(q, qd) - g(q) = Mdot qd - dT/dq, with T and M from the poses only."""
    m, q, qd, *_ = state(kind, 2)
    n = m["n"]
    z = np.zeros(n)
    h = RB.rnea(m, q, qd, z) - RB.rnea(m, q, z, z)
    eps = 1e-5
    Mdot = (mass_from_energy(m, q + eps * qd) - mass_from_energy(m, q - eps * qd)) / (2 * eps)
    dTdq = np.array([(kinetic(m, q + eps * np.eye(n)[j], qd) - kinetic(m, q - eps * np.eye(n)[j], qd)) / (2 * eps)
                     for j in range(n)])
    assert rel(h, Mdot @ qd - dTdq) < 1e-7


@pytest.mark.parametrize("kind", ["humanoid", "quadruped"])
def test_foot_wrenches_enter_as_minus_jacobian_transpose(kind):
    m, q, _, _, _, F, _ = state(kind, 3)
    n = m["n"]
    z = np.zeros(n)
    ext = RB.rnea(m, q, z, z, F) - RB.rnea(m, q, z, z)
    R, p = poses(m, q)
    want = np.zeros(n)
    fd = m["foot_dim"]
    for f, b in enumerate(m["foot_body"]):
        for j in range(n):
            Rc, pc = poses(m, q + 1j * 1e-30 * np.eye(n)[j])
            v = (pc[b] + Rc[b] @ m["foot_offset"][f]).imag / 1e-30   # point velocity per unit qd_j
            W = (Rc[b].imag / 1e-30) @ R[b].T
            w = np.array([W[2, 1], W[0, 2], W[1, 0]])                 # angular velocity per unit qd_j
            want[j] -= v @ F[f * fd:f * fd + 3]
            if fd == 6:
                want[j] -= w @ F[f * fd + 3:f * fd + 6]
    assert rel(ext, want) < 1e-12


@pytest.mark.parametrize("kind", ["humanoid", "quadruped"])
def test_foot_jacobian_is_rneas_wrench_map(kind):
    """-J' F from the oracle's foot Jacobian (kinematics only) equals the foot
    wrenches' term of RNEA (force propagation), for several wrenches; the
    no-slip rows carry J on the velocities only."""
    m, q, *_ = state(kind, 2)
    n = m["n"]
    z = np.zeros(n)
    J = RB.foot_jacobian(m, q)
    s = synth.model_states(m, 3, seed=17)
    for F in s["F"]:
        assert rel(-J.T @ F, RB.rnea(m, q, z, z, F) - RB.rnea(m, q, z, z)) < 1e-12
    rows = RB.noslip_rows(m, np.concatenate([q, z]))
    assert np.all(rows[:, :n] == 0) and np.array_equal(rows[:, n:], J)


@pytest.mark.parametrize("kind", ["humanoid", "quadruped"])
def test_forward_dynamics_inverts_rnea(kind):
    m, q, qd, _, tau, F, _ = state(kind)
    qdd = RB.forward_dynamics(m, q, qd, tau, F)
    gen = RB.rnea(m, q, qd, qdd, F)
    assert np.abs(gen[:6]).max() < 1e-9 * np.abs(tau).max() and rel(gen[6:], tau) < 1e-11


@pytest.mark.parametrize("kind", ["humanoid", "quadruped"])
def test_linearisation(kind):
    """A, B by complex steps equal central differences of the step; B equals
    the closed form dt [dt; 1] M^-1 [S', J'] with M and J from the poses."""
    m, q, qd, _, tau, F, dt = state(kind, 1)
    n, nj = m["n"], m["n_joints"]
    x, u = np.concatenate([q, qd]), np.concatenate([tau, F])
    A, B, c = RB.linearize(m, x, u, dt)
    eps = 1e-6
    Af = np.column_stack([(RB.step(m, x + eps * e, u, dt) - RB.step(m, x - eps * e, u, dt)) / (2 * eps)
                          for e in np.eye(len(x))])
    assert rel(A, Af) < 1e-6
    assert rel(RB.step(m, x, u, dt), A @ x + B @ u + c) < 1e-12
    # closed form of B: d qdd / du = M^-1 [S', J']
    M = mass_from_energy(m, q)
    G = np.zeros((n, len(u)))
    G[6:, :nj] = np.eye(nj)
    z = np.zeros(n)
    for k in range(len(u) - nj):
        e = np.zeros(len(u) - nj)
        e[k] = 1.0
        G[:, nj + k] = -(RB.rnea(m, q, z, z, e) - RB.rnea(m, q, z, z))   # J' e_k
    dqdd = np.linalg.solve(M, G)
    assert rel(B, np.vstack([dt * dt * dqdd, dt * dqdd])) < 1e-10


def test_mpc_torque_is_pd_plus_feedforward():
    m, q, qd, qdd, _, F, _ = state("humanoid")
    tr = RB.rnea(m, q, qd, qdd, F)
    q1, qd1 = q + 0.01, qd - 0.02
    t = RB.mpc_torque(m, tr, q1, qd1, q, qd, kp=50.0, kd=2.0)
    assert np.allclose(t, 50.0 * 0.01 + 2.0 * (-0.02) + tr[6:], rtol=0, atol=1e-12)


# planted mistakes: each is a textual change of a copy of rigid_body.py; at
# least one pin above must fail on the copy
import os
import types

SRC = os.path.join(os.path.dirname(RB.__file__), "rigid_body.py")
MUTANTS = [
    ("joint rotation not transposed", "return plucker(axis_rotation(a, qi).T,", "return plucker(axis_rotation(a, qi),"),
    ("velocity-product acceleration dropped", "a[i] = X[i] @ ap + S * qdd[i] + crm(v[i]) @ (S * qd[i])",
     "a[i] = X[i] @ ap + S * qdd[i]"),
    ("gyroscopic force dropped", "f[i] = I @ a[i] + crf(v[i]) @ (I @ v[i])", "f[i] = I @ a[i]"),
    ("foot wrench with the wrong sign", "f[b] = f[b] - np.linalg.inv(X0[b]).T @ fw", "f[b] = f[b] + np.linalg.inv(X0[b]).T @ fw"),
    ("force transmitted without the transpose", "f[par] = f[par] + X[i].T @ f[i]", "f[par] = f[par] + X[i] @ f[i]"),
    ("inertia without the parallel-axis term", "I[:3, :3] = Ic + m * C @ C.T", "I[:3, :3] = Ic"),
    ("gravity downward", "a_root[5] = model[\"gravity\"]", "a_root[5] = -model[\"gravity\"]"),
    ("explicit instead of semi-implicit Euler", "return np.concatenate([q + dt * qd1, qd1])",
     "return np.concatenate([q + dt * qd, qd1])"),
    ("armature dropped", "tau = tau + np.asarray(model[\"armature\"]) * qdd", "tau = tau"),
]


def _mutant(text):
    mod = types.ModuleType("oracle._rigid_body_mutant")
    mod.__package__ = "oracle"
    exec(compile(text, SRC + " (mutant)", "exec"), mod.__dict__)
    return mod


def _checks():
    # fast pins first; the Lagrange pin last
    return [test_gravity_torques_are_the_potential_gradient, test_mass_matrix_is_the_kinetic_energy_hessian,
            test_foot_wrenches_enter_as_minus_jacobian_transpose, test_linearisation,
            test_bias_forces_satisfy_lagrange]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(name, old, new, monkeypatch):
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation site not unique/present: {name}"
    monkeypatch.setattr(__import__(__name__), "RB", _mutant(text.replace(old, new)))
    caught = False
    for chk in _checks():
        try:
            chk("quadruped")
        except Exception:  # a failing pin (or a crash of the broken copy)
            caught = True
            break
    assert caught, f"no pin failed for mutant: {name}"
