"""Rigid-body dynamics of the real-time iteration's front and back end, for the
FP64 oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this module; the HIP product path never does.

Alg. 1 forms the QP from the robot model (f_KKT) and, after the QP
iterations, computes feed-forward torques by the recursive Newton-Euler
algorithm (f_RNEA, Eq. (rnea)) and the commanded torques with a PD term
(Eq. (mpc_torque)).  This module writes those steps out for a kinematic tree
(``synth.articulated_model``) in plain numpy, in spatial (6D) vector algebra
(angular part first), every function also valid for complex arguments so
that tests can differentiate it by complex steps:

* ``rnea``: inverse dynamics M(q) qdd + h(q, qd) - J(q)' F, gravity entering
  as an upward acceleration of the root, foot wrenches F (world frame, at the
  contact points; force then moment for 6D feet) as external forces, and each
  joint's armature (its actuator's reflected rotor inertia) times its qdd;
* ``mass_matrix``: M(q), column j = rnea(q, 0, e_j) - rnea(q, 0, 0);
* ``forward_dynamics``: qdd = M^-1 (S' tau + J' F - h), with S' tau the joint
  torques in the joint coordinates (the six base coordinates unactuated);
* ``step``: the semi-implicit Euler step of Eq. (mpc_formulation),
  qd+ = qd + dt qdd(q, qd, u), q+ = q + dt qd+, on the state x = (q, qd) and
  input u = (joint torques, foot wrenches) -- the layout of the QP's shapes;
* ``linearize``: the QP data of one stage about (x, u): A = df/dx, B = df/du
  by complex steps (exact to rounding), c = f(x, u) - A x - B u;
* ``mpc_torque``: Eq. (mpc_torque) for the joints, tau = Kp (q_mpc - q) +
  Kd (qd_mpc - qd) + tau_rnea;
* ``foot_jacobian``, ``noslip_rows``: the feet's velocity Jacobian and the
  no-slip rows J_f v = 0 of Eq. (mpc_formulation) over the state.

Conventions (readings): a joint's frame sits at its offset in the parent
frame with the parent's orientation; a revolute joint rotates the body frame
about its axis by q, a prismatic one translates it along the axis; a body's
inertia is its mass, centre of mass and principal inertia in the body frame;
a joint's armature adds armature_i qdd_i to its torque, so M(q) gains it on
the diagonal (models without the key have none).
"""
from __future__ import annotations

import numpy as np


def skew(v):
    return np.array([[0, -v[2], v[1]], [v[2], 0, -v[0]], [-v[1], v[0], 0]], dtype=np.result_type(v, 1.0))


def axis_rotation(a, th):
    """Rotation matrix (body axes in parent coordinates) by angle th about the
    unit axis a (Rodrigues)."""
    K = skew(a)
    return np.eye(3) + np.sin(th) * K + (1 - np.cos(th)) * (K @ K)


def plucker(E, r):
    """Motion transform from frame A to frame B, where E maps A coordinates to
    B coordinates and r is B's origin in A coordinates."""
    X = np.zeros((6, 6), dtype=np.result_type(E, r))
    X[:3, :3] = E
    X[3:, 3:] = E
    X[3:, :3] = -E @ skew(r)
    return X


def crm(v):
    """Spatial cross product for motion vectors, v x ."""
    M = np.zeros((6, 6), dtype=v.dtype)
    M[:3, :3] = skew(v[:3])
    M[3:, 3:] = skew(v[:3])
    M[3:, :3] = skew(v[3:])
    return M


def crf(v):
    """Spatial cross product for force vectors, v x* = -(v x)'."""
    return -crm(v).T


def spatial_inertia(m, c, Ic):
    """Spatial inertia at the body origin of mass m with centre of mass c and
    rotational inertia Ic about c (body frame)."""
    C = skew(c)
    I = np.zeros((6, 6))
    I[:3, :3] = Ic + m * C @ C.T
    I[:3, 3:] = m * C
    I[3:, :3] = m * C.T
    I[3:, 3:] = m * np.eye(3)
    return I


def joint_transform(model, i, qi):
    """Transform from body i's parent frame to body i's frame at joint value qi."""
    a = model["axis"][i]
    if model["jtype"][i] == 1:  # prismatic
        return plucker(np.eye(3, dtype=np.result_type(qi, 1.0)), model["offset"][i] + qi * a)
    return plucker(axis_rotation(a, qi).T, model["offset"][i].astype(np.result_type(qi, 1.0)))


def motion_subspace(model, i):
    S = np.zeros(6)
    if model["jtype"][i] == 1:
        S[3:] = model["axis"][i]
    else:
        S[:3] = model["axis"][i]
    return S


def kinematics(model, q):
    """World-to-body transforms X0[i] (motion), body rotations R[i] (body axes
    in world coordinates) and origins p[i] (world)."""
    n = model["n"]
    X, X0, R, p = [], [], [], []
    for i in range(n):
        Xi = joint_transform(model, i, q[i])
        par = model["parent"][i]
        X.append(Xi)
        X0.append(Xi if par < 0 else Xi @ X0[par])
        if model["jtype"][i] == 1:
            Ri = np.eye(3, dtype=np.result_type(q, 1.0))
            off = model["offset"][i] + q[i] * model["axis"][i]
        else:
            Ri = axis_rotation(model["axis"][i], q[i])
            off = model["offset"][i]
        if par < 0:
            R.append(Ri)
            p.append(off.astype(np.result_type(q, 1.0)))
        else:
            R.append(R[par] @ Ri)
            p.append(p[par] + R[par] @ off)
    return X, X0, R, p


def foot_wrench_world(model, q, F):
    """The feet's wrenches as spatial forces at the world origin, per foot."""
    _, _, R, p = kinematics(model, q)
    nf, fd = len(model["foot_body"]), model["foot_dim"]
    out = []
    for f in range(nf):
        b = model["foot_body"][f]
        pt = p[b] + R[b] @ model["foot_offset"][f]
        force = F[f * fd:f * fd + 3]
        moment = F[f * fd + 3:f * fd + 6] if fd == 6 else np.zeros(3)
        out.append((b, np.concatenate([moment + np.cross(pt, force), force])))
    return out


def foot_jacobian(model, q, h: float = 1e-30):
    """The feet's velocity Jacobian in the world frame: per foot, the contact
    point's linear velocity (3 rows), then for 6D feet the foot body's angular
    velocity (3 rows), per unit generalised velocity ([n_feet*foot_dim][n]),
    by complex steps of the world poses along each coordinate (the coordinates
    are additive, so d/dq_j of a pose is its velocity for qd = e_j)."""
    n, fd = model["n"], model["foot_dim"]
    _, _, R, p = kinematics(model, q)
    J = np.zeros((len(model["foot_body"]) * fd, n))
    for j in range(n):
        _, _, Rc, pc = kinematics(model, q + 1j * h * np.eye(n)[j])
        for f, b in enumerate(model["foot_body"]):
            J[f * fd:f * fd + 3, j] = (pc[b] + Rc[b] @ model["foot_offset"][f]).imag / h
            if fd == 6:
                W = (Rc[b].imag / h) @ R[b].T
                J[f * fd + 3:f * fd + 6, j] = [W[2, 1], W[0, 2], W[1, 0]]
    return J


def noslip_rows(model, x):
    """The no-slip rows J_f v = 0 over the state x = (q, qd): zero on the
    positions, the feet's velocity Jacobian at q on the velocities."""
    n = model["n"]
    J = foot_jacobian(model, np.asarray(x[:n], dtype=float))
    return np.hstack([np.zeros_like(J), J])


def rnea(model, q, qd, qdd, F=None):
    """Inverse dynamics (Eq. (rnea)): M(q) qdd + h(q, qd) - J(q)' F."""
    n = model["n"]
    dt = np.result_type(q, qd, qdd, 1.0)
    X, X0, _, _ = kinematics(model, q)
    a_root = np.zeros(6, dtype=dt)
    a_root[5] = model["gravity"]  # gravity as an upward acceleration of the root
    v = [None] * n
    a = [None] * n
    f = [None] * n
    for i in range(n):
        S = motion_subspace(model, i)
        par = model["parent"][i]
        vp = np.zeros(6, dtype=dt) if par < 0 else v[par]
        ap = a_root if par < 0 else a[par]
        v[i] = X[i] @ vp + S * qd[i]
        a[i] = X[i] @ ap + S * qdd[i] + crm(v[i]) @ (S * qd[i])
        I = spatial_inertia(model["mass"][i], model["com"][i], np.diag(model["inertia"][i]))
        f[i] = I @ a[i] + crf(v[i]) @ (I @ v[i])
    if F is not None:
        for b, fw in foot_wrench_world(model, q, F):
            f[b] = f[b] - np.linalg.inv(X0[b]).T @ fw  # world force into body coordinates
    tau = np.zeros(n, dtype=dt)
    if "armature" in model:
        tau = tau + np.asarray(model["armature"]) * qdd
    for i in range(n - 1, -1, -1):
        tau[i] = tau[i] + motion_subspace(model, i) @ f[i]
        par = model["parent"][i]
        if par >= 0:
            f[par] = f[par] + X[i].T @ f[i]
    return tau


def mass_matrix(model, q):
    n = model["n"]
    z = np.zeros(n)
    g = rnea(model, q, z, z)
    M = np.zeros((n, n), dtype=np.result_type(q, 1.0))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        M[:, j] = rnea(model, q, z, e) - g
    return M


def forward_dynamics(model, q, qd, tau, F):
    """qdd = M(q)^-1 (S' tau + J' F - h(q, qd)) (tau: joint torques)."""
    n = model["n"]
    gen = np.zeros(n, dtype=np.result_type(tau, 1.0))
    gen[6:] = tau
    return np.linalg.solve(mass_matrix(model, q), gen - rnea(model, q, qd, np.zeros(n), F))


def step(model, x, u, dt):
    """Semi-implicit Euler step of Eq. (mpc_formulation) on x = (q, qd), u =
    (joint torques, foot wrenches)."""
    n, nj = model["n"], model["n_joints"]
    q, qd = x[:n], x[n:]
    qdd = forward_dynamics(model, q, qd, u[:nj], u[nj:])
    qd1 = qd + dt * qdd
    return np.concatenate([q + dt * qd1, qd1])


def linearize(model, x, u, dt, h: float = 1e-30):
    """A = df/dx, B = df/du by complex steps, c = f(x, u) - A x - B u."""
    nx, nu = len(x), len(u)
    A = np.zeros((nx, nx))
    B = np.zeros((nx, nu))
    for j in range(nx):
        xc = x.astype(complex)
        xc[j] += 1j * h
        A[:, j] = step(model, xc, u.astype(complex), dt).imag / h
    for j in range(nu):
        uc = u.astype(complex)
        uc[j] += 1j * h
        B[:, j] = step(model, x.astype(complex), uc, dt).imag / h
    c = step(model, x, u, dt) - A @ x - B @ u
    return A, B, c


def mpc_torque(model, tau_rnea, q_mpc, qd_mpc, q, qd, kp, kd):
    """Eq. (mpc_torque) for the joints (the last n_joints coordinates)."""
    j = slice(6, model["n"])
    return kp * (q_mpc[j] - q[j]) + kd * (qd_mpc[j] - qd[j]) + tau_rnea[j]
