"""Seeded synthetic MPC QP batches.

This module only draws inputs: per-stage dynamics (A_k, B_k, c_k), diagonal
cost weights, torque limits, friction coefficients, contact schedules,
initial states and references.  It contains none of the solver's arithmetic
(no bounds, penalties, factorisations or iterations), so both the FP64 CPU
oracle and the HIP path can consume the same problems.

The problem class is the linearised whole-body MPC QP of the paper's MPC
formulation (Sec. III-A, Eq. (mpc_formulation)) under real-time iteration
(Sec. III-B): one QP per agent per control step, with a floating-base state
of 48 entries, foot contact wrenches/forces, a torque box, unilateral contact
and a friction pyramid.  The robot model itself is not available, so the
stage matrices are random with the documented distributions.

Random streams: every agent owns a PCG64 stream seeded with
``SeedSequence([seed, stream_id, agent_id])``; per-step disturbances use
``SeedSequence([seed, stream_id, agent_id, 1_000_000 + step])``.  Any agent
subset therefore reproduces exactly.

Layout (all arrays row-major, agents concatenated in agent order, so a
uniform batch is the plain [B][N][...] tensor):
  A      [sum_a N_a*nx_a*nx_a]     B  [sum_a N_a*nx_a*nu_a]
  c      [sum_a N_a*nx_a]          q  [sum_a nx_a]    r [sum_a nu_a]
  x_ref  [sum_a (N_a+1)*nx_a]      x0 [sum_a nx_a]
  tau_max[sum_a n_tau_a]           mu [n_agents]
  stance [sum_a N_a*n_feet_a] (uint8, 1 = foot in stance)
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np

DT = 0.01


@dataclasses.dataclass(frozen=True)
class Shape:
    """Per-agent problem shape.

    ``u = [tau (n_tau); w_1; ...; w_{n_feet}]`` with ``w`` a 6D wrench
    (f_x, f_y, f_z, m_x, m_y, m_z) when ``foot_dim == 6`` or a 3D force when
    ``foot_dim == 3``.  ``nu == n_tau + n_feet * foot_dim``.
    """

    N: int
    nx: int
    nu: int
    n_tau: int
    n_feet: int
    foot_dim: int

    def __post_init__(self):
        if self.nu != self.n_tau + self.n_feet * self.foot_dim:
            raise ValueError("nu must equal n_tau + n_feet*foot_dim")
        if self.foot_dim not in (3, 6):
            raise ValueError("foot_dim must be 3 or 6")

    @property
    def m(self) -> int:
        """Constraint rows per stage: identity rows on u plus 4 pyramid rows per foot."""
        return self.nu + 4 * self.n_feet

    def as_tuple(self):
        return (self.N, self.nx, self.nu, self.n_tau, self.n_feet, self.foot_dim)


def humanoid(N: int = 10) -> Shape:
    """24-DoF floating-base humanoid: q, v (48), 18 torques + two 6D foot wrenches."""
    return Shape(N=N, nx=48, nu=30, n_tau=18, n_feet=2, foot_dim=6)


def quadruped(N: int = 10) -> Shape:
    """Quadruped-shaped agent: 36 states, 12 torques + four 3D foot forces."""
    return Shape(N=N, nx=36, nu=24, n_tau=12, n_feet=4, foot_dim=3)


def agent_rng(seed: int, stream_id: int, agent_id: int, *extra: int) -> np.random.Generator:
    return np.random.Generator(
        np.random.PCG64(np.random.SeedSequence([seed, stream_id, agent_id, *extra])))


@dataclasses.dataclass
class Batch:
    """A batch of agents' raw QP data (see module docstring for the layout)."""

    shapes: List[Shape]
    A: np.ndarray
    B: np.ndarray
    c: np.ndarray
    q: np.ndarray
    r: np.ndarray
    x_ref: np.ndarray
    x0: np.ndarray
    tau_max: np.ndarray
    mu: np.ndarray
    stance: np.ndarray
    seed: int = 0
    stream_id: int = 0
    agent_ids: Optional[np.ndarray] = None

    @property
    def n_agents(self) -> int:
        return len(self.shapes)

    @property
    def uniform(self) -> bool:
        return len(set(self.shapes)) <= 1

    def offsets(self) -> dict:
        """Start offset of each agent in each flat array (int64, length n_agents+1)."""
        return compute_offsets(self.shapes)

    def astype(self, dtype) -> "Batch":
        f = lambda a: np.ascontiguousarray(a, dtype=dtype)
        return dataclasses.replace(self, A=f(self.A), B=f(self.B), c=f(self.c), q=f(self.q),
                                   r=f(self.r), x_ref=f(self.x_ref), x0=f(self.x0),
                                   tau_max=f(self.tau_max), mu=f(self.mu))

    def subset(self, idx: Sequence[int]) -> "Batch":
        """Agents ``idx`` (in that order) as a new batch."""
        off = self.offsets()
        parts = {k: [] for k in ("A", "B", "c", "q", "r", "x_ref", "x0", "tau_max", "stance")}
        for a in idx:
            for k in parts:
                parts[k].append(getattr(self, k)[off[k][a]:off[k][a + 1]])
        ids = self.agent_ids if self.agent_ids is not None else np.arange(self.n_agents)
        return Batch(shapes=[self.shapes[a] for a in idx],
                     mu=np.ascontiguousarray(self.mu[list(idx)]),
                     seed=self.seed, stream_id=self.stream_id,
                     agent_ids=np.asarray([ids[a] for a in idx], dtype=np.int64),
                     **{k: np.ascontiguousarray(np.concatenate(v)) for k, v in parts.items()})


_FIELDS = {
    "A": lambda s: s.N * s.nx * s.nx,
    "B": lambda s: s.N * s.nx * s.nu,
    "c": lambda s: s.N * s.nx,
    "q": lambda s: s.nx,
    "r": lambda s: s.nu,
    "x_ref": lambda s: (s.N + 1) * s.nx,
    "x0": lambda s: s.nx,
    "tau_max": lambda s: s.n_tau,
    "stance": lambda s: s.N * s.n_feet,
    # solution-side arrays (used by bindings and tests)
    "x": lambda s: (s.N + 1) * s.nx,
    "u": lambda s: s.N * s.nu,
    "z": lambda s: s.N * s.m,
    "u0": lambda s: s.nu,
}


def compute_offsets(shapes: Sequence[Shape]) -> dict:
    out = {}
    for k, f in _FIELDS.items():
        sizes = np.fromiter((f(s) for s in shapes), dtype=np.int64, count=len(shapes))
        o = np.zeros(len(shapes) + 1, dtype=np.int64)
        np.cumsum(sizes, out=o[1:])
        out[k] = o
    return out


def _draw_agent(rng, s: Shape, *, stance_p, q_log, r_log, r_scale, dt=DT):
    """Draw one agent's data in a fixed order: A, B, c, q, r, tau_max, mu, the
    per-foot stance probabilities, stance, x0, x_ref."""
    G = rng.standard_normal((s.N, s.nx, s.nx)) / np.sqrt(s.nx)
    A = G * dt
    A[:, np.arange(s.nx), np.arange(s.nx)] += 1.0
    B = rng.standard_normal((s.N, s.nx, s.nu)) * (dt / np.sqrt(s.nu))
    c = rng.standard_normal((s.N, s.nx)) * 1e-3
    q = 10.0 ** rng.uniform(q_log[0], q_log[1], s.nx)
    r = r_scale * 10.0 ** rng.uniform(r_log[0], r_log[1], s.nu)
    tau_max = rng.uniform(20.0, 100.0, s.n_tau)
    mu = rng.uniform(0.4, 1.0)
    if stance_p is None:  # per-foot stance probability ~ U[0.3, 0.9]
        p = rng.uniform(0.3, 0.9, s.n_feet)
    else:
        p = np.full(s.n_feet, stance_p)
    stance = (rng.random((s.N, s.n_feet)) < p[None, :]).astype(np.uint8)
    x0 = rng.standard_normal(s.nx)
    x_ref = rng.standard_normal((s.N + 1, s.nx))
    return A, B, c, q, r, x_ref, x0, tau_max, mu, stance


def make_batch(shapes: Sequence[Shape], *, seed: int = 0, stream_id: int = 0,
               agent_ids: Optional[Sequence[int]] = None, stance_p: Optional[float] = 0.6,
               q_log=(-2.0, 2.0), r_log=(-4.0, -1.0), r_scale: float = 1.0,
               dtype=np.float64) -> Batch:
    """Draw a batch; agent ``i`` uses stream (seed, stream_id, agent_ids[i])."""
    shapes = list(shapes)
    if agent_ids is None:
        agent_ids = range(len(shapes))
    agent_ids = np.asarray(list(agent_ids), dtype=np.int64)
    off = compute_offsets(shapes)
    out = {k: np.empty(int(off[k][-1]), dtype=dtype)
           for k in ("A", "B", "c", "q", "r", "x_ref", "x0", "tau_max")}
    stance = np.empty(int(off["stance"][-1]), dtype=np.uint8)
    mu = np.empty(len(shapes), dtype=dtype)
    for i, (s, aid) in enumerate(zip(shapes, agent_ids)):
        rng = agent_rng(seed, stream_id, int(aid))
        A, B, c, q, r, x_ref, x0, tau_max, m_, st = _draw_agent(
            rng, s, stance_p=stance_p, q_log=q_log, r_log=r_log, r_scale=r_scale)
        for k, v in (("A", A), ("B", B), ("c", c), ("q", q), ("r", r), ("x_ref", x_ref),
                     ("x0", x0), ("tau_max", tau_max)):
            out[k][off[k][i]:off[k][i + 1]] = v.ravel()
        stance[off["stance"][i]:off["stance"][i + 1]] = st.ravel()
        mu[i] = m_
    return Batch(shapes=shapes, stance=stance, mu=mu, seed=seed, stream_id=stream_id,
                 agent_ids=agent_ids, **out)


# --- the five benchmark configurations -------------------------------------------------

def small_humanoid_batch(n_agents: int = 64, seed: int = 0, agent_ids=None, dtype=np.float64) -> Batch:
    """64 humanoid agents, N=10, stance Bernoulli(0.6), solved in FP64 for 50 iterations."""
    ids = range(n_agents) if agent_ids is None else agent_ids
    return make_batch([humanoid(10)] * len(list(ids)), seed=seed, stream_id=0,
                      agent_ids=ids, dtype=dtype)


def humanoid_batch(n_agents: int = 4096, seed: int = 0, agent_ids=None, dtype=np.float64) -> Batch:
    """RL-training shape: the small batch's generator at 4096 humanoid agents, N=10."""
    ids = range(n_agents) if agent_ids is None else agent_ids
    return make_batch([humanoid(10)] * len(list(ids)), seed=seed, stream_id=1,
                      agent_ids=ids, dtype=dtype)


def uneven_batch_shapes(n_agents: int = 8192, seed: int = 0, stream_id: int = 2,
                   agent_ids=None) -> List[Shape]:
    """Uneven batch: N ~ U{5..20}, 50/50 humanoid / quadruped, from a per-agent stream."""
    ids = range(n_agents) if agent_ids is None else agent_ids
    shapes = []
    for aid in ids:
        rng = agent_rng(seed, stream_id, int(aid), 7)
        kind = rng.integers(0, 2)
        N = int(rng.integers(5, 21))
        shapes.append(humanoid(N) if kind == 0 else quadruped(N))
    return shapes


def uneven_batch(n_agents: int = 8192, seed: int = 0, agent_ids=None, dtype=np.float64,
            stream_id: int = 2) -> Batch:
    ids = list(range(n_agents) if agent_ids is None else agent_ids)
    shapes = uneven_batch_shapes(seed=seed, stream_id=stream_id, agent_ids=ids)
    return make_batch(shapes, seed=seed, stream_id=stream_id, agent_ids=ids,
                      stance_p=None, dtype=dtype)


def conditioned_humanoid_batch(n_agents: int = 16384, kappa: float = 1e4, seed: int = 0, agent_ids=None,
            dtype=np.float64) -> Batch:
    """Mixed-precision sweep: humanoid N=16, Q and R with condition number ``kappa``.

    Q = diag(10^U[-h, h]) and R = 3.16e-3 * diag(10^U[-h, h]) with h = log10(kappa)/2,
    centred on the geometric means of the small humanoid batch's draws (1 and 10^-2.5).
    """
    ids = range(n_agents) if agent_ids is None else agent_ids
    h = 0.5 * np.log10(kappa)
    cid = 300 + int(round(np.log10(kappa)))
    return make_batch([humanoid(16)] * len(list(ids)), seed=seed, stream_id=cid,
                      agent_ids=ids, q_log=(-h, h), r_log=(-h, h), r_scale=10 ** -2.5,
                      dtype=dtype)


def joint_limits(batch: Batch, seed: int = 0):
    """Joint position and velocity limits (Eq. (mpc_formulation)), flat, nx per
    agent: the state is (q, v) of a floating base (6 coordinates) plus joints,
    so components 6 .. nx/2 - 1 (positions) and nx/2 + 6 .. nx - 1 (velocities)
    get a box, drawn per agent and component (positions +-U[1, 2], velocities
    +-U[1.5, 3]) and widened to hold the agent's x0 with a margin of 0.3;
    the base components are free (+-inf).  Own stream per agent (extra key
    2_000_000), so the problem draws are untouched."""
    ids = batch.agent_ids if batch.agent_ids is not None else np.arange(batch.n_agents)
    off = batch.offsets()
    lo_all, hi_all = [], []
    for a, (s, aid) in enumerate(zip(batch.shapes, ids)):
        rng = agent_rng(seed, batch.stream_id, int(aid), 2_000_000)
        half = s.nx // 2
        lo = np.full(s.nx, -np.inf)
        hi = np.full(s.nx, np.inf)
        for base, (wlo, whi) in ((0, (1.0, 2.0)), (half, (1.5, 3.0))):
            j = np.arange(base + 6, base + half)
            lo[j] = -rng.uniform(wlo, whi, j.size)
            hi[j] = rng.uniform(wlo, whi, j.size)
        x0 = np.asarray(batch.x0[off["x0"][a]:off["x0"][a + 1]], dtype=np.float64)
        lim = np.isfinite(lo)
        lo[lim] = np.minimum(lo[lim], x0[lim] - 0.3)
        hi[lim] = np.maximum(hi[lim], x0[lim] + 0.3)
        lo_all.append(lo)
        hi_all.append(hi)
    dt = batch.A.dtype
    return np.concatenate(lo_all).astype(dt), np.concatenate(hi_all).astype(dt)


def foot_jacobians(batch: Batch, seed: int = 0):
    """Velocity Jacobians of the feet for the no-slip rows J_f v = 0 of
    Eq. (mpc_formulation), flat, n_feet * foot_dim rows of nx columns per
    agent (row-major): the state is (q, v) of a floating base plus joints, so
    the position half is zero; each foot's rows act on the base twist
    (columns nx/2 .. nx/2 + 5, entries N(0, 1/4)) and on the joints of its own
    leg (the joints split into n_feet consecutive blocks, entries N(0, 1)).
    The Jacobian at the linearisation point, the same at every stage.  Own
    stream per agent (extra key 3_000_000)."""
    ids = batch.agent_ids if batch.agent_ids is not None else np.arange(batch.n_agents)
    out = []
    for s, aid in zip(batch.shapes, ids):
        rng = agent_rng(seed, batch.stream_id, int(aid), 3_000_000)
        half = s.nx // 2
        nj = half - 6
        J = np.zeros((s.n_feet * s.foot_dim, s.nx))
        for f in range(s.n_feet):
            rows = slice(f * s.foot_dim, (f + 1) * s.foot_dim)
            J[rows, half:half + 6] = 0.5 * rng.standard_normal((s.foot_dim, 6))
            j0, j1 = half + 6 + f * nj // s.n_feet, half + 6 + (f + 1) * nj // s.n_feet
            J[rows, j0:j1] = rng.standard_normal((s.foot_dim, j1 - j0))
        out.append(J.ravel())
    dt = batch.A.dtype
    if not out:
        return np.zeros(0, dtype=dt)
    return np.concatenate(out).astype(dt)


def step_noise(batch: Batch, step: int, std: float = 1e-2) -> np.ndarray:
    """Per-step state disturbance, N(0, std^2), laid out like ``x0``."""
    ids = batch.agent_ids if batch.agent_ids is not None else np.arange(batch.n_agents)
    parts = []
    for s, aid in zip(batch.shapes, ids):
        rng = agent_rng(batch.seed, batch.stream_id, int(aid), 1_000_000 + step)
        parts.append(rng.standard_normal(s.nx) * std)
    return np.concatenate(parts)


# ------------------------------------------------------------------------------
# Synthetic articulated models (the front and back end of the real-time
# iteration need a robot model; the paper's MIT Humanoid is not available, so a
# tree of the same size stands in).  Only parameters are drawn here.
# ------------------------------------------------------------------------------

JOINT_REVOLUTE, JOINT_PRISMATIC = 0, 1


def _limb(parent, joints, rng, mass, length, first_offset):
    """Bodies of one limb: (parent, joint type, axis, offset of the joint in the
    parent frame, mass, centre of mass, principal inertia)."""
    out = []
    for i, ax in enumerate(joints):
        off = np.array(first_offset if i == 0 else [0.0, 0.0, -length[i - 1]])
        m = mass[i] * rng.uniform(0.8, 1.2)
        ln = length[i] if i < len(length) else 0.05
        com = np.array([rng.uniform(-0.01, 0.01), rng.uniform(-0.01, 0.01), -0.5 * ln])
        rad = 0.04 * rng.uniform(0.8, 1.2)
        ic = m * np.array([(3 * rad ** 2 + ln ** 2) / 12, (3 * rad ** 2 + ln ** 2) / 12, rad ** 2 / 2])
        out.append((parent, JOINT_REVOLUTE, np.eye(3)[ax], off, m, com, ic))
        parent = None  # the next joint hangs from this body
    return out


def articulated_model(kind: str = "humanoid", seed: int = 0) -> dict:
    """A floating-base tree with the size of the humanoid (18 joints: two legs
    of hip yaw/roll/pitch, knee, ankle; two arms of shoulder pitch/roll/yaw,
    elbow) or of the quadruped (4 legs of hip abduction/flexion, knee).  The
    floating base is a chain of three prismatic joints along the world axes and
    three revolute joints z, y, x (yaw, pitch, roll) carrying the base body, so
    the generalised coordinates are additive (q = base position, ZYX angles,
    joint angles; qd their rates).  Returns per body: parent (-1 for the first),
    joint type, joint axis (joint frame), the joint frame's offset in the
    parent frame (rotation identity), mass, centre of mass and principal
    inertia (body frame), and the armature: the reflected inertia of the
    joint's geared actuator, U(0.01, 0.05) kg m^2 per actuated joint (0 for the
    six base coordinates), which adds to the mass matrix's diagonal; per foot:
    its body and the contact point's offset in that body's frame; foot_dim (6:
    force and moment, 3: force)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 4_000_000, 0 if kind == "humanoid" else 1])))
    bodies = []
    # virtual base joints: x, y, z translation, then z, y, x rotation; massless
    for ax in range(3):
        bodies.append((len(bodies) - 1, JOINT_PRISMATIC, np.eye(3)[ax], np.zeros(3), 0.0, np.zeros(3), np.zeros(3)))
    for ax in (2, 1, 0):
        bodies.append((len(bodies) - 1, JOINT_REVOLUTE, np.eye(3)[ax], np.zeros(3), 0.0, np.zeros(3), np.zeros(3)))
    base = len(bodies) - 1  # the roll joint's body is the base
    if kind == "humanoid":
        mb = 12.0 * rng.uniform(0.9, 1.1)
        bodies[base] = bodies[base][:4] + (mb, np.array([0.0, 0.0, 0.1]), mb * np.array([0.12, 0.10, 0.05]))
        feet = []
        for side in (1.0, -1.0):
            leg = _limb(base, [2, 0, 1, 1, 1], rng, [1.0, 1.0, 3.0, 2.0, 0.6], [0.05, 0.05, 0.30, 0.30, 0.05],
                        [0.0, 0.09 * side, -0.05])
            first = len(bodies)
            for i, b in enumerate(leg):
                bodies.append(((first + i - 1) if i else base,) + b[1:])
            feet.append((len(bodies) - 1, np.array([0.03, 0.0, -0.05])))
        for side in (1.0, -1.0):
            arm = _limb(base, [1, 0, 2, 1], rng, [0.8, 0.8, 1.0, 0.6], [0.05, 0.05, 0.25, 0.25],
                        [0.0, 0.17 * side, 0.35])
            first = len(bodies)
            for i, b in enumerate(arm):
                bodies.append(((first + i - 1) if i else base,) + b[1:])
        foot_dim = 6
    else:
        mb = 9.0 * rng.uniform(0.9, 1.1)
        bodies[base] = bodies[base][:4] + (mb, np.zeros(3), mb * np.array([0.04, 0.10, 0.12]))
        feet = []
        for sx in (1.0, -1.0):
            for sy in (1.0, -1.0):
                leg = _limb(base, [0, 1, 1], rng, [0.6, 1.2, 0.3], [0.08, 0.21, 0.21],
                            [0.19 * sx, 0.05 * sy, 0.0])
                first = len(bodies)
                for i, b in enumerate(leg):
                    bodies.append(((first + i - 1) if i else base,) + b[1:])
                feet.append((len(bodies) - 1, np.array([0.0, 0.0, -0.21])))
        foot_dim = 3
    nb = len(bodies)
    arng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(
        [seed, 4_000_001, 0 if kind == "humanoid" else 1])))
    armature = np.concatenate([np.zeros(6), arng.uniform(0.01, 0.05, nb - 6)])
    return dict(
        kind=kind, n=nb, n_joints=nb - 6, gravity=9.81,
        parent=np.array([b[0] for b in bodies], dtype=np.int32),
        jtype=np.array([b[1] for b in bodies], dtype=np.int32),
        axis=np.array([b[2] for b in bodies]), offset=np.array([b[3] for b in bodies]),
        mass=np.array([b[4] for b in bodies]), com=np.array([b[5] for b in bodies]),
        inertia=np.array([b[6] for b in bodies]), armature=armature,
        foot_body=np.array([f[0] for f in feet], dtype=np.int32), foot_offset=np.array([f[1] for f in feet]),
        foot_dim=foot_dim)


def model_states(model: dict, n: int, seed: int = 0, dt: float = 0.02):
    """n seeded configurations near a standing pose for the model: q (base
    height 0.6 m, small base angles, joint angles N(0, 0.2)), qd N(0, 0.3),
    qdd N(0, 1), joint torques N(0, 5) and foot forces (vertical ~ weight per
    foot, tangential within the friction cone; moments N(0, 0.5) for 6D)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 4_100_000])))
    nq = model["n"]
    nf, fd = len(model["foot_body"]), model["foot_dim"]
    q = np.zeros((n, nq))
    q[:, 0:2] = rng.uniform(-0.5, 0.5, (n, 2))
    q[:, 2] = 0.6 + rng.uniform(-0.05, 0.05, n)
    q[:, 3:6] = rng.normal(0, 0.1, (n, 3))
    q[:, 6:] = rng.normal(0, 0.2, (n, nq - 6))
    qd = rng.normal(0, 0.3, (n, nq))
    qdd = rng.normal(0, 1.0, (n, nq))
    tau = rng.normal(0, 5.0, (n, nq - 6))
    w = model["mass"].sum() * model["gravity"] / nf
    F = np.zeros((n, nf, fd))
    F[:, :, 2] = w * rng.uniform(0.5, 1.5, (n, nf))
    F[:, :, :2] = rng.uniform(-0.3, 0.3, (n, nf, 2)) * F[:, :, 2:3]
    if fd == 6:
        F[:, :, 3:] = rng.normal(0, 0.5, (n, nf, 3))
    return dict(q=q, qd=qd, qdd=qdd, tau=tau, F=F.reshape(n, nf * fd), dt=dt)
