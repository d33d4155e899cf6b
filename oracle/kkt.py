"""The paper's own inner solve, for the FP64 oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this module; the HIP product path never does.

The QP of each agent is put in OSQP's standard form and solved by OSQP's
iteration with the quasi-definite KKT matrix of Eq. (kkt_system) factored
once by LDL^T (Eq. (ldl)) and every iteration's linear system solved by
Eq. (backsolve_2) (forward substitution, diagonal scaling, backward
substitution), as Sec. III-B and Alg. 1 describe.  Unlike the rest of the
oracle, which keeps the dynamics rows exact, the dynamics here are ordinary
equality rows of the constraint matrix with the finite penalty
rho_eq_scale * rho (reading: OSQP's own treatment of equality rows).

Standard form (x_0 = xbar0 substituted into the first dynamics row):
  v = (x_1 .. x_N, u_0 .. u_{N-1}),  min 1/2 v'Pv + q'v,  l <= A v <= h,
  P = blkdiag(Q, .., Q, R, .., R),  q = (-Q r_1, .., -Q r_N, -R ubar_0, ..),
  rows of A: dynamics of stage k, x_{k+1} - A_k x_k - B_k u_k in
  [c_k, c_k] (c_0 + A_0 xbar0 at k = 0), then the input rows C_k u_k in
  [l_k, h_k] of the stage bounds.
Per-row penalty rho (OSQP's rule): equality rows rho_eq_scale * rho, rows
with both bounds infinite rho_min, others rho.

One OSQP iteration (Sec. 3.2 of the OSQP paper, relaxation alpha):
  [P + sigma I, A'; A, -diag(1/rho)] (xt, nu) = (sigma v - q, z - y/rho)
  zt = z + (nu - y) / rho
  v <- alpha xt + (1 - alpha) v
  z+ = clip(alpha zt + (1 - alpha) z + y/rho, l, h)
  y <- y + rho (alpha zt + (1 - alpha) z - z+),  z <- z+.
Cold start (reading, as the rest of the oracle): u = 0, x rolled out from
xbar0 under u = 0, z = A v (so the dynamics rows start at their bounds),
y = 0.  A warm start re-uses (v, z, y) as they are.

The LDL^T is taken of A_K under a symmetric permutation that interleaves
the unknowns stage by stage -- (u_k, the input rows of stage k, the dynamics
rows of stage k, x_{k+1}) for k = 0 .. N-1 -- so that the permuted matrix is
banded; the factorisation is the plain right-looking LDL^T without pivoting
(A_K is quasi-definite, so every leading minor is non-singular), restricted
to the band, which fill-in never leaves.
"""
from __future__ import annotations

from typing import Optional

import numpy as np
from scipy.linalg import solve_triangular

from . import Settings, constraint_matrix, stage_bounds


def standard_form(ag, settings: Optional[Settings] = None) -> dict:
    """P (diagonal, as a vector), q, A, l, h, rho of one agent (see above)."""
    st = settings or Settings.default()
    s = ag["s"]
    N, nx, nu = s.N, s.nx, s.nu
    C = constraint_matrix(s, ag["mu"])
    m = C.shape[0]
    lb, hb, _ = stage_bounds(s, ag["tau_max"], ag["stance"], st)
    nv = N * nx + N * nu
    xo = lambda k: (k - 1) * nx        # x_k, k = 1..N
    uo = lambda k: N * nx + k * nu     # u_k, k = 0..N-1
    Pd = np.concatenate([np.tile(ag["q"], N), np.tile(ag["r"], N)])
    q = np.zeros(nv)
    for k in range(1, N + 1):
        q[xo(k):xo(k) + nx] = -ag["q"] * ag["x_ref"][k]
    if ag.get("u_ref") is not None:
        for k in range(N):
            q[uo(k):uo(k) + nu] = -ag["r"] * ag["u_ref"][k]
    nrow = N * nx + N * m
    A = np.zeros((nrow, nv))
    lo = np.zeros(nrow)
    hi = np.zeros(nrow)
    for k in range(N):
        rws = slice(k * nx, (k + 1) * nx)
        A[rws, xo(k + 1):xo(k + 1) + nx] = np.eye(nx)
        if k >= 1:
            A[rws, xo(k):xo(k) + nx] = -ag["A"][k]
        A[rws, uo(k):uo(k) + nu] = -ag["B"][k]
        rhs = ag["c"][k] + (ag["A"][0] @ ag["x0"] if k == 0 else 0.0)
        lo[rws] = rhs
        hi[rws] = rhs
    for k in range(N):
        rws = slice(N * nx + k * m, N * nx + (k + 1) * m)
        A[rws, uo(k):uo(k) + nu] = C
        lo[rws] = lb[k]
        hi[rws] = hb[k]
    rho = np.where(lo == hi, st.rho_eq_scale * st.rho, st.rho)
    rho = np.where(np.isinf(lo) & np.isinf(hi), st.rho_min, rho)
    return dict(P=Pd, q=q, A=A, l=lo, h=hi, rho=rho, nv=nv, m=m)


def kkt_matrix(prob, sigma: float) -> np.ndarray:
    """A_K = [[P + sigma I, A'], [A, -diag(1/rho)]] of Eq. (kkt_system)."""
    nv, nr = prob["nv"], prob["A"].shape[0]
    K = np.zeros((nv + nr, nv + nr))
    K[:nv, :nv] = np.diag(prob["P"] + sigma)
    K[:nv, nv:] = prob["A"].T
    K[nv:, :nv] = prob["A"]
    K[nv:, nv:] = -np.diag(1.0 / prob["rho"])
    return K


def stage_order(s) -> np.ndarray:
    """The interleaving permutation of the KKT unknowns [v; nu]: for every
    stage k, u_k, the input rows of stage k, the dynamics rows of stage k,
    x_{k+1}."""
    N, nx, nu = s.N, s.nx, s.nu
    m = nu + 4 * s.n_feet
    nv = N * nx + N * nu
    order = []
    for k in range(N):
        order += list(range(N * nx + k * nu, N * nx + (k + 1) * nu))        # u_k
        order += list(range(nv + N * nx + k * m, nv + N * nx + (k + 1) * m))  # input rows
        order += list(range(nv + k * nx, nv + (k + 1) * nx))                # dynamics rows
        order += list(range(k * nx, (k + 1) * nx))                          # x_{k+1}
    return np.array(order)


def bandwidth(K: np.ndarray) -> int:
    i, j = np.nonzero(K)
    return int(np.abs(i - j).max()) if i.size else 0


def ldl(K: np.ndarray):
    """LDL^T of a symmetric matrix without pivoting (Eq. (ldl)): unit lower L
    and the diagonal d, column by column, each column's update confined to
    the band (the matrix has no entry outside it, and fill-in stays inside)."""
    n = K.shape[0]
    b = bandwidth(K)
    W = np.array(K, dtype=np.float64)
    L = np.eye(n)
    d = np.zeros(n)
    for j in range(n):
        d[j] = W[j, j]
        e = min(n, j + b + 1)
        col = W[j + 1:e, j] / d[j]
        L[j + 1:e, j] = col
        W[j + 1:e, j + 1:e] -= d[j] * np.outer(col, col)
    return L, d


def ldl_solve(L: np.ndarray, d: np.ndarray, rhs: np.ndarray) -> np.ndarray:
    """Eq. (backsolve_2): v = L^-T D^-1 L^-1 b (forward substitution, diagonal
    scaling, backward substitution)."""
    w = solve_triangular(L, rhs, lower=True, unit_diagonal=True)
    w = w / d
    return solve_triangular(L.T, w, lower=False, unit_diagonal=True)


class Factor:
    """The factorised KKT system of one agent: A_K permuted to the stage
    order, factored once; ``solve`` maps a right-hand side in the natural
    order to the solution in the natural order."""

    def __init__(self, prob, sigma: float, s):
        self.K = kkt_matrix(prob, sigma)
        self.perm = stage_order(s)
        Kp = self.K[np.ix_(self.perm, self.perm)]
        self.L, self.d = ldl(Kp)

    def solve(self, rhs: np.ndarray) -> np.ndarray:
        out = np.empty_like(rhs)
        out[self.perm] = ldl_solve(self.L, self.d, rhs[self.perm])
        return out


def cold_start(ag, prob) -> tuple:
    """u = 0, x rolled out from xbar0, z = A v, y = 0."""
    s = ag["s"]
    N, nx = s.N, s.nx
    x = np.zeros((N + 1, nx))
    x[0] = ag["x0"]
    for k in range(N):
        x[k + 1] = ag["A"][k] @ x[k] + ag["c"][k]
    v = np.concatenate([x[1:].ravel(), np.zeros(N * s.nu)])
    return v, prob["A"] @ v, np.zeros(prob["A"].shape[0])


def solve(ag, *, iters: int = 50, warm=None, settings: Optional[Settings] = None,
          tol: float = 0.0) -> dict:
    """OSQP on the standard form with the LDL^T-factored KKT system: ``iters``
    iterations (with ``tol`` > 0, stop early once the primal and dual
    residuals |Av - z|, |Pv + q + A'y| are below tol).  ``warm``: (v, z, y)
    from a previous solve.  Returns x [N+1, nx] (x_0 = xbar0), u [N, nu], the
    input rows' z, y [N, m], the dynamics rows' zd, yd [N, nx], v, the full
    z and y, and the iteration count."""
    st = settings or Settings.default()
    s = ag["s"]
    N, nx, nu = s.N, s.nx, s.nu
    prob = standard_form(ag, st)
    fac = Factor(prob, st.sigma, s)
    if warm is None:
        v, z, y = cold_start(ag, prob)
    else:
        v, z, y = (np.array(w, dtype=np.float64) for w in warm)
    A, rho, lo, hi = prob["A"], prob["rho"], prob["l"], prob["h"]
    nv = prob["nv"]
    alpha = st.alpha
    it = 0
    for it in range(1, iters + 1):
        sol = fac.solve(np.concatenate([st.sigma * v - prob["q"], z - y / rho]))
        xt, nuk = sol[:nv], sol[nv:]
        zt = z + (nuk - y) / rho
        v = alpha * xt + (1.0 - alpha) * v
        w = alpha * zt + (1.0 - alpha) * z
        zn = np.clip(w + y / rho, lo, hi)
        y = y + rho * (w - zn)
        z = zn
        if tol > 0:
            rp = np.abs(A @ v - z).max()
            rd = np.abs(prob["P"] * v + prob["q"] + A.T @ y).max()
            if rp < tol and rd < tol:
                break
    x = np.vstack([ag["x0"][None, :], v[:N * nx].reshape(N, nx)])
    u = v[N * nx:].reshape(N, nu)
    m = prob["m"]
    return dict(x=x, u=u, z=z[N * nx:].reshape(N, m), y=y[N * nx:].reshape(N, m),
                zd=z[:N * nx].reshape(N, nx), yd=y[:N * nx].reshape(N, nx), v=v, z_all=z, y_all=y,
                iters=it)


def solve_batch(batch, *, iters: int = 50, warm=None, x0=None, settings: Optional[Settings] = None
                ) -> dict:
    """``solve`` for every agent of a ``synth.Batch``, flat layouts as the rest
    of the oracle (x, u, z, y; zd, yd with N nx per agent).  ``warm``: dict of
    flat u, z, y, zd, yd and x (x_0 included, N+1 states per agent)."""
    from . import agent as agent_of
    o = batch.offsets()
    outs = []
    for a in range(batch.n_agents):
        ag = agent_of(batch, a)
        s = ag["s"]
        if x0 is not None:
            ag["x0"] = np.asarray(x0[o["x0"][a]:o["x0"][a + 1]], dtype=np.float64)
        w = None
        if warm is not None:
            N, nx, nu, m = s.N, s.nx, s.nu, s.nu + 4 * s.n_feet
            xa = np.asarray(warm["x"][o["x"][a]:o["x"][a + 1]], dtype=np.float64)[nx:]
            ua = np.asarray(warm["u"][o["u"][a]:o["u"][a + 1]], dtype=np.float64)
            za = np.asarray(warm["z"][o["z"][a]:o["z"][a + 1]], dtype=np.float64)
            ya = np.asarray(warm["y"][o["z"][a]:o["z"][a + 1]], dtype=np.float64)
            zda = np.asarray(warm["zd"][o["c"][a]:o["c"][a + 1]], dtype=np.float64)
            yda = np.asarray(warm["yd"][o["c"][a]:o["c"][a + 1]], dtype=np.float64)
            w = (np.concatenate([xa, ua]), np.concatenate([zda, za]), np.concatenate([yda, ya]))
        outs.append(solve(ag, iters=iters, warm=w, settings=settings))
    cat = lambda k: np.concatenate([np.ravel(r[k]) for r in outs])
    return dict(x=cat("x"), u=cat("u"), z=cat("z"), y=cat("y"), zd=cat("zd"), yd=cat("yd"))
