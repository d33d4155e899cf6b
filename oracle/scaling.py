"""Ruiz equilibration and adaptive rho for the FP64 oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this module; the HIP product path never does.

Alg. 1 scales the KKT system with Ruiz equilibration (f_Ruiz) before the
factorisation, and the paper's QP iterations are OSQP's (Sec. III-B), whose
step-size rule rescales rho from the ratio of the primal and dual residuals.
This module writes both out for one agent, plainly and in the order of those
descriptions, on the dense stacked QP (variables x_1..x_N, u_0..u_{N-1};
dynamics rows x_{k+1} - A_k x_k - B_k u_k = c_k; constraint rows C_k u_k):

* ``ruiz``: iterated equilibration of the KKT matrix [[P, A'], [A, 0]] --
  every primal column and every dynamics row is divided by the square root of
  its infinity norm (norms below 1e-4 count as 1, above 1e4 as 1e4), then the
  cost is divided by max(mean column norm of P, |q|_inf) under the same
  limits.  Readings (the solver's structure has to survive the scaling):
  a state component has one scale for every stage (Q is stage invariant), an
  input component likewise, the x and y forces of every foot share one scale
  and each other force or moment component one scale over the feet (one
  friction coefficient per agent); the dynamics rows have a scale per state
  component; a constraint row's scale is fixed by its input scales (identity
  rows 1 / d_j, pyramid facets 1 / d_fxy) so that the scaled rows are again
  [I; pyramid] with the friction coefficient mu d_fz / d_fxy.  The column
  norms run over the whole KKT column (its P, dynamics and constraint
  entries); tied groups take the largest norm of their members.
* ``scale_agent`` / ``scale_state`` / ``unscale_state``: the scaled problem
  (A_k -> D^-1 A_k D, B_k -> D^-1 B_k D_u, c_k -> D^-1 c_k, Q -> c D Q D,
  R -> c D_u R D_u, x_ref and x0 -> D^-1, tau_max -> tau_max / d_tau) and the
  change of variables of the iterate (x = D x^, u = D_u u^, z = E^-1 z^,
  y = E y^ / c).
* ``rho_estimate``: OSQP's rule rho sqrt((|r_prim| / max(|Cu|, |z|)) /
  (|r_dual| / max(|Px|, |C'y|, |q|))) on the scaled problem, clipped to
  [1e-6, 1e6] and rounded to the nearest power of 2^(1/4) (reading: a grid
  keeps the update from hinging on the last bits of the residuals).
* ``solve``: Ruiz, then the QP iterations in segments of ``rho_interval``
  (the oracle's own fixed-iteration solve, warm-started from the previous
  segment), with rho replaced by its estimate between segments when it moved
  by more than ``rho_tolerance`` either way, then the iterate unscaled.
"""
from __future__ import annotations

from typing import Optional

import numpy as np

from . import Settings, constraint_matrix, residuals, rows
from . import solve as solve_unscaled

MIN_SCALING, MAX_SCALING = 1e-4, 1e4
RHO_MIN, RHO_MAX = 1e-6, 1e6


def input_groups(s) -> np.ndarray:
    """Scale group of every input component: torques one each; foot forces and
    moments one per component over the feet, with f_x and f_y together."""
    g = np.arange(s.nu)
    for f in range(s.n_feet):
        for c in range(s.foot_dim):
            j = s.n_tau + f * s.foot_dim + c
            g[j] = s.n_tau + (0 if c == 1 else c)  # f_y joins f_x; feet share
    return g


def stacked(ag):
    """Dense stacked QP of one agent: P (diagonal, as a vector), q, the
    dynamics rows Aeq and the constraint rows Cs (over x_1..x_N, u_0..u_{N-1})."""
    s = ag["s"]
    N, nx, nu = s.N, s.nx, s.nu
    m = rows(s)
    n = N * nx + N * nu
    xi = lambda k: N * 0 + (k - 1) * nx  # x_k, k >= 1
    ui = lambda k: N * nx + k * nu
    P = np.concatenate([np.tile(ag["q"], N), np.tile(ag["r"], N)])
    q = np.concatenate([-(ag["q"] * ag["x_ref"][1:]).ravel(), np.zeros(N * nu)])
    Aeq = np.zeros((N * nx, n))
    for k in range(N):
        r0 = k * nx
        Aeq[r0:r0 + nx, xi(k + 1):xi(k + 1) + nx] = np.eye(nx)
        if k >= 1:
            Aeq[r0:r0 + nx, xi(k):xi(k) + nx] = -ag["A"][k]
        Aeq[r0:r0 + nx, ui(k):ui(k) + nu] = -ag["B"][k]
    C = constraint_matrix(s, ag["mu"])
    Cs = np.zeros((N * m, n))
    for k in range(N):
        Cs[k * m:(k + 1) * m, ui(k):ui(k) + nu] = C
    return P, q, Aeq, Cs


def _limit(v):
    v = np.array(v, dtype=np.float64)
    v[v < MIN_SCALING] = 1.0
    return np.minimum(v, MAX_SCALING)


def row_scales(s, Du):
    """Scale of every constraint row of one stage, fixed by the input scales."""
    m = rows(s)
    e = np.empty(m)
    e[:s.nu] = 1.0 / Du
    for f in range(s.n_feet):
        e[s.nu + 4 * f:s.nu + 4 * f + 4] = 1.0 / Du[s.n_tau + f * s.foot_dim]
    return e


def ruiz(ag, iters: int = 10) -> dict:
    """Scale factors (Dx [nx], Du [nu], Ed [nx], cost c) after ``iters`` rounds."""
    s = ag["s"]
    N, nx, nu = s.N, s.nx, s.nu
    P, q, Aeq, Cs = stacked(ag)
    grp = input_groups(s)
    Dx, Du, Ed, c = np.ones(nx), np.ones(nu), np.ones(nx), 1.0
    for _ in range(iters):
        d = np.concatenate([np.tile(Dx, N), np.tile(Du, N)])
        ed = np.tile(Ed, N)
        ec = np.tile(row_scales(s, Du), N)
        Ph = c * d * d * P
        Ah = np.abs(Aeq) * ed[:, None] * d[None, :]
        Ch = np.abs(Cs) * ec[:, None] * d[None, :]
        col = np.maximum(np.abs(Ph), np.maximum(Ah.max(axis=0), Ch.max(axis=0)))
        drow = Ah.max(axis=1)
        # tied groups take the largest norm of their members
        cx = col[:N * nx].reshape(N, nx).max(axis=0)
        cu_stage = col[N * nx:].reshape(N, nu).max(axis=0)
        cu = np.array([cu_stage[grp == grp[j]].max() for j in range(nu)])
        ce = drow.reshape(N, nx).max(axis=0)
        Dx = Dx / np.sqrt(_limit(cx))
        Du = Du / np.sqrt(_limit(cu))
        Ed = Ed / np.sqrt(_limit(ce))
        # cost normalisation
        d = np.concatenate([np.tile(Dx, N), np.tile(Du, N)])
        pn = np.abs(c * d * d * P).mean()
        qn = _limit([np.abs(c * d * q).max()])[0]
        c = c / _limit([max(pn, qn)])[0]
    return dict(Dx=Dx, Du=Du, Ed=Ed, c=c)


def scale_agent(ag, sc) -> dict:
    """The scaled agent (same layout as ``oracle.agent``)."""
    s = ag["s"]
    Dx, Du, c = sc["Dx"], sc["Du"], sc["c"]
    out = dict(ag)
    out["A"] = ag["A"] * Dx[None, None, :] / Dx[None, :, None]
    out["B"] = ag["B"] * Du[None, None, :] / Dx[None, :, None]
    out["c"] = ag["c"] / Dx[None, :]
    out["q"] = c * Dx * Dx * ag["q"]
    out["r"] = c * Du * Du * ag["r"]
    out["x_ref"] = ag["x_ref"] / Dx[None, :]
    out["x0"] = ag["x0"] / Dx
    out["tau_max"] = ag["tau_max"] / Du[:s.n_tau]
    if s.n_feet:
        b = s.n_tau
        out["mu"] = ag["mu"] * Du[b + 2] / Du[b]
    return out


def scale_state(s, sc, u, z, y):
    """(u, z, y) of the original problem -> the scaled problem's."""
    e = row_scales(s, sc["Du"])
    return (np.asarray(u).reshape(s.N, s.nu) / sc["Du"],
            np.asarray(z).reshape(s.N, -1) * e,
            sc["c"] * np.asarray(y).reshape(s.N, -1) / e)


def unscale_state(s, sc, x, u, z, y):
    e = row_scales(s, sc["Du"])
    return (np.asarray(x).reshape(s.N + 1, s.nx) * sc["Dx"],
            np.asarray(u).reshape(s.N, s.nu) * sc["Du"],
            np.asarray(z).reshape(s.N, -1) / e,
            np.asarray(y).reshape(s.N, -1) * e / sc["c"])


def rho_estimate(agh, x, u, z, y, rho: float, settings: Optional[Settings] = None,
                 raw: bool = False) -> float:
    """OSQP's residual-balancing estimate of rho on the scaled problem (``raw``:
    before clipping and rounding to the grid)."""
    s = agh["s"]
    st = settings or Settings.default(rho=rho)
    res, _ = residuals(s, agh["A"], agh["B"], agh["c"], agh["q"], agh["r"], agh["x_ref"],
                       agh["x0"], agh["tau_max"], agh["mu"], agh["stance"], x, u, z, y,
                       settings=st)
    C = constraint_matrix(s, agh["mu"])
    u = np.asarray(u).reshape(s.N, s.nu)
    x = np.asarray(x).reshape(s.N + 1, s.nx)
    z = np.asarray(z).reshape(s.N, -1)
    y = np.asarray(y).reshape(s.N, -1)
    cu = np.abs(u @ C.T).max()
    zn = np.abs(z).max()
    px = max(np.abs(x[1:] * agh["q"]).max(), np.abs(u * agh["r"]).max())
    cty = np.abs(y @ C).max()
    qn = np.abs(agh["x_ref"][1:] * agh["q"]).max()
    tiny = 1e-30
    prim = res[0] / max(cu, zn, tiny)
    dual = res[1] / max(px, cty, qn, tiny)
    est = rho * np.sqrt(prim / max(dual, tiny))
    if raw:
        return float(est)
    return grid(est)


def grid(est: float) -> float:
    """An estimate clipped to [1e-6, 1e6] and rounded to the nearest power of 2^(1/4)."""
    est = min(max(est, RHO_MIN), RHO_MAX)
    return float(2.0 ** (np.round(4.0 * np.log2(est)) / 4.0))


def decide(rho: float, raw: float, tolerance: float = 5.0) -> float:
    """The rho after an update with raw estimate ``raw``."""
    est = grid(raw)
    return est if (est > tolerance * rho or est < rho / tolerance) else rho


def solve(ag, *, iters: int = 50, ruiz_iters: int = 10, rho_interval: int = 0,
          rho_tolerance: float = 5.0, warm=None, settings: Optional[Settings] = None,
          tol: float = 1e-10, max_iters: int = 1_000_000) -> dict:
    """Scaled solve of one agent; ``warm`` = (u, z, y) of the original problem.
    ``rho_interval`` 0 keeps rho fixed.  ``iters <= 0`` runs the scaled problem
    to convergence (the oracle's converge mode, fixed rho).  Returns the
    unscaled iterate, the residuals and objective of the original problem, the
    scale factors, the rho of every segment and the raw estimate of every update."""
    s = ag["s"]
    st0 = settings or Settings.default()
    sc = ruiz(ag, ruiz_iters) if ruiz_iters > 0 else dict(
        Dx=np.ones(s.nx), Du=np.ones(s.nu), Ed=np.ones(s.nx), c=1.0)
    agh = scale_agent(ag, sc)
    state = None if warm is None else scale_state(s, sc, *warm)
    rho = st0.rho
    rhos = []
    raws = []  # (rho before, raw estimate) of every update
    done = 0
    out = None
    if iters <= 0:
        out = solve_unscaled(s, agh["A"], agh["B"], agh["c"], agh["q"], agh["r"], agh["x_ref"],
                             agh["x0"], agh["tau_max"], agh["mu"], agh["stance"], iters=0,
                             warm=state, settings=st0, tol=tol, max_iters=max_iters)
        rhos.append(rho)
    while done < iters:
        k = iters - done if rho_interval <= 0 else min(rho_interval, iters - done)
        st = Settings(rho=rho, sigma=st0.sigma, alpha=st0.alpha, rho_eq_scale=st0.rho_eq_scale,
                      rho_min=st0.rho_min)
        out = solve_unscaled(s, agh["A"], agh["B"], agh["c"], agh["q"], agh["r"], agh["x_ref"],
                             agh["x0"], agh["tau_max"], agh["mu"], agh["stance"], iters=k,
                             warm=state, settings=st)
        rhos.append(rho)
        done += k
        state = (out["u"], out["z"], out["y"])
        if out["status"] != 0:
            break
        if done < iters and rho_interval > 0:
            raw = rho_estimate(agh, out["x"], out["u"], out["z"], out["y"], rho, st, raw=True)
            raws.append((rho, raw))
            rho = decide(rho, raw, rho_tolerance)
    x, u, z, y = unscale_state(s, sc, out["x"], out["u"], out["z"], out["y"])
    res, obj = residuals(s, ag["A"], ag["B"], ag["c"], ag["q"], ag["r"], ag["x_ref"], ag["x0"],
                         ag["tau_max"], ag["mu"], ag["stance"], x, u, z, y, settings=st0)
    return dict(x=x, u=u, z=z, y=y, res=res, objective=obj, status=out["status"], scale=sc,
                rhos=rhos, estimates=raws)
