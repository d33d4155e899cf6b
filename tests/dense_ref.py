"""Dense, independent formulations used to pin the oracle (CPU, NumPy/SciPy).

Nothing here calls the oracle's arithmetic: each helper is written from the
problem statement (stacked QP with the dynamics as equality rows) and solved
with dense linear algebra, brute force or a different algorithm.
"""
from __future__ import annotations

import itertools

import numpy as np

INF = np.inf


def C_dense(s, mu):
    """Constraint rows of one stage: identity on u, then the 4 friction-pyramid
    facets per foot (f_x - mu f_z, -f_x - mu f_z, f_y - mu f_z, -f_y - mu f_z)."""
    m = s.nu + 4 * s.n_feet
    C = np.zeros((m, s.nu))
    C[: s.nu, : s.nu] = np.eye(s.nu)
    for f in range(s.n_feet):
        b = s.n_tau + f * s.foot_dim
        fx, fy, fz = b, b + 1, b + 2
        rows = [(fx, 1.0), (fx, -1.0), (fy, 1.0), (fy, -1.0)]
        for j, (col, sgn) in enumerate(rows):
            C[s.nu + 4 * f + j, col] = sgn
            C[s.nu + 4 * f + j, fz] = -mu
    return C


def bounds_table(s, tau_max, stance):
    """(l, h) per stage straight from the problem statement."""
    m = s.nu + 4 * s.n_feet
    l = np.zeros((s.N, m))
    h = np.zeros((s.N, m))
    for k in range(s.N):
        l[k, : s.n_tau], h[k, : s.n_tau] = -np.asarray(tau_max), np.asarray(tau_max)
        for f in range(s.n_feet):
            w = slice(s.n_tau + f * s.foot_dim, s.n_tau + (f + 1) * s.foot_dim)
            pyr = slice(s.nu + 4 * f, s.nu + 4 * f + 4)
            if stance[k, f]:
                l[k, w], h[k, w] = -INF, INF
                l[k, s.n_tau + f * s.foot_dim + 2] = 0.0  # f_z >= 0
                l[k, pyr], h[k, pyr] = -INF, 0.0
            else:
                l[k, w], h[k, w] = 0.0, 0.0
                l[k, pyr], h[k, pyr] = -INF, INF
    return l, h


def rho_table(l, h, rho=0.1, rho_eq=100.0, rho_min=1e-6):
    out = np.full(l.shape, rho)
    out[l == h] = rho_eq
    out[np.isinf(l) & np.isinf(h)] = rho_min
    return out


def complementarity_natural(l, h, z, y):
    """Largest violation of "z in [l, h] and y in the normal cone of [l, h] at z",
    as the projection (natural) residual |z - Pi_[l,h](z + y)| together with the
    distance of z from [l, h].  Both vanish exactly at a complementary pair:
    y > 0 only where z = h, y < 0 only where z = l."""
    nat = np.abs(z - np.clip(z + y, l, h))
    out = np.maximum(np.maximum(z - h, l - z), 0.0)
    return float(max(nat.max(), out.max()))


def dynamics_rows(s, A, B, c, x0):
    """G v = b for v = [x_1..x_N, u_0..u_{N-1}]: x_{k+1} - A_k x_k - B_k u_k = c_k."""
    N, nx, nu = s.N, s.nx, s.nu
    nv = N * nx + N * nu
    G = np.zeros((N * nx, nv))
    b = np.zeros(N * nx)
    for k in range(N):
        r = slice(k * nx, (k + 1) * nx)
        G[r, k * nx:(k + 1) * nx] = np.eye(nx)  # x_{k+1}
        if k > 0:
            G[r, (k - 1) * nx:k * nx] = -A[k]
        G[r, N * nx + k * nu:N * nx + (k + 1) * nu] = -B[k]
        b[r] = c[k] + (A[0] @ x0 if k == 0 else 0.0)
    return G, b


def x_subproblem(s, q, r, x_ref, C, rho, sigma, xj, uj, z, y):
    """Hessian and gradient-at-0 of the ADMM x-subproblem objective
       sum_k 1/2 (x_k - r_k)' Q (x_k - r_k) + sigma/2 |x_k - x_k^j|^2          (k = 1..N)
     + sum_k 1/2 u_k' R u_k + sigma/2 |u_k - u_k^j|^2
           + 1/2 sum_i rho_i (C u_k - z_k + y_k / rho)_i^2                    (k = 0..N-1)
    in v = [x_1..x_N, u_0..u_{N-1}] (constant terms dropped)."""
    N, nx, nu = s.N, s.nx, s.nu
    nv = N * nx + N * nu
    H = np.zeros((nv, nv))
    g = np.zeros(nv)
    for k in range(1, N + 1):
        sl = slice((k - 1) * nx, k * nx)
        H[sl, sl] = np.diag(q) + sigma * np.eye(nx)
        g[sl] = -q * x_ref[k] - sigma * xj[k]
    for k in range(N):
        sl = slice(N * nx + k * nu, N * nx + (k + 1) * nu)
        D = np.diag(rho[k])
        H[sl, sl] = np.diag(r) + sigma * np.eye(nu) + C.T @ D @ C
        g[sl] = -sigma * uj[k] + C.T @ D @ (-z[k] + y[k] / rho[k])
    return H, g


def x_subproblem_objective(s, q, r, x_ref, C, rho, sigma, xj, uj, z, y, v):
    """The same objective evaluated directly (used to pin ``x_subproblem``)."""
    N, nx, nu = s.N, s.nx, s.nu
    x = v[: N * nx].reshape(N, nx)
    u = v[N * nx:].reshape(N, nu)
    f = 0.0
    for k in range(1, N + 1):
        e = x[k - 1] - x_ref[k]
        f += 0.5 * np.sum(q * e * e) + 0.5 * sigma * np.sum((x[k - 1] - xj[k]) ** 2)
    for k in range(N):
        f += 0.5 * np.sum(r * u[k] ** 2) + 0.5 * sigma * np.sum((u[k] - uj[k]) ** 2)
        t = C @ u[k] - z[k] + y[k] / rho[k]
        f += 0.5 * np.sum(rho[k] * t * t)
    return f


def kkt_solve(H, g, G, b):
    """min 1/2 v'Hv + g'v  s.t. G v = b, by one dense solve of the KKT matrix."""
    n, p = H.shape[0], G.shape[0]
    K = np.zeros((n + p, n + p))
    K[:n, :n] = H
    K[:n, n:] = G.T
    K[n:, :n] = G
    sol = np.linalg.solve(K, np.concatenate([-g, b]))
    return sol[:n], sol[n:]


def split(s, v, x0):
    N, nx = s.N, s.nx
    x = np.vstack([x0[None, :], v[: N * nx].reshape(N, nx)])
    u = v[N * nx:].reshape(N, s.nu)
    return x, u


def dense_admm(s, A, B, c, q, r, x_ref, x0, tau_max, mu, stance, iters, *, rho=0.1,
               sigma=1e-6, alpha=1.6, rho_eq=100.0, rho_min=1e-6, warm=None):
    """OSQP iterations (relaxed x-update, projection, dual ascent) with every
    x-update solved by a dense KKT solve of the stacked problem."""
    C = C_dense(s, mu)
    l, h = bounds_table(s, tau_max, stance)
    rr = rho_table(l, h, rho, rho_eq, rho_min)
    G, b = dynamics_rows(s, A, B, c, x0)
    m = C.shape[0]
    if warm is None:
        u = np.zeros((s.N, s.nu))
        z = np.zeros((s.N, m))
        y = np.zeros((s.N, m))
    else:
        u, z, y = (np.array(w, dtype=np.float64) for w in warm)
    x = rollout(s, A, B, c, x0, u)
    for _ in range(iters):
        H, g = x_subproblem(s, q, r, x_ref, C, rr, sigma, x, u, z, y)
        v, _ = kkt_solve(H, g, G, b)
        xt, ut = split(s, v, x0)
        zeta = ut @ C.T
        x = alpha * xt + (1 - alpha) * x
        x[0] = x0
        u = alpha * ut + (1 - alpha) * u
        w = alpha * zeta + (1 - alpha) * z
        zn = np.clip(w + y / rr, l, h)
        y = y + rr * (w - zn)
        z = zn
    return x, u, z, y


def rollout(s, A, B, c, x0, u):
    x = np.zeros((s.N + 1, s.nx))
    x[0] = x0
    for k in range(s.N):
        x[k + 1] = A[k] @ x[k] + B[k] @ u[k] + c[k]
    return x


def condensed(s, A, B, c, x0):
    """x_{1..N} = Phi x0 + Gam u + gam, built by simulating the dynamics."""
    N, nx, nu = s.N, s.nx, s.nu
    zero_u = np.zeros((N, nu))
    base = rollout(s, A, B, c, x0, zero_u)[1:].ravel()
    Gam = np.zeros((N * nx, N * nu))
    for j in range(N * nu):
        e = np.zeros(N * nu)
        e[j] = 1.0
        xs = rollout(s, A, B, np.zeros_like(c), np.zeros(nx), e.reshape(N, nu))[1:].ravel()
        Gam[:, j] = xs
    return base, Gam


def unconstrained_optimum(s, A, B, c, q, r, x_ref, x0):
    """Normal equations of the condensed least-squares LQR: (G'QG + R) u = -G'Q(x_free - r)."""
    base, Gam = condensed(s, A, B, c, x0)
    Qb = np.kron(np.eye(s.N), np.diag(q))
    Rb = np.kron(np.eye(s.N), np.diag(r))
    rhs = -Gam.T @ Qb @ (base - x_ref[1:].ravel())
    u = np.linalg.solve(Gam.T @ Qb @ Gam + Rb, rhs)
    return u.reshape(s.N, s.nu)


def brute_force_qp(s, A, B, c, q, r, x_ref, x0, tau_max, mu, stance, tol=1e-9):
    """Exact QP optimum by enumerating which bounded rows sit at which bound.

    Every bounded row is inactive, at its lower bound, or at its upper bound
    (equality rows are always active).  For each choice the equality-
    constrained QP is solved densely; the optimum is the choice whose primal
    point satisfies all bounds and whose multipliers have the right signs
    (>= 0 at an upper bound, <= 0 at a lower bound)."""
    C = C_dense(s, mu)
    l, h = bounds_table(s, tau_max, stance)
    G, b = dynamics_rows(s, A, B, c, x0)
    N, nx, nu = s.N, s.nx, s.nu
    nv = N * nx + N * nu
    H = np.zeros((nv, nv))
    g = np.zeros(nv)
    for k in range(1, N + 1):
        sl = slice((k - 1) * nx, k * nx)
        H[sl, sl] = np.diag(q)
        g[sl] = -q * x_ref[k]
    H[N * nx:, N * nx:] = np.kron(np.eye(N), np.diag(r))
    rows = []  # (k, i, choices)
    for k in range(N):
        for i in range(C.shape[0]):
            lo, hi = l[k, i], h[k, i]
            if lo == hi:
                rows.append((k, i, ("eq",)))
                continue
            ch = ["free"]
            if np.isfinite(lo):
                ch.append("lo")
            if np.isfinite(hi):
                ch.append("hi")
            rows.append((k, i, tuple(ch)))
    best = None
    for combo in itertools.product(*[ch for (_, _, ch) in rows]):
        E, e, kinds = [], [], []
        for (k, i, _), kind in zip(rows, combo):
            if kind == "free":
                continue
            row = np.zeros(nv)
            row[N * nx + k * nu:N * nx + (k + 1) * nu] = C[i]
            E.append(row)
            e.append(l[k, i] if kind in ("lo", "eq") else h[k, i])
            kinds.append(kind)
        GG = np.vstack([G] + ([np.array(E)] if E else []))
        bb = np.concatenate([b, np.array(e)])
        try:
            v, lam = kkt_solve(H, g, GG, bb)
        except np.linalg.LinAlgError:
            continue
        mult = lam[G.shape[0]:]
        x, u = split(s, v, x0)
        cu = u @ C.T
        if np.any(cu < l - tol) or np.any(cu > h + tol):
            continue
        ok = True
        for kind, mm in zip(kinds, mult):
            if kind == "hi" and mm < -tol:
                ok = False
            if kind == "lo" and mm > tol:
                ok = False
        if not ok:
            continue
        y = np.zeros((N, C.shape[0]))
        j = 0
        for (k, i, _), kind in zip(rows, combo):
            if kind != "free":
                y[k, i] = mult[j]
                j += 1
        best = (x, u, y)
        break
    return best


def osqp_dense(s, A, B, c, q, r, x_ref, x0, tau_max, mu, stance, *, rho=0.1, sigma=1e-6,
               alpha=1.6, rho_eq_scale=1e3, iters=20000, tol=1e-11):
    """The paper's form of the iteration: OSQP on the stacked QP with the
    dynamics as equality rows of the constraint matrix (finite rho_eq), using
    the quasi-definite KKT matrix [[P + sigma I, A'], [A, -rho^{-1} I]]
    factorised once (Eq. (kkt_system), Eq. (ldl))."""
    C = C_dense(s, mu)
    l, h = bounds_table(s, tau_max, stance)
    G, b = dynamics_rows(s, A, B, c, x0)
    N, nx, nu = s.N, s.nx, s.nu
    nv = N * nx + N * nu
    P = np.zeros((nv, nv))
    qv = np.zeros(nv)
    for k in range(1, N + 1):
        sl = slice((k - 1) * nx, k * nx)
        P[sl, sl] = np.diag(q)
        qv[sl] = -q * x_ref[k]
    P[N * nx:, N * nx:] = np.kron(np.eye(N), np.diag(r))
    Cb = np.zeros((N * C.shape[0], nv))
    for k in range(N):
        Cb[k * C.shape[0]:(k + 1) * C.shape[0], N * nx + k * nu:N * nx + (k + 1) * nu] = C
    Am = np.vstack([G, Cb])
    lo = np.concatenate([b, l.ravel()])
    hi = np.concatenate([b, h.ravel()])
    rv = np.where(lo == hi, rho * rho_eq_scale, rho)
    rv = np.where(np.isinf(lo) & np.isinf(hi), 1e-6, rv)
    Kkkt = np.block([[P + sigma * np.eye(nv), Am.T], [Am, -np.diag(1.0 / rv)]])
    x = np.zeros(nv)
    z = np.zeros(Am.shape[0])
    z[: G.shape[0]] = b
    y = np.zeros(Am.shape[0])
    for _ in range(iters):
        sol = np.linalg.solve(Kkkt, np.concatenate([sigma * x - qv, z - y / rv]))
        xt, nu_ = sol[:nv], sol[nv:]
        zt = z + (nu_ - y) / rv
        x = alpha * xt + (1 - alpha) * x
        zn = np.clip(alpha * zt + (1 - alpha) * z + y / rv, lo, hi)
        y = y + rv * (alpha * zt + (1 - alpha) * z - zn)
        z = zn
        rp = np.abs(Am @ x - z).max()
        rd = np.abs(P @ x + qv + Am.T @ y).max()
        if rp < tol and rd < tol:
            break
    xs, us = split(s, x, x0)
    return xs, us


def state_rho(x_lo, x_hi, rho=0.1, rho_eq=100.0, rho_min=1e-6):
    """OSQP's penalty rule for the state rows (joint limits), per component."""
    x_lo, x_hi = np.asarray(x_lo, dtype=float), np.asarray(x_hi, dtype=float)
    out = np.full(x_lo.shape, rho)
    out[x_lo == x_hi] = rho_eq
    out[np.isinf(x_lo) & np.isinf(x_hi)] = rho_min
    return out


def dense_admm_limits(s, A, B, c, q, r, x_ref, x0, tau_max, mu, stance, x_lo, x_hi, iters, *,
                      rho=0.1, sigma=1e-6, alpha=1.6, rho_eq=100.0, rho_min=1e-6):
    """dense_admm with the joint-limit rows x_lo <= x_k <= x_hi (k = 1..N) added
    to the splitting: one more row block C_x = I on every state, its own
    (z_x, y_x), projection and dual update; the x-subproblem gains
    rho_x/2 |x_k - z_x + y_x/rho_x|^2."""
    C = C_dense(s, mu)
    l, h = bounds_table(s, tau_max, stance)
    rr = rho_table(l, h, rho, rho_eq, rho_min)
    rx = state_rho(x_lo, x_hi, rho, rho_eq, rho_min)
    G, b = dynamics_rows(s, A, B, c, x0)
    m = C.shape[0]
    N, nx = s.N, s.nx
    u = np.zeros((N, s.nu))
    z = np.zeros((N, m))
    y = np.zeros((N, m))
    zx = np.zeros((N, nx))
    yx = np.zeros((N, nx))
    x = rollout(s, A, B, c, x0, u)
    for _ in range(iters):
        H, g = x_subproblem(s, q, r, x_ref, C, rr, sigma, x, u, z, y)
        for k in range(1, N + 1):
            sl = slice((k - 1) * nx, k * nx)
            H[sl, sl] += np.diag(rx)
            g[sl] += rx * (-zx[k - 1] + yx[k - 1] / rx)
        v, _ = kkt_solve(H, g, G, b)
        xt, ut = split(s, v, x0)
        zeta = ut @ C.T
        x = alpha * xt + (1 - alpha) * x
        x[0] = x0
        u = alpha * ut + (1 - alpha) * u
        w = alpha * zeta + (1 - alpha) * z
        zn = np.clip(w + y / rr, l, h)
        y = y + rr * (w - zn)
        z = zn
        wx = alpha * xt[1:] + (1 - alpha) * zx
        zxn = np.clip(wx + yx / rx, x_lo, x_hi)
        yx = yx + rx * (wx - zxn)
        zx = zxn
    return x, u, z, y, zx, yx


def brute_force_qp_limits(s, A, B, c, q, r, x_ref, x0, tau_max, mu, stance, x_lo, x_hi,
                          tol=1e-9):
    """brute_force_qp with the joint-limit rows x_lo <= x_k <= x_hi (k = 1..N)
    among the enumerated rows.  Returns (x, u, y, y_x) or None."""
    C = C_dense(s, mu)
    l, h = bounds_table(s, tau_max, stance)
    G, b = dynamics_rows(s, A, B, c, x0)
    N, nx, nu = s.N, s.nx, s.nu
    nv = N * nx + N * nu
    H = np.zeros((nv, nv))
    g = np.zeros(nv)
    for k in range(1, N + 1):
        sl = slice((k - 1) * nx, k * nx)
        H[sl, sl] = np.diag(q)
        g[sl] = -q * x_ref[k]
    H[N * nx:, N * nx:] = np.kron(np.eye(N), np.diag(r))
    rows = []  # (row vector, lo, hi)
    for k in range(N):
        for i in range(C.shape[0]):
            vec = np.zeros(nv)
            vec[N * nx + k * nu:N * nx + (k + 1) * nu] = C[i]
            rows.append((vec, l[k, i], h[k, i], ("u", k, i)))
    for k in range(1, N + 1):
        for i in range(nx):
            vec = np.zeros(nv)
            vec[(k - 1) * nx + i] = 1.0
            rows.append((vec, x_lo[i], x_hi[i], ("x", k - 1, i)))
    choices = []
    for vec, lo, hi, _ in rows:
        if lo == hi:
            choices.append(("eq",))
            continue
        ch = ["free"]
        if np.isfinite(lo):
            ch.append("lo")
        if np.isfinite(hi):
            ch.append("hi")
        choices.append(tuple(ch))
    for combo in itertools.product(*choices):
        E, e, kinds, tags = [], [], [], []
        for (vec, lo, hi, tag), kind in zip(rows, combo):
            if kind == "free":
                continue
            E.append(vec)
            e.append(lo if kind in ("lo", "eq") else hi)
            kinds.append(kind)
            tags.append(tag)
        GG = np.vstack([G] + ([np.array(E)] if E else []))
        bb = np.concatenate([b, np.array(e)])
        try:
            v, lam = kkt_solve(H, g, GG, bb)
        except np.linalg.LinAlgError:
            continue
        mult = lam[G.shape[0]:]
        vals = np.array([vec @ v for vec, _, _, _ in rows])
        los = np.array([lo for _, lo, _, _ in rows])
        his = np.array([hi for _, _, hi, _ in rows])
        if np.any(vals < los - tol) or np.any(vals > his + tol):
            continue
        if any((kd == "hi" and mm < -tol) or (kd == "lo" and mm > tol) for kd, mm in zip(kinds, mult)):
            continue
        x, u = split(s, v, x0)
        y = np.zeros((N, C.shape[0]))
        yx = np.zeros((N, nx))
        for (kind_, k, i), mm in zip(tags, mult):
            if kind_ == "u":
                y[k, i] = mm
            else:
                yx[k, i] = mm
        return x, u, y, yx
    return None


def contact_table(s, stance, rho=0.1, rho_eq=100.0, rho_min=1e-6):
    """Bounds and penalties [N, n_feet*foot_dim] of the no-slip rows of x_k,
    k = 1..N (row k-1): equality rows J_f v_k = 0 for a foot in stance at stage
    min(k, N-1), free rows for a swinging foot."""
    nc = s.n_feet * s.foot_dim
    l = np.full((s.N, nc), -np.inf)
    h = np.full((s.N, nc), np.inf)
    rr = np.full((s.N, nc), rho_min)
    for k in range(1, s.N + 1):
        phase = stance[min(k, s.N - 1)]
        for f in range(s.n_feet):
            if phase[f]:
                sl = slice(f * s.foot_dim, (f + 1) * s.foot_dim)
                l[k - 1, sl] = 0.0
                h[k - 1, sl] = 0.0
                rr[k - 1, sl] = rho_eq
    return l, h, rr


def dense_admm_state_rows(s, A, B, c, q, r, x_ref, x0, tau_max, mu, stance, iters, *, x_lo=None,
                          x_hi=None, J=None, rho=0.1, sigma=1e-6, alpha=1.6, rho_eq=100.0,
                          rho_min=1e-6):
    """dense_admm with state rows on x_1..x_N added to the splitting: the joint
    limits (identity rows, x_lo/x_hi) and the no-slip rows (rows J, bounds of
    contact_table), each block with its own (z, y), projection and dual update;
    the x-subproblem gains rho/2 |Cx x_k - z + y/rho|^2 for each block."""
    C = C_dense(s, mu)
    l, h = bounds_table(s, tau_max, stance)
    rr = rho_table(l, h, rho, rho_eq, rho_min)
    G, b = dynamics_rows(s, A, B, c, x0)
    N, nx = s.N, s.nx
    blocks = []  # (Cx [rows, nx], lo [N, rows], hi [N, rows], rho [N, rows])
    if x_lo is not None:
        rx = state_rho(x_lo, x_hi, rho, rho_eq, rho_min)
        blocks.append((np.eye(nx), np.tile(x_lo, (N, 1)), np.tile(x_hi, (N, 1)), np.tile(rx, (N, 1))))
    if J is not None:
        blocks.append((np.asarray(J, dtype=float),) + contact_table(s, stance, rho, rho_eq, rho_min))
    m = C.shape[0]
    u = np.zeros((N, s.nu))
    z = np.zeros((N, m))
    y = np.zeros((N, m))
    zs = [np.zeros((N, Cx.shape[0])) for Cx, *_ in blocks]
    ys = [np.zeros((N, Cx.shape[0])) for Cx, *_ in blocks]
    x = rollout(s, A, B, c, x0, u)
    for _ in range(iters):
        H, g = x_subproblem(s, q, r, x_ref, C, rr, sigma, x, u, z, y)
        for (Cx, lo, hi, rb), zb, yb in zip(blocks, zs, ys):
            for k in range(1, N + 1):
                sl = slice((k - 1) * nx, k * nx)
                H[sl, sl] += Cx.T @ np.diag(rb[k - 1]) @ Cx
                g[sl] += Cx.T @ (yb[k - 1] - rb[k - 1] * zb[k - 1])
        v, _ = kkt_solve(H, g, G, b)
        xt, ut = split(s, v, x0)
        zeta = ut @ C.T
        x = alpha * xt + (1 - alpha) * x
        x[0] = x0
        u = alpha * ut + (1 - alpha) * u
        w = alpha * zeta + (1 - alpha) * z
        zn = np.clip(w + y / rr, l, h)
        y = y + rr * (w - zn)
        z = zn
        for bi, (Cx, lo, hi, rb) in enumerate(blocks):
            wb = alpha * (xt[1:] @ Cx.T) + (1 - alpha) * zs[bi]
            zbn = np.clip(wb + ys[bi] / rb, lo, hi)
            ys[bi] = ys[bi] + rb * (wb - zbn)
            zs[bi] = zbn
    out = dict(x=x, u=u, z=z, y=y)
    bi = 0
    if x_lo is not None:
        out.update(zx=zs[bi], yx=ys[bi])
        bi += 1
    if J is not None:
        out.update(zc=zs[bi], yc=ys[bi])
    return out


def brute_force_qp_contacts(s, A, B, c, q, r, x_ref, x0, tau_max, mu, stance, J, tol=1e-9):
    """brute_force_qp with the no-slip rows of stance feet as equality
    constraints on x_1..x_N (contact_table); only the input rows are
    enumerated.  Returns (x, u, y, y_c) or None."""
    C = C_dense(s, mu)
    l, h = bounds_table(s, tau_max, stance)
    lc, hc, _ = contact_table(s, stance)
    G, b = dynamics_rows(s, A, B, c, x0)
    N, nx, nu = s.N, s.nx, s.nu
    J = np.asarray(J, dtype=float)
    nc = J.shape[0]
    nv = N * nx + N * nu
    H = np.zeros((nv, nv))
    g = np.zeros(nv)
    for k in range(1, N + 1):
        sl = slice((k - 1) * nx, k * nx)
        H[sl, sl] = np.diag(q)
        g[sl] = -q * x_ref[k]
    H[N * nx:, N * nx:] = np.kron(np.eye(N), np.diag(r))
    eq_rows, eq_tags = [], []
    for k in range(1, N + 1):
        for i in range(nc):
            if lc[k - 1, i] == hc[k - 1, i]:
                vec = np.zeros(nv)
                vec[(k - 1) * nx:k * nx] = J[i]
                eq_rows.append(vec)
                eq_tags.append((k - 1, i))
    rows = []
    for k in range(N):
        for i in range(C.shape[0]):
            vec = np.zeros(nv)
            vec[N * nx + k * nu:N * nx + (k + 1) * nu] = C[i]
            rows.append((vec, l[k, i], h[k, i], (k, i)))
    choices = []
    for vec, lo, hi, _ in rows:
        if lo == hi:
            choices.append(("eq",))
            continue
        ch = ["free"]
        if np.isfinite(lo):
            ch.append("lo")
        if np.isfinite(hi):
            ch.append("hi")
        choices.append(tuple(ch))
    G2 = np.vstack([G] + ([np.array(eq_rows)] if eq_rows else []))
    b2 = np.concatenate([b, np.zeros(len(eq_rows))])
    for combo in itertools.product(*choices):
        E, e, kinds, tags = [], [], [], []
        for (vec, lo, hi, tag), kind in zip(rows, combo):
            if kind == "free":
                continue
            E.append(vec)
            e.append(lo if kind in ("lo", "eq") else hi)
            kinds.append(kind)
            tags.append(tag)
        GG = np.vstack([G2] + ([np.array(E)] if E else []))
        bb = np.concatenate([b2, np.array(e)])
        try:
            v, lam = kkt_solve(H, g, GG, bb)
        except np.linalg.LinAlgError:
            continue
        mult = lam[G2.shape[0]:]
        vals = np.array([vec @ v for vec, _, _, _ in rows])
        los = np.array([lo for _, lo, _, _ in rows])
        his = np.array([hi for _, _, hi, _ in rows])
        if np.any(vals < los - tol) or np.any(vals > his + tol):
            continue
        if any((kd == "hi" and mm < -tol) or (kd == "lo" and mm > tol) for kd, mm in zip(kinds, mult)):
            continue
        x, u = split(s, v, x0)
        y = np.zeros((N, C.shape[0]))
        for (k, i), mm in zip(tags, mult):
            y[k, i] = mm
        yc = np.zeros((N, nc))
        for (k, i), mm in zip(eq_tags, lam[G.shape[0]:G2.shape[0]]):
            yc[k, i] = mm
        return x, u, y, yc
    return None


def osqp_dense_fixed(s, A, B, c, q, r, x_ref, x0, tau_max, mu, stance, iters, *, rho=0.1,
                     sigma=1e-6, alpha=1.6, rho_eq_scale=1e3, rho_min=1e-6, warm=None):
    """``iters`` OSQP iterations on the stacked QP with the dynamics as equality
    rows (finite rho_eq), each solving the quasi-definite KKT system of
    Eq. (kkt_system) with a dense solve.  Cold start: u = 0, x rolled out
    from x0, z = A v (the rows' values), y = 0; ``warm`` = (v, z, y).
    Returns x [N+1, nx], u [N, nu], the input rows' z, y [N, m] and the
    dynamics rows' zd, yd [N, nx]."""
    C = C_dense(s, mu)
    l, h = bounds_table(s, tau_max, stance)
    G, b = dynamics_rows(s, A, B, c, x0)
    N, nx, nu = s.N, s.nx, s.nu
    m = C.shape[0]
    nv = N * nx + N * nu
    P = np.zeros((nv, nv))
    qv = np.zeros(nv)
    for k in range(1, N + 1):
        sl = slice((k - 1) * nx, k * nx)
        P[sl, sl] = np.diag(q)
        qv[sl] = -q * x_ref[k]
    P[N * nx:, N * nx:] = np.kron(np.eye(N), np.diag(r))
    Cb = np.zeros((N * m, nv))
    for k in range(N):
        Cb[k * m:(k + 1) * m, N * nx + k * nu:N * nx + (k + 1) * nu] = C
    Am = np.vstack([G, Cb])
    lo = np.concatenate([b, l.ravel()])
    hi = np.concatenate([b, h.ravel()])
    rv = np.where(lo == hi, rho * rho_eq_scale, rho)
    rv = np.where(np.isinf(lo) & np.isinf(hi), rho_min, rv)
    K = np.block([[P + sigma * np.eye(nv), Am.T], [Am, -np.diag(1.0 / rv)]])
    if warm is None:
        xs = rollout(s, A, B, c, x0, np.zeros((N, nu)))
        v = np.concatenate([xs[1:].ravel(), np.zeros(N * nu)])
        z = Am @ v
        y = np.zeros(Am.shape[0])
    else:
        v, z, y = (np.array(w, dtype=float) for w in warm)
    for _ in range(iters):
        sol = np.linalg.solve(K, np.concatenate([sigma * v - qv, z - y / rv]))
        vt, nu_ = sol[:nv], sol[nv:]
        zt = z + (nu_ - y) / rv
        v = alpha * vt + (1 - alpha) * v
        w = alpha * zt + (1 - alpha) * z
        zn = np.clip(w + y / rv, lo, hi)
        y = y + rv * (w - zn)
        z = zn
    xs, us = split(s, v, x0)
    return dict(x=xs, u=us, z=z[N * nx:].reshape(N, m), y=y[N * nx:].reshape(N, m),
                zd=z[:N * nx].reshape(N, nx), yd=y[:N * nx].reshape(N, nx), v=v, z_all=z, y_all=y)
