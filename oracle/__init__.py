"""FP64 CPU oracle for the batched MPC QP solve -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  The HIP product path never does, and the two
share no code: the oracle is plain C in ``mpc_oracle.c`` (IEEE double, plain
loops, OpenMP over agents) plus this ctypes wrapper.

Every function below follows the paper's MPC solve (Sec. III-B, Eq.
(kkt_system)-(backsolve_2), Alg. 1) under the readings listed at the top of
``mpc_oracle.c``.  Pins that tie it to mathematics independent of itself live
in ``tests/test_oracle_pins.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libmpc_oracle.so")
_SRC = os.path.join(_HERE, "mpc_oracle.c")

OK, CONVERGED, NOT_PD, NONFINITE = 0, 1, 2, 3


def build(force: bool = True, src: str = _SRC, out: str = _SO) -> str:
    """Compile the oracle with gcc (IEEE semantics: no fast-math, no FP contraction)."""
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off",
                               "-fno-fast-math", "-shared", "-fPIC", "-Wall", "-I", _HERE, "-o",
                               tmp, src, "-lm"])
        os.replace(tmp, out)
    return out


class Settings(ctypes.Structure):
    _fields_ = [("rho", ctypes.c_double), ("sigma", ctypes.c_double),
                ("alpha", ctypes.c_double), ("rho_eq_scale", ctypes.c_double),
                ("rho_min", ctypes.c_double)]

    @classmethod
    def default(cls, **kw) -> "Settings":
        v = dict(rho=0.1, sigma=1e-6, alpha=1.6, rho_eq_scale=1e3, rho_min=1e-6)
        v.update(kw)
        return cls(**v)


class _Shape(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("N", "nx", "nu", "n_tau", "n_feet", "foot_dim")]


_lib = None
_lib_path = None
_D = ctypes.POINTER(ctypes.c_double)
_U8 = ctypes.POINTER(ctypes.c_uint8)
_I32 = ctypes.POINTER(ctypes.c_int32)


def use_library(path: Optional[str]) -> None:
    """Point the wrapper at another build of the oracle (None = the default one).
    Used by the mutation tests, which load deliberately broken copies."""
    global _lib, _lib_path
    _lib, _lib_path = None, path


def lib():
    global _lib
    if _lib is None:
        path = _lib_path or _SO
        if path == _SO and not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(path)
        P = ctypes.POINTER
        L.orc_rows.argtypes = [P(_Shape)]
        L.orc_rows.restype = ctypes.c_int32
        L.orc_constraint_matrix.argtypes = [P(_Shape), ctypes.c_double, _D]
        L.orc_stage_bounds.argtypes = [P(_Shape), P(Settings), _D, _U8, _D, _D, _D]
        L.orc_factor.argtypes = [P(_Shape), P(Settings), _D, _D, _D, _D, _D, _D, ctypes.c_double,
                                 _D, _D, _D, _D, _D, _D]
        L.orc_contact_rows.argtypes = [P(_Shape)]
        L.orc_contact_rows.restype = ctypes.c_int32
        L.orc_contact_bounds.argtypes = [P(_Shape), P(Settings), _U8, _D, _D, _D]
        L.orc_contact_weight.argtypes = [P(_Shape), _D, _D, _D]
        L.orc_state_penalties.argtypes = [P(_Shape), P(Settings), _D, _D, _D]
        L.orc_factor.restype = ctypes.c_int
        L.orc_xupdate.argtypes = [P(_Shape), _D, _D, _D, _D, _D, _D, _D, _D, _D, _D, _D]
        L.orc_residuals.argtypes = [P(_Shape), P(Settings), _D, _D, _D, _D, _D, _D, _D, _D, _D,
                                    ctypes.c_double, _U8, _D, _D, _D, _D, _D, _D, _D, _D, _D, _D,
                                    _D, _D, _D]
        L.orc_solve.argtypes = [P(_Shape), P(Settings), _D, _D, _D, _D, _D, _D, _D, _D, _D,
                                ctypes.c_double, _U8, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                ctypes.c_int, _D, _D, _D, _D, _D, _D, ctypes.POINTER(ctypes.c_int),
                                _D, _D, _D, _D, _D, _D, _D]
        L.orc_solve.restype = ctypes.c_int
        L.orc_solve_batch.argtypes = [ctypes.c_int32, _I32, P(Settings), _D, _D, _D, _D, _D, _D,
                                      _D, _D, _D, _D, _U8, ctypes.c_int, ctypes.c_int, _D, _D, _D,
                                      _D, _D, _D, _I32, ctypes.c_int, _D, _D, _D, _D, _D, _D, _D]
        L.orc_solve_batch.restype = ctypes.c_int
        L.orc_advance_batch.argtypes = [ctypes.c_int32, _I32, _D, _D, _D, _D, _D, _D, _D]
        _lib = L
    return _lib


def _d(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _shape(s) -> _Shape:
    return _Shape(*s.as_tuple())


def rows(s) -> int:
    return s.nu + 4 * s.n_feet


def constraint_matrix(s, mu: float) -> np.ndarray:
    C = np.zeros((rows(s), s.nu))
    lib().orc_constraint_matrix(ctypes.byref(_shape(s)), float(mu), _d(C))
    return C


def stage_bounds(s, tau_max, stance, settings: Optional[Settings] = None):
    """(l, h, rho), each [N][m]."""
    st = settings or Settings.default()
    m = rows(s)
    l, h, rho = (np.zeros((s.N, m)) for _ in range(3))
    stance = np.ascontiguousarray(stance, dtype=np.uint8)
    lib().orc_stage_bounds(ctypes.byref(_shape(s)), ctypes.byref(st), _d(_f64(tau_max)),
                           stance.ctypes.data_as(_U8), _d(l), _d(h), _d(rho))
    return l, h, rho


def state_penalties(s, x_lo, x_hi, settings: Optional[Settings] = None) -> np.ndarray:
    """Penalties rho_x [nx] of the state rows (joint limits)."""
    st = settings or Settings.default()
    out = np.zeros(s.nx)
    lib().orc_state_penalties(ctypes.byref(_shape(s)), ctypes.byref(st), _d(_f64(x_lo)),
                              _d(_f64(x_hi)), _d(out))
    return out


def contact_rows(s) -> int:
    """No-slip rows per stage: n_feet * foot_dim."""
    return int(lib().orc_contact_rows(ctypes.byref(_shape(s))))


def contact_bounds(s, stance, settings: Optional[Settings] = None):
    """(l, h, rho) [N, nc] of the no-slip rows of x_1..x_N."""
    st = settings or Settings.default()
    nc = contact_rows(s)
    l, h, rho = (np.zeros((s.N, nc)) for _ in range(3))
    stance = np.ascontiguousarray(stance, dtype=np.uint8)
    lib().orc_contact_bounds(ctypes.byref(_shape(s)), ctypes.byref(st), stance.ctypes.data_as(_U8),
                             _d(l), _d(h), _d(rho))
    return l, h, rho


def contact_weight(s, J, rho_c) -> np.ndarray:
    """Qadd [N+1, nx, nx] = J' diag(rho_c,k) J per stage (zero at k = 0)."""
    out = np.zeros((s.N + 1, s.nx, s.nx))
    lib().orc_contact_weight(ctypes.byref(_shape(s)), _d(_f64(J)), _d(_f64(rho_c)), _d(out))
    return out


def factor(s, A, B, c, q, r, rho, mu, settings: Optional[Settings] = None, qx=None, Qadd=None):
    """Riccati factor: returns (status, K [N,nu,nx], L [N,nu,nu], s [N,nx], P [N+1,nx,nx]).
    ``qx`` [nx]: joint-limit penalties added to the state weight; ``Qadd``
    [N+1, nx, nx]: per-stage additions to it (no-slip rows)."""
    st = settings or Settings.default()
    K = np.zeros((s.N, s.nu, s.nx))
    L = np.zeros((s.N, s.nu, s.nu))
    sv = np.zeros((s.N, s.nx))
    P = np.zeros((s.N + 1, s.nx, s.nx))
    status = lib().orc_factor(ctypes.byref(_shape(s)), ctypes.byref(st), _d(_f64(A)), _d(_f64(B)),
                              _d(_f64(c)), _d(_f64(q)), _d(_f64(r)), _d(_f64(rho)), float(mu),
                              _d(K), _d(L), _d(sv), _d(P), _d(None if qx is None else _f64(qx)),
                              _d(None if Qadd is None else _f64(Qadd)))
    return status, K, L, sv, P


def xupdate(s, A, B, c, K, L, sv, x0, qt, rt):
    """One back-sweep + rollout: returns (xt [N+1,nx], ut [N,nu])."""
    xt = np.zeros((s.N + 1, s.nx))
    ut = np.zeros((s.N, s.nu))
    lib().orc_xupdate(ctypes.byref(_shape(s)), _d(_f64(A)), _d(_f64(B)), _d(_f64(c)), _d(_f64(K)),
                      _d(_f64(L)), _d(_f64(sv)), _d(_f64(x0)), _d(_f64(qt)), _d(_f64(rt)),
                      _d(xt), _d(ut))
    return xt, ut


def residuals(s, A, B, c, q, r, x_ref, x0, tau_max, mu, stance, x, u, z, y, u_ref=None,
              settings: Optional[Settings] = None, x_lo=None, x_hi=None, zx=None, yx=None,
              J=None, zc=None, yc=None):
    """(res[4] = primal, dual, dynamics, complementarity; objective).  With joint
    limits (x_lo, x_hi [nx]) the state rows' (zx, yx) [N][nx] take part, with
    no-slip rows (J [nc, nx]) their (zc, yc) [N][nc]."""
    st = settings or Settings.default()
    res = np.zeros(4)
    obj = np.zeros(1)
    stance = np.ascontiguousarray(stance, dtype=np.uint8)
    lib().orc_residuals(ctypes.byref(_shape(s)), ctypes.byref(st), _d(_f64(A)), _d(_f64(B)),
                        _d(_f64(c)), _d(_f64(q)), _d(_f64(r)), _d(_f64(x_ref)),
                        _d(None if u_ref is None else _f64(u_ref)), _d(_f64(x0)),
                        _d(_f64(tau_max)), float(mu), stance.ctypes.data_as(_U8), _d(_f64(x)),
                        _d(_f64(u)), _d(_f64(z)), _d(_f64(y)), _d(res), _d(obj),
                        *_limits(x_lo, x_hi, zx, yx), *_contacts(J, zc, yc))
    return res, float(obj[0])


def _limits(x_lo, x_hi, zx, yx):
    if x_lo is None:
        return (None, None, None, None)
    return tuple(_d(_f64(v)) for v in (x_lo, x_hi, zx, yx))


def _contacts(J, zc, yc):
    if J is None:
        return (None, None, None)
    return tuple(_d(_f64(v)) for v in (J, zc, yc))


def solve(s, A, B, c, q, r, x_ref, x0, tau_max, mu, stance, *, iters=50, warm=None,
          u_ref=None, tol=1e-10, max_iters=1_000_000, settings: Optional[Settings] = None,
          x_lo=None, x_hi=None, J=None):
    """Solve one agent.  ``iters <= 0`` selects converge mode.

    ``warm`` is None (cold) or a tuple (u, z, y), followed by (zx, yx) with
    joint limits (x_lo, x_hi) and by (zc, yc) with no-slip rows (J [nc, nx]).
    Returns a dict with x, u, z, y, (zx, yx,) (zc, yc,) res, objective, status,
    iters.
    """
    st = settings or Settings.default()
    m = rows(s)
    x = np.zeros((s.N + 1, s.nx))
    if warm is None:
        u, z, y = np.zeros((s.N, s.nu)), np.zeros((s.N, m)), np.zeros((s.N, m))
    else:
        u, z, y = (np.array(v, dtype=np.float64, order="C").reshape(shp)
                   for v, shp in zip(warm[:3], ((s.N, s.nu), (s.N, m), (s.N, m))))
    zx = yx = None
    if x_lo is not None:
        if warm is None:
            zx, yx = np.zeros((s.N, s.nx)), np.zeros((s.N, s.nx))
        else:
            zx, yx = (np.array(v, dtype=np.float64, order="C").reshape(s.N, s.nx) for v in warm[3:5])
    zc = yc = None
    if J is not None:
        nc = contact_rows(s)
        if warm is None:
            zc, yc = np.zeros((s.N, nc)), np.zeros((s.N, nc))
        else:
            w0 = 5 if x_lo is not None else 3
            zc, yc = (np.array(v, dtype=np.float64, order="C").reshape(s.N, nc)
                      for v in warm[w0:w0 + 2])
    res = np.zeros(4)
    obj = np.zeros(1)
    it = ctypes.c_int(0)
    stance = np.ascontiguousarray(stance, dtype=np.uint8)
    status = lib().orc_solve(ctypes.byref(_shape(s)), ctypes.byref(st), _d(_f64(A)), _d(_f64(B)),
                             _d(_f64(c)), _d(_f64(q)), _d(_f64(r)), _d(_f64(x_ref)),
                             _d(None if u_ref is None else _f64(u_ref)), _d(_f64(x0)),
                             _d(_f64(tau_max)), float(mu), stance.ctypes.data_as(_U8), int(iters),
                             0 if warm is None else 1, float(tol), int(max_iters), _d(x), _d(u),
                             _d(z), _d(y), _d(res), _d(obj), ctypes.byref(it),
                             *_limits(x_lo, x_hi, zx, yx), *_contacts(J, zc, yc))
    out = dict(x=x, u=u, z=z, y=y, res=res, objective=float(obj[0]), status=status,
               iters=it.value)
    if x_lo is not None:
        out.update(zx=zx, yx=yx)
    if J is not None:
        out.update(zc=zc, yc=yc)
    return out


def agent(batch, a: int) -> dict:
    """Agent ``a`` of a ``synth.Batch`` as shaped FP64 arrays."""
    s = batch.shapes[a]
    o = batch.offsets()
    g = lambda k: np.asarray(getattr(batch, k)[o[k][a]:o[k][a + 1]], dtype=np.float64)
    return dict(s=s, A=g("A").reshape(s.N, s.nx, s.nx), B=g("B").reshape(s.N, s.nx, s.nu),
                c=g("c").reshape(s.N, s.nx), q=g("q"), r=g("r"),
                x_ref=g("x_ref").reshape(s.N + 1, s.nx), x0=g("x0"), tau_max=g("tau_max"),
                mu=float(batch.mu[a]),
                stance=np.asarray(batch.stance[o["stance"][a]:o["stance"][a + 1]],
                                  dtype=np.uint8).reshape(s.N, s.n_feet))


def _shapes_arr(batch) -> np.ndarray:
    return np.ascontiguousarray(np.array([s.as_tuple() for s in batch.shapes], dtype=np.int32)
                                .reshape(-1, 6))


def solve_batch(batch, *, iters=50, warm=None, x0=None, u_ref=None, n_threads=0,
                settings: Optional[Settings] = None, x_lo=None, x_hi=None, J=None) -> dict:
    """Fixed-iteration solve of every agent of a ``synth.Batch`` (flat layouts).

    ``warm`` is None or a dict with flat u, z, y (and zx, yx with joint limits,
    zc, yc with no-slip rows).  ``x0`` overrides batch.x0.  ``x_lo``/``x_hi``
    (flat, nx per agent): joint limits.  ``J`` (flat, n_feet*foot_dim x nx per
    agent): no-slip rows.  Returns flat x, u, z, y, (zx, yx,) (zc, yc,) res
    [n,4], objective [n], status [n], threads.
    """
    st = settings or Settings.default()
    o = batch.offsets()
    n = batch.n_agents
    x = np.zeros(int(o["x"][-1]))
    if warm is None:
        u, z, y = np.zeros(int(o["u"][-1])), np.zeros(int(o["z"][-1])), np.zeros(int(o["z"][-1]))
    else:
        u, z, y = (np.array(warm[k], dtype=np.float64) for k in ("u", "z", "y"))
    zx = yx = None
    if x_lo is not None:
        nzx = int(o["c"][-1])
        if warm is None:
            zx, yx = np.zeros(nzx), np.zeros(nzx)
        else:
            zx, yx = (np.array(warm[k], dtype=np.float64) for k in ("zx", "yx"))
    zc = yc = None
    if J is not None:
        nzc = sum(sh.N * sh.n_feet * sh.foot_dim for sh in batch.shapes)
        if warm is None:
            zc, yc = np.zeros(nzc), np.zeros(nzc)
        else:
            zc, yc = (np.array(warm[k], dtype=np.float64) for k in ("zc", "yc"))
    res = np.zeros((n, 4))
    obj = np.zeros(n)
    status = np.zeros(n, dtype=np.int32)
    shapes = _shapes_arr(batch)
    stance = np.ascontiguousarray(batch.stance, dtype=np.uint8)
    x0v = _f64(batch.x0 if x0 is None else x0)
    threads = lib().orc_solve_batch(
        n, shapes.ctypes.data_as(_I32), ctypes.byref(st), _d(_f64(batch.A)), _d(_f64(batch.B)),
        _d(_f64(batch.c)), _d(_f64(batch.q)), _d(_f64(batch.r)), _d(_f64(batch.x_ref)),
        _d(None if u_ref is None else _f64(u_ref)), _d(x0v), _d(_f64(batch.tau_max)),
        _d(_f64(batch.mu)), stance.ctypes.data_as(_U8), int(iters), 0 if warm is None else 1,
        _d(x), _d(u), _d(z), _d(y), _d(res), _d(obj), status.ctypes.data_as(_I32),
        int(n_threads), *_limits(x_lo, x_hi, zx, yx), *_contacts(J, zc, yc))
    out = dict(x=x, u=u, z=z, y=y, res=res, objective=obj, status=status, threads=threads)
    if x_lo is not None:
        out.update(zx=zx, yx=yx)
    if J is not None:
        out.update(zc=zc, yc=yc)
    return out


def advance_batch(batch, x0, u, noise) -> np.ndarray:
    """x0_next = A_0 x0 + B_0 u_0 + c_0 + noise for every agent (flat layouts)."""
    out = np.zeros_like(_f64(x0))
    shapes = _shapes_arr(batch)
    lib().orc_advance_batch(batch.n_agents, shapes.ctypes.data_as(_I32), _d(_f64(batch.A)),
                            _d(_f64(batch.B)), _d(_f64(batch.c)), _d(_f64(x0)), _d(_f64(u)),
                            _d(_f64(noise)), _d(out))
    return out
