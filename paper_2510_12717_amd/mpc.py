"""ctypes binding of the C ABI in ``include/mpc.h`` (argument marshalling only).

Every step of the solve runs in the HIP library ``libmpc_hip.so``; PyTorch is
used here only to hold device memory and to name the stream.  If the library
is missing the binding raises -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmpc_hip.so")

MPC_OK, MPC_ERR_INVALID_ARG, MPC_ERR_OUT_OF_MEMORY, MPC_ERR_HIP = 0, 1, 2, 3
MPC_ERR_UNSUPPORTED_SHAPE, MPC_ERR_BUSY, MPC_ERR_NOT_READY = 4, 5, 6
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2, "fp16": 3, "fp32r": 4, "fp32mfma": 5}
AGENT_OK, AGENT_CONVERGED, AGENT_NOT_PD, AGENT_NONFINITE, AGENT_SUPERSEDED = 0, 1, 2, 3, 4


class MPCError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mpc error {code}: {msg}")
        self.code = code


class Shape(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("N", "nx", "nu", "n_tau", "n_feet", "foot_dim")]


class PlanDesc(ctypes.Structure):
    _fields_ = [("n_agents", ctypes.c_int32), ("shapes", ctypes.POINTER(Shape)),
                ("precision", ctypes.c_int32), ("admm_iters", ctypes.c_int32),
                ("rho", ctypes.c_double), ("sigma", ctypes.c_double), ("alpha", ctypes.c_double),
                ("rho_eq_scale", ctypes.c_double), ("rho_min", ctypes.c_double),
                ("max_refine_sweeps", ctypes.c_int32), ("refine_tol", ctypes.c_double),
                ("device", ctypes.c_int32), ("kernel", ctypes.c_int32),
                ("scaling_iters", ctypes.c_int32), ("rho_interval", ctypes.c_int32),
                ("rho_tolerance", ctypes.c_double), ("joint_limits", ctypes.c_int32),
                ("no_slip", ctypes.c_int32), ("inner_solve", ctypes.c_int32),
                ("riccati_scan", ctypes.c_int32)]


class ProblemBatch(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("A", "B", "c", "q_diag", "r_diag", "x_ref", "x0",
                                               "tau_max", "mu", "stance", "u_ref")] + \
               [("warm_start", ctypes.c_int32), ("x_lo", ctypes.c_void_p), ("x_hi", ctypes.c_void_p),
                ("J_foot", ctypes.c_void_p)]


class GroupInfo(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("family", "N", "nx", "nu", "n_feet", "n_agents",
                                              "threads", "lds_bytes")]


class ServerDesc(ctypes.Structure):
    _fields_ = [("solver", PlanDesc), ("hbm_budget_bytes", ctypes.c_int64),
                ("max_batch", ctypes.c_int32), ("max_inflight", ctypes.c_int32),
                ("supersede", ctypes.c_int32)]


class ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "submitted", "completed", "batches", "evictions", "pending", "inflight",
        "resident_controllers", "resident_bytes", "arena_bytes", "arena_free_bytes", "superseded")]


class ModelDesc(ctypes.Structure):
    _fields_ = [("n_bodies", ctypes.c_int32), ("n_feet", ctypes.c_int32),
                ("foot_dim", ctypes.c_int32), ("gravity", ctypes.c_double),
                ("parent", ctypes.c_void_p), ("joint_type", ctypes.c_void_p),
                ("axis", ctypes.c_void_p), ("offset", ctypes.c_void_p), ("mass", ctypes.c_void_p),
                ("com", ctypes.c_void_p), ("inertia", ctypes.c_void_p),
                ("armature", ctypes.c_void_p),
                ("foot_body", ctypes.c_void_p), ("foot_offset", ctypes.c_void_p)]


class Solution(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("u0", "x", "u", "z", "y", "objective",
                                               "residuals", "status", "zx", "yx", "zc", "yc", "zd",
                                               "yd")]


# every symbol the header declares
EXPORTS = ("mpc_plan_desc_default", "mpc_plan_create", "mpc_plan_destroy", "mpc_solve",
           "mpc_get_solution", "mpc_set_warm_state", "mpc_set_warm_limits", "mpc_set_warm_contacts",
           "mpc_set_warm_kkt",
           "mpc_advance_state", "mpc_plan_set_timing",
           "mpc_plan_get_timing", "mpc_plan_get_config", "mpc_plan_export_factor",
           "mpc_plan_get_rho", "mpc_plan_get_scaling", "mpc_plan_get_groups", "mpc_plan_autotune", "mpc_plan_capture", "mpc_plan_replay",
           "mpc_server_desc_default", "mpc_server_create", "mpc_server_destroy",
           "mpc_server_clock", "mpc_server_submit", "mpc_server_submit_many", "mpc_server_poll",
           "mpc_server_drain", "mpc_server_get_state", "mpc_server_get_stats",
           "mpc_solve_noalloc", "mpc_model_create", "mpc_model_destroy", "mpc_rnea",
           "mpc_linearize", "mpc_rti_torque", "mpc_last_error", "mpc_version")

_lib = None


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP solver library not built: {LIB_PATH} "
                               "(run `python -m paper_2510_12717_amd.build`)")
        L = ctypes.CDLL(LIB_PATH)
        P, V, I32 = ctypes.POINTER, ctypes.c_void_p, ctypes.c_int32
        L.mpc_plan_desc_default.argtypes = [P(PlanDesc)]
        L.mpc_plan_desc_default.restype = None
        L.mpc_plan_create.argtypes = [P(PlanDesc), P(V)]
        L.mpc_plan_destroy.argtypes = [V]
        L.mpc_solve.argtypes = [V, P(ProblemBatch), V]
        L.mpc_get_solution.argtypes = [V, P(Solution), V]
        L.mpc_set_warm_state.argtypes = [V, V, V, V, V]
        L.mpc_set_warm_limits.argtypes = [V, V, V, V]
        L.mpc_set_warm_contacts.argtypes = [V, V, V, V]
        L.mpc_set_warm_kkt.argtypes = [V, V, V, V, V]
        L.mpc_advance_state.argtypes = [V, P(ProblemBatch), V, V, V]
        L.mpc_plan_set_timing.argtypes = [V, I32]
        L.mpc_plan_get_timing.argtypes = [V, P(ctypes.c_double), P(ctypes.c_int64)]
        L.mpc_plan_get_config.argtypes = [V, P(I32), P(I32), P(I32)]
        L.mpc_plan_export_factor.argtypes = [V, I32, V, V, V, V, V]
        L.mpc_plan_get_rho.argtypes = [V, V, P(I32), V]
        L.mpc_plan_get_scaling.argtypes = [V, V, V]
        L.mpc_plan_get_groups.argtypes = [V, P(GroupInfo), I32, P(I32)]
        L.mpc_plan_autotune.argtypes = [V, P(ProblemBatch), I32, V]
        L.mpc_plan_capture.argtypes = [V, P(ProblemBatch), V, V]
        L.mpc_plan_replay.argtypes = [V, V]
        D = ctypes.c_double
        L.mpc_server_desc_default.argtypes = [P(ServerDesc)]
        L.mpc_server_desc_default.restype = None
        L.mpc_server_create.argtypes = [P(ServerDesc), P(V)]
        L.mpc_server_destroy.argtypes = [V]
        L.mpc_server_clock.argtypes = [V]
        L.mpc_server_clock.restype = D
        L.mpc_server_submit.argtypes = [V, ctypes.c_int64, P(Shape), P(ProblemBatch), V, V, D,
                                        P(ctypes.c_int64)]
        L.mpc_server_submit_many.argtypes = [V, I32, V, V, V, V, V, V, V]
        L.mpc_server_poll.argtypes = [V, V, V, I32, P(I32)]
        L.mpc_server_drain.argtypes = [V]
        L.mpc_server_get_state.argtypes = [V, ctypes.c_int64, V, V, V, V, V]
        L.mpc_server_get_stats.argtypes = [V, P(ServerStats)]
        L.mpc_solve_noalloc.argtypes = [P(PlanDesc), P(ProblemBatch), P(Solution), V]
        L.mpc_solve_noalloc.restype = ctypes.c_int
        L.mpc_model_create.argtypes = [P(ModelDesc), I32, P(V)]
        L.mpc_model_destroy.argtypes = [V]
        L.mpc_rnea.argtypes = [V, I32, V, V, V, V, V, V]
        L.mpc_linearize.argtypes = [V, I32, I32, D, I32, V, V, V, V, V, V, V, V]
        L.mpc_rti_torque.argtypes = [V, I32, I32, D, D, D, I32, V, V, V, V, V]
        for f in ("mpc_model_create", "mpc_model_destroy", "mpc_rnea", "mpc_linearize",
                  "mpc_rti_torque"):
            getattr(L, f).restype = ctypes.c_int
        for f in ("mpc_server_create", "mpc_server_destroy", "mpc_server_submit",
                  "mpc_server_submit_many", "mpc_server_poll", "mpc_server_drain",
                  "mpc_server_get_state", "mpc_server_get_stats"):
            getattr(L, f).restype = ctypes.c_int
        for f in ("mpc_plan_create", "mpc_plan_destroy", "mpc_solve", "mpc_get_solution",
                  "mpc_set_warm_state", "mpc_set_warm_limits", "mpc_set_warm_contacts",
                  "mpc_set_warm_kkt", "mpc_advance_state",
                  "mpc_plan_set_timing",
                  "mpc_plan_get_timing", "mpc_plan_get_config", "mpc_plan_export_factor",
                  "mpc_plan_get_rho", "mpc_plan_get_scaling",
                  "mpc_plan_get_groups", "mpc_plan_autotune", "mpc_plan_capture",
                  "mpc_plan_replay"):
            getattr(L, f).restype = ctypes.c_int
        L.mpc_last_error.restype = ctypes.c_char_p
        L.mpc_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(code: int):
    if code != MPC_OK:
        raise MPCError(code, lib().mpc_last_error().decode())


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return t.data_ptr()


def _stream_handle(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def to_device(batch, dtype: str = "fp32", device: str = "cuda") -> Dict[str, "object"]:
    """Copy a ``synth.Batch`` to device tensors in the plan's io type."""
    import torch
    td = torch.float64 if dtype == "fp64" else torch.float32
    out = {}
    for k in ("A", "B", "c", "q", "r", "x_ref", "x0", "tau_max", "mu"):
        out[k] = torch.from_numpy(np.ascontiguousarray(getattr(batch, k))).to(device=device,
                                                                               dtype=td)
    out["stance"] = torch.from_numpy(np.ascontiguousarray(batch.stance, dtype=np.uint8)).to(device)
    return out


class Plan:
    """A solver plan for a fixed batch of agent shapes (see ``mpc_plan_create``)."""

    def __init__(self, shapes: Sequence, precision: str = "fp32", iters: int = 50,
                 device: int = 0, kernel: str = "auto", **consts):
        L = lib()
        self.shapes = list(shapes)
        self.precision = precision
        arr = (Shape * len(self.shapes))(*[Shape(*s.as_tuple()) for s in self.shapes])
        self._shapes_arr = arr
        d = PlanDesc()
        L.mpc_plan_desc_default(ctypes.byref(d))
        d.n_agents = len(self.shapes)
        d.shapes = ctypes.cast(arr, ctypes.POINTER(Shape))
        d.precision = PRECISIONS[precision]
        d.admm_iters = int(iters)
        d.device = int(device)
        d.kernel = {"auto": 0, "generic": 1, "fused": 2, "persistent": 3}[kernel]
        for k, v in consts.items():
            setattr(d, k, v)
        h = ctypes.c_void_p()
        _check(L.mpc_plan_create(ctypes.byref(d), ctypes.byref(h)))
        self._h = h
        self.n = len(self.shapes)
        self.dtype = "fp64" if precision == "fp64" else "fp32"  # io type
        m = [s.nu + 4 * s.n_feet for s in self.shapes]
        self.limits = bool(consts.get("joint_limits", 0))
        self.contacts = bool(consts.get("no_slip", 0))
        self.kkt = bool(consts.get("inner_solve", 0))
        self.sizes = dict(x=sum((s.N + 1) * s.nx for s in self.shapes),
                          zx=sum(s.N * s.nx for s in self.shapes),
                          zc=sum(s.N * s.n_feet * s.foot_dim for s in self.shapes),
                          u=sum(s.N * s.nu for s in self.shapes),
                          z=sum(s.N * mm for s, mm in zip(self.shapes, m)),
                          u0=sum(s.nu for s in self.shapes))

    def close(self):
        if getattr(self, "_h", None):
            _check(lib().mpc_plan_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _batch(self, prob, warm_start: bool) -> ProblemBatch:
        b = ProblemBatch()
        b.A, b.B, b.c = _ptr(prob["A"]), _ptr(prob["B"]), _ptr(prob["c"])
        b.q_diag, b.r_diag = _ptr(prob["q"]), _ptr(prob["r"])
        b.x_ref, b.x0 = _ptr(prob["x_ref"]), _ptr(prob["x0"])
        b.tau_max, b.mu, b.stance = _ptr(prob["tau_max"]), _ptr(prob["mu"]), _ptr(prob["stance"])
        b.u_ref = _ptr(prob.get("u_ref"))
        b.x_lo, b.x_hi = _ptr(prob.get("x_lo")), _ptr(prob.get("x_hi"))
        b.J_foot = _ptr(prob.get("J_foot"))
        b.warm_start = 1 if warm_start else 0
        self._keep = prob  # inputs must outlive the stream's use of them
        return b

    def solve(self, prob, warm_start: bool = False, stream=None):
        b = self._batch(prob, warm_start)
        _check(lib().mpc_solve(self._h, ctypes.byref(b), _stream_handle(stream)))

    def get_solution(self, stream=None, out=None) -> Dict[str, "object"]:
        import torch
        td = torch.float64 if self.dtype == "fp64" else torch.float32
        dev = torch.device("cuda", torch.cuda.current_device())
        if out is None:
            out = dict(u0=torch.empty(self.sizes["u0"], dtype=td, device=dev),
                       x=torch.empty(self.sizes["x"], dtype=td, device=dev),
                       u=torch.empty(self.sizes["u"], dtype=td, device=dev),
                       z=torch.empty(self.sizes["z"], dtype=td, device=dev),
                       y=torch.empty(self.sizes["z"], dtype=td, device=dev),
                       objective=torch.empty(self.n, dtype=td, device=dev),
                       residuals=torch.empty((self.n, 4), dtype=torch.float64, device=dev),
                       status=torch.empty(self.n, dtype=torch.int32, device=dev))
            if self.limits:
                out["zx"] = torch.empty(self.sizes["zx"], dtype=td, device=dev)
                out["yx"] = torch.empty(self.sizes["zx"], dtype=td, device=dev)
            if self.contacts:
                out["zc"] = torch.empty(self.sizes["zc"], dtype=td, device=dev)
                out["yc"] = torch.empty(self.sizes["zc"], dtype=td, device=dev)
            if self.kkt:
                out["zd"] = torch.empty(self.sizes["zx"], dtype=td, device=dev)
                out["yd"] = torch.empty(self.sizes["zx"], dtype=td, device=dev)
        s = Solution()
        for k in ("u0", "x", "u", "z", "y", "objective", "residuals", "status", "zx", "yx", "zc", "yc",
                  "zd", "yd"):
            setattr(s, k, _ptr(out.get(k)))
        _check(lib().mpc_get_solution(self._h, ctypes.byref(s), _stream_handle(stream)))
        return out

    def set_warm_state(self, u, z, y, stream=None):
        _check(lib().mpc_set_warm_state(self._h, _ptr(u), _ptr(z), _ptr(y),
                                        _stream_handle(stream)))

    def set_warm_limits(self, zx, yx, stream=None):
        _check(lib().mpc_set_warm_limits(self._h, _ptr(zx), _ptr(yx), _stream_handle(stream)))

    def set_warm_kkt(self, x, zd, yd, stream=None):
        _check(lib().mpc_set_warm_kkt(self._h, _ptr(x), _ptr(zd), _ptr(yd), _stream_handle(stream)))

    def set_warm_contacts(self, zc, yc, stream=None):
        _check(lib().mpc_set_warm_contacts(self._h, _ptr(zc), _ptr(yc), _stream_handle(stream)))

    def advance_state(self, prob, noise, x0_next, stream=None):
        b = self._batch(prob, False)
        _check(lib().mpc_advance_state(self._h, ctypes.byref(b), _ptr(noise), _ptr(x0_next),
                                       _stream_handle(stream)))

    def set_timing(self, enable: bool = True):
        _check(lib().mpc_plan_set_timing(self._h, 1 if enable else 0))

    def get_timing(self):
        ms = (ctypes.c_double * 3)()
        n = (ctypes.c_int64 * 3)()
        _check(lib().mpc_plan_get_timing(self._h, ms, n))
        names = ("factor", "admm", "residual")
        return {k: (ms[i], n[i]) for i, k in enumerate(names)}

    def config(self):
        k, t, l = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().mpc_plan_get_config(self._h, ctypes.byref(k), ctypes.byref(t),
                                         ctypes.byref(l)))
        return dict(kernel={1: "generic", 2: "fused", 3: "generic+fused",
                            4: "mixed_precision"}.get(k.value, str(k.value)),
                    threads_per_agent=t.value, lds_bytes=l.value)

    def groups(self):
        """Launch groups: list of dicts (family 'generic' | 'fused', N, nx, nu, n_feet,
        n_agents, threads, lds_bytes)."""
        n = ctypes.c_int32()
        _check(lib().mpc_plan_get_groups(self._h, None, 0, ctypes.byref(n)))
        arr = (GroupInfo * max(n.value, 1))()
        _check(lib().mpc_plan_get_groups(self._h, arr, n.value, ctypes.byref(n)))
        out = []
        for g in arr[:n.value]:
            d = {f: getattr(g, f) for f, _ in GroupInfo._fields_}
            d["family"] = {1: "generic", 2: "fused", 4: "mixed_precision"}[g.family]
            out.append(d)
        return out

    def autotune(self, prob, reps: int = 3, stream=None):
        b = self._batch(prob, False)
        _check(lib().mpc_plan_autotune(self._h, ctypes.byref(b), int(reps),
                                       _stream_handle(stream)))
        return self.groups()

    def capture(self, prob, warm_start: bool = True, noise=None, x0_next=None):
        """Capture solve (+ plant step when x0_next is given) into the plan's graph."""
        b = self._batch(prob, warm_start)
        self._graph_keep = (prob, noise, x0_next)
        _check(lib().mpc_plan_capture(self._h, ctypes.byref(b), _ptr(noise), _ptr(x0_next)))

    def replay(self, stream=None):
        _check(lib().mpc_plan_replay(self._h, _stream_handle(stream)))

    def get_rho(self, stream=None):
        """The rho every agent ran each segment of the last solve with, [n][segments]
        (plans with rho_interval > 0)."""
        import torch
        ns = ctypes.c_int32()
        _check(lib().mpc_plan_get_rho(self._h, None, ctypes.byref(ns), None))
        out = torch.empty((self.n, ns.value), dtype=torch.float64,
                          device=torch.device("cuda", torch.cuda.current_device()))
        _check(lib().mpc_plan_get_rho(self._h, _ptr(out), None, _stream_handle(stream)))
        return out

    def get_scaling(self, stream=None):
        """Every agent's scale record [n][128] (D_x at 0.., D_u at 64.., cost factor at 96)."""
        import torch
        out = torch.empty((self.n, 128), dtype=torch.float64,
                          device=torch.device("cuda", torch.cuda.current_device()))
        _check(lib().mpc_plan_get_scaling(self._h, _ptr(out), _stream_handle(stream)))
        return out

    def export_factor(self, agent: int, stream=None):
        """(K, A_cl, Hinv, s) of one agent from the last solve (generic kernels only)."""
        import torch
        td = torch.float64 if self.dtype == "fp64" else torch.float32
        sh = self.shapes[agent]
        dev = torch.device("cuda", torch.cuda.current_device())
        K = torch.empty((sh.N, sh.nu, sh.nx), dtype=td, device=dev)
        Acl = torch.empty((sh.N, sh.nx, sh.nx), dtype=td, device=dev)
        Hi = torch.empty((sh.N, sh.nu, sh.nu), dtype=td, device=dev)
        sv = torch.empty((sh.N, sh.nx), dtype=td, device=dev)
        _check(lib().mpc_plan_export_factor(self._h, int(agent), _ptr(K), _ptr(Acl), _ptr(Hi),
                                            _ptr(sv), _stream_handle(stream)))
        return K, Acl, Hi, sv


def solution_buffers(shapes, dtype: str = "fp32") -> Dict[str, "object"]:
    """Device tensors for the solution of a batch of ``shapes`` (the caller's
    buffers of ``mpc_get_solution`` / ``mpc_solve_noalloc``)."""
    import torch
    td = torch.float64 if dtype == "fp64" else torch.float32
    dev = torch.device("cuda", torch.cuda.current_device())
    n = len(shapes)
    nx = sum((s.N + 1) * s.nx for s in shapes)
    nu = sum(s.N * s.nu for s in shapes)
    nz = sum(s.N * (s.nu + 4 * s.n_feet) for s in shapes)
    return dict(u0=torch.empty(sum(s.nu for s in shapes), dtype=td, device=dev),
                x=torch.empty(nx, dtype=td, device=dev), u=torch.empty(nu, dtype=td, device=dev),
                z=torch.empty(nz, dtype=td, device=dev), y=torch.empty(nz, dtype=td, device=dev),
                objective=torch.empty(n, dtype=td, device=dev),
                residuals=torch.empty((n, 4), dtype=torch.float64, device=dev),
                status=torch.empty(n, dtype=torch.int32, device=dev))


def solve_noalloc(shapes: Sequence, prob, out, warm_start: bool = False, iters: int = 50,
                  device: int = 0, stream=None, **consts):
    """``mpc_solve_noalloc``: FP32 solve of a one-shape batch with no plan and no
    device allocation; ``out`` (see ``solution_buffers``) holds the iterate and,
    with ``warm_start``, the start."""
    L = lib()
    arr = (Shape * len(shapes))(*[Shape(*s.as_tuple()) for s in shapes])
    d = PlanDesc()
    L.mpc_plan_desc_default(ctypes.byref(d))
    d.n_agents = len(shapes)
    d.shapes = ctypes.cast(arr, ctypes.POINTER(Shape))
    d.precision = PRECISIONS["fp32"]
    d.admm_iters = int(iters)
    d.device = int(device)
    for k, v in consts.items():
        setattr(d, k, v)
    b = ProblemBatch()
    b.A, b.B, b.c = _ptr(prob["A"]), _ptr(prob["B"]), _ptr(prob["c"])
    b.q_diag, b.r_diag = _ptr(prob["q"]), _ptr(prob["r"])
    b.x_ref, b.x0 = _ptr(prob["x_ref"]), _ptr(prob["x0"])
    b.tau_max, b.mu, b.stance = _ptr(prob["tau_max"]), _ptr(prob["mu"]), _ptr(prob["stance"])
    b.u_ref = _ptr(prob.get("u_ref"))
    b.warm_start = 1 if warm_start else 0
    s = Solution()
    for k in ("u0", "x", "u", "z", "y", "objective", "residuals", "status"):
        setattr(s, k, _ptr(out.get(k)))
    _check(L.mpc_solve_noalloc(ctypes.byref(d), ctypes.byref(b), ctypes.byref(s),
                               _stream_handle(stream)))
    return out


def agent_problems(prob, batch, agents=None):
    """Per-agent ``ProblemBatch`` records pointing into a device-resident batch
    (``to_device`` output) -- the request data of a served controller."""
    import torch
    off = batch.offsets()
    esz = prob["A"].element_size()
    agents = range(batch.n_agents) if agents is None else agents
    arr = (ProblemBatch * len(list(agents)))()
    base = {k: prob[k].data_ptr() for k in ("A", "B", "c", "q", "r", "x_ref", "x0", "tau_max",
                                            "mu", "stance")}
    for j, a in enumerate(agents):
        b = arr[j]
        at = lambda k, key=None: int(base[k] + int(off[key or k][a]) * esz)
        b.A, b.B, b.c = at("A"), at("B"), at("c")
        b.q_diag, b.r_diag = at("q"), at("r")
        b.x_ref, b.x0, b.tau_max = at("x_ref"), at("x0"), at("tau_max")
        b.mu = int(base["mu"] + int(a) * esz)
        b.stance = int(base["stance"] + int(off["stance"][a]))
        b.u_ref = None
        b.warm_start = 1
    return arr


class Server:
    """Served request loop (see ``mpc_server_create``)."""

    def __init__(self, precision: str = "fp32", iters: int = 50, hbm_budget_bytes: int = 1 << 30,
                 max_batch: int = 4096, max_inflight: int = 3, device: int = 0,
                 supersede: bool = False, **consts):
        L = lib()
        d = ServerDesc()
        L.mpc_server_desc_default(ctypes.byref(d))
        d.solver.precision = PRECISIONS[precision]
        d.solver.admm_iters = int(iters)
        d.solver.device = int(device)
        for k, v in consts.items():
            setattr(d.solver, k, v)
        d.hbm_budget_bytes = int(hbm_budget_bytes)
        d.max_batch = int(max_batch)
        d.max_inflight = int(max_inflight)
        d.supersede = 1 if supersede else 0
        h = ctypes.c_void_p()
        _check(L.mpc_server_create(ctypes.byref(d), ctypes.byref(h)))
        self._h = h
        self.dtype = "fp64" if precision == "fp64" else "fp32"
        self._keep = []

    def close(self):
        if getattr(self, "_h", None):
            _check(lib().mpc_server_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def clock(self) -> float:
        return lib().mpc_server_clock(self._h)

    def submit(self, ctrl: int, shape, problem: "ProblemBatch", u0_out, warm: bool = True,
               status_out=None, t_arrival: Optional[float] = None) -> int:
        problem.warm_start = 1 if warm else 0
        sh = Shape(*shape.as_tuple())
        t = ctypes.c_int64()
        ta = self.clock() if t_arrival is None else float(t_arrival)
        _check(lib().mpc_server_submit(self._h, int(ctrl), ctypes.byref(sh), ctypes.byref(problem),
                                       _ptr(u0_out), _ptr(status_out), ta, ctypes.byref(t)))
        return t.value

    def submit_many(self, ctrls: np.ndarray, shapes, problems, u0_ptrs: np.ndarray,
                    t_arrival: np.ndarray, status_ptrs: Optional[np.ndarray] = None) -> np.ndarray:
        """Bulk submission: ``shapes``/``problems`` hold one Shape / ProblemBatch
        record per request (ctypes arrays, or numpy arrays of the raw records),
        ``u0_ptrs`` (and optionally ``status_ptrs``) device addresses (uint64)."""
        n = len(ctrls)
        ctrls = np.ascontiguousarray(ctrls, dtype=np.int64)
        u0 = np.ascontiguousarray(u0_ptrs, dtype=np.uint64)
        ta = np.ascontiguousarray(t_arrival, dtype=np.float64)
        st = None if status_ptrs is None else np.ascontiguousarray(status_ptrs, dtype=np.uint64)
        tk = np.empty(n, dtype=np.int64)
        addr = lambda a: a.ctypes.data if isinstance(a, np.ndarray) else ctypes.addressof(a)
        _check(lib().mpc_server_submit_many(self._h, n, ctrls.ctypes.data, addr(shapes),
                                            addr(problems), u0.ctypes.data,
                                            None if st is None else st.ctypes.data,
                                            ta.ctypes.data, tk.ctypes.data))
        return tk

    def poll(self, cap: int = 1 << 16):
        tk = np.empty(cap, dtype=np.int64)
        tm = np.empty(cap, dtype=np.float64)
        n = ctypes.c_int32()
        _check(lib().mpc_server_poll(self._h, tk.ctypes.data, tm.ctypes.data, cap, ctypes.byref(n)))
        return tk[:n.value], tm[:n.value]

    def drain(self):
        _check(lib().mpc_server_drain(self._h))

    def get_state(self, ctrl: int, shape, stream=None):
        import torch
        td = torch.float64 if self.dtype == "fp64" else torch.float32
        m = shape.nu + 4 * shape.n_feet
        dev = torch.device("cuda", torch.cuda.current_device())
        out = dict(x=torch.empty((shape.N + 1) * shape.nx, dtype=td, device=dev),
                   u=torch.empty(shape.N * shape.nu, dtype=td, device=dev),
                   z=torch.empty(shape.N * m, dtype=td, device=dev),
                   y=torch.empty(shape.N * m, dtype=td, device=dev))
        _check(lib().mpc_server_get_state(self._h, int(ctrl), _ptr(out["x"]), _ptr(out["u"]),
                                          _ptr(out["z"]), _ptr(out["y"]), _stream_handle(stream)))
        return out

    def stats(self):
        st = ServerStats()
        _check(lib().mpc_server_get_stats(self._h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}


class RobotModel:
    """A kinematic tree on the device (``mpc_model_create``) with the real-time
    iteration's front and back end: ``rnea`` (Eq. (rnea)), ``linearize``
    (f_KKT of Alg. 1: A_k, B_k, c_k of the semi-implicit Euler step about a
    trajectory) and ``rti_torque`` (f_RNEA and Eq. (mpc_torque)).  ``model`` is
    a dict with the fields of ``synth.articulated_model``; arrays are FP64 device
    tensors."""

    def __init__(self, model, device: int = 0):
        L = lib()
        n = int(model["n"])
        self.n = n
        self.n_feet = len(model["foot_body"])
        self.foot_dim = int(model["foot_dim"])
        self.nx = 2 * n
        self.nj = n - 6
        self.nu = self.nj + self.n_feet * self.foot_dim
        f64 = lambda a, k: np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1, k))
        i32 = lambda a: np.ascontiguousarray(np.asarray(a, dtype=np.int32).reshape(-1))
        self._keep = dict(parent=i32(model["parent"]), jtype=i32(model["jtype"]),
                          axis=f64(model["axis"], 3), offset=f64(model["offset"], 3),
                          mass=f64(model["mass"], 1), com=f64(model["com"], 3),
                          inertia=f64(model["inertia"], 3),
                          armature=f64(model.get("armature", np.zeros(n)), 1),
                          foot_body=i32(model["foot_body"]),
                          foot_offset=f64(model["foot_offset"], 3))
        k = self._keep
        d = ModelDesc()
        d.n_bodies, d.n_feet, d.foot_dim = n, self.n_feet, self.foot_dim
        d.gravity = float(model["gravity"])
        d.parent, d.joint_type = k["parent"].ctypes.data, k["jtype"].ctypes.data
        d.axis, d.offset, d.mass = k["axis"].ctypes.data, k["offset"].ctypes.data, k["mass"].ctypes.data
        d.com, d.inertia = k["com"].ctypes.data, k["inertia"].ctypes.data
        d.armature = k["armature"].ctypes.data
        d.foot_body = k["foot_body"].ctypes.data if self.n_feet else None
        d.foot_offset = k["foot_offset"].ctypes.data if self.n_feet else None
        h = ctypes.c_void_p()
        _check(L.mpc_model_create(ctypes.byref(d), int(device), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _check(lib().mpc_model_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def rnea(self, q, qd, qdd, F=None, stream=None):
        import torch
        tau = torch.empty_like(q)
        _check(lib().mpc_rnea(self._h, int(q.shape[0]), _ptr(q), _ptr(qd), _ptr(qdd), _ptr(F),
                              _ptr(tau), _stream_handle(stream)))
        return tau

    def linearize(self, x, u, dt: float, out=None, J_foot=None, stream=None):
        """x [n_agents, N + 1, nx] (x_N unused) and u [n_agents, N, nu], the
        solution's layouts, float64 or float32 -> A, B, c (same dtype), status.
        ``out``: optional (A, B, c) tensors to write into (e.g. a batch's);
        ``J_foot``: optional tensor [n_agents * n_feet * foot_dim * nx] that
        receives the no-slip rows at x_0."""
        import torch
        na, N = int(x.shape[0]), int(u.shape[1])
        if tuple(x.shape[1:]) != (N + 1, self.nx) or tuple(u.shape[1:]) != (N, self.nu):
            raise ValueError("x must be [n, N+1, nx] and u [n, N, nu]")
        prec = _io_precision(x, u)
        dev = x.device
        if out is None:
            A = torch.empty((na, N, self.nx, self.nx), dtype=x.dtype, device=dev)
            B = torch.empty((na, N, self.nx, self.nu), dtype=x.dtype, device=dev)
            c = torch.empty((na, N, self.nx), dtype=x.dtype, device=dev)
        else:
            A, B, c = out
            for t, k in ((A, na * N * self.nx * self.nx), (B, na * N * self.nx * self.nu),
                         (c, na * N * self.nx)):
                if t.dtype != x.dtype or t.numel() != k or not t.is_contiguous():
                    raise ValueError("out tensors must match the shapes and dtype")
        if J_foot is not None and (J_foot.dtype != x.dtype or not J_foot.is_contiguous() or
                                   J_foot.numel() != na * self.n_feet * self.foot_dim * self.nx):
            raise ValueError("J_foot must hold n_agents * n_feet * foot_dim * nx of x's dtype")
        status = torch.zeros(na, dtype=torch.int32, device=dev)
        _check(lib().mpc_linearize(self._h, na, N, float(dt), prec, _ptr(x), _ptr(u), _ptr(A),
                                   _ptr(B), _ptr(c), _ptr(J_foot), _ptr(status),
                                   _stream_handle(stream)))
        return A, B, c, status

    def rti_torque(self, dt: float, kp: float, kd: float, x, u, x_meas, stream=None):
        """x [count, N + 1, nx], u [count, N, nu] (a solution), measured state
        x_meas [count, nx] -> joint torques [count, n - 6] (same dtype)."""
        import torch
        cnt, N = int(x.shape[0]), int(u.shape[1])
        if (tuple(x.shape[1:]) != (N + 1, self.nx) or tuple(u.shape[1:]) != (N, self.nu)
                or tuple(x_meas.shape) != (cnt, self.nx)):
            raise ValueError("x must be [n, N+1, nx], u [n, N, nu] and x_meas [n, nx]")
        prec = _io_precision(x, u, x_meas)
        tau = torch.empty((cnt, self.nj), dtype=x.dtype, device=x.device)
        _check(lib().mpc_rti_torque(self._h, cnt, N, float(dt), float(kp), float(kd), prec, _ptr(x),
                                    _ptr(u), _ptr(x_meas), _ptr(tau), _stream_handle(stream)))
        return tau


def _io_precision(*ts):
    import torch
    dt = ts[0].dtype
    if any(t.dtype != dt or not t.is_contiguous() for t in ts):
        raise ValueError("arrays must be contiguous and share one dtype")
    if dt == torch.float64:
        return PRECISIONS["fp64"]
    if dt == torch.float32:
        return PRECISIONS["fp32"]
    raise ValueError("float64 or float32 arrays")
