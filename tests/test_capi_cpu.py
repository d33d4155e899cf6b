"""C ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import pytest

from paper_2510_12717_amd import mpc
from paper_2510_12717_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    text = open(os.path.join(ROOT, "include", "mpc.h")).read()
    return sorted(set(re.findall(r"\b(mpc_[a-z_]+)\s*\(", text)))


def test_header_symbols_exported():
    L = mpc.lib()
    syms = header_symbols()
    assert "mpc_solve" in syms and "mpc_plan_create" in syms
    for s in syms:
        assert hasattr(L, s), s
    assert set(syms) == set(mpc.EXPORTS)


def test_version_and_defaults():
    L = mpc.lib()
    assert b"gfx950" in L.mpc_version()
    d = mpc.PlanDesc()
    L.mpc_plan_desc_default(ctypes.byref(d))
    assert (d.precision, d.admm_iters) == (1, 50)
    assert (d.rho, d.sigma, d.alpha, d.rho_eq_scale, d.rho_min) == (0.1, 1e-6, 1.6, 1e3, 1e-6)


def _create(**over):
    L = mpc.lib()
    shapes = over.pop("shapes", [synth.humanoid(10)] * 2)
    arr = (mpc.Shape * max(1, len(shapes)))(*[mpc.Shape(*s.as_tuple()) for s in shapes])
    d = mpc.PlanDesc()
    L.mpc_plan_desc_default(ctypes.byref(d))
    d.n_agents = len(shapes)
    d.shapes = ctypes.cast(arr, ctypes.POINTER(mpc.Shape))
    for k, v in over.items():
        setattr(d, k, v)
    h = ctypes.c_void_p()
    return L.mpc_plan_create(ctypes.byref(d), ctypes.byref(h)), L.mpc_last_error().decode()


@pytest.mark.parametrize("over,code", [
    (dict(n_agents=0), mpc.MPC_ERR_INVALID_ARG),
    (dict(precision=9), mpc.MPC_ERR_INVALID_ARG),
    (dict(admm_iters=0), mpc.MPC_ERR_INVALID_ARG),
    (dict(rho=0.0), mpc.MPC_ERR_INVALID_ARG),
    (dict(alpha=2.0), mpc.MPC_ERR_INVALID_ARG),
    (dict(rho_min=-1.0), mpc.MPC_ERR_INVALID_ARG),
    (dict(kernel=7), mpc.MPC_ERR_INVALID_ARG),
])
def test_invalid_descriptions_rejected(over, code):
    rc, msg = _create(**over)
    assert rc == code and msg


def test_unsupported_shapes_rejected():
    bad = synth.Shape.__new__(synth.Shape)
    object.__setattr__(bad, "N", 10)
    for k, v in dict(nx=65, nu=30, n_tau=18, n_feet=2, foot_dim=6).items():
        object.__setattr__(bad, k, v)
    rc, msg = _create(shapes=[synth.humanoid(10), bad])
    assert rc == mpc.MPC_ERR_UNSUPPORTED_SHAPE and "agent 1" in msg
    object.__setattr__(bad, "nx", 48)
    object.__setattr__(bad, "nu", 31)  # nu != n_tau + n_feet * foot_dim
    rc, _ = _create(shapes=[bad])
    assert rc == mpc.MPC_ERR_UNSUPPORTED_SHAPE


def test_null_arguments():
    L = mpc.lib()
    h = ctypes.c_void_p()
    assert L.mpc_plan_create(None, ctypes.byref(h)) == mpc.MPC_ERR_INVALID_ARG
    assert L.mpc_solve(None, None, None) == mpc.MPC_ERR_INVALID_ARG
    assert L.mpc_get_solution(None, None, None) == mpc.MPC_ERR_INVALID_ARG
    assert L.mpc_plan_destroy(None) == mpc.MPC_ERR_INVALID_ARG
