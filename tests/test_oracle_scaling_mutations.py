"""The scaling pins catch plausible mistakes: each case plants one error in a
copy of oracle/scaling.py (a dropped square root, a transposed scale, a lost
cost factor, a wrong residual), loads it in place of the module, and checks
that at least one pin of tests/test_oracle_scaling.py fails."""
import importlib.util
import os
import sys

import pytest

import oracle
import test_oracle_scaling as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "scaling.py")

MUTANTS = [
    ("no square root in the column step", "Dx = Dx / np.sqrt(_limit(cx))", "Dx = Dx / _limit(cx)"),
    ("A scaled the wrong way round", 'out["A"] = ag["A"] * Dx[None, None, :] / Dx[None, :, None]',
     'out["A"] = ag["A"] * Dx[None, :, None] / Dx[None, None, :]'),
    ("B scaled by D on the wrong side", 'out["B"] = ag["B"] * Du[None, None, :] / Dx[None, :, None]',
     'out["B"] = ag["B"] * Du[None, None, :]'),
    ("cost scale missing on R", 'out["r"] = c * Du * Du * ag["r"]', 'out["r"] = Du * Du * ag["r"]'),
    ("y unscaled without the cost factor", "np.asarray(y).reshape(s.N, -1) * e / sc[\"c\"])",
     "np.asarray(y).reshape(s.N, -1) * e)"),
    ("friction coefficient not rescaled", 'out["mu"] = ag["mu"] * Du[b + 2] / Du[b]',
     'out["mu"] = ag["mu"]'),
    ("constraint rows ignored by the norms", "col = np.maximum(np.abs(Ph), np.maximum(Ah.max(axis=0), Ch.max(axis=0)))",
     "col = np.maximum(np.abs(Ph), Ah.max(axis=0))"),
    ("rho ratio inverted", "est = rho * np.sqrt(prim / max(dual, tiny))",
     "est = rho * np.sqrt(dual / max(prim, tiny))"),
    ("rho kept on a change", "return est if (est > tolerance * rho or est < rho / tolerance) else rho",
     "return rho"),
    ("threshold test inverted", "return est if (est > tolerance * rho or est < rho / tolerance) else rho",
     "return rho if (est > tolerance * rho or est < rho / tolerance) else est"),
]

CHECKS = [
    lambda: pins.test_scaled_problem_is_the_scaled_kkt(pins.tiny(), False),
    lambda: pins.test_scaled_problem_is_the_scaled_kkt(pins.synth.quadruped(2), True),
    lambda: pins.test_first_step_on_a_cost_dominated_problem(),
    lambda: pins.test_scaling_keeps_the_optimum(),
    lambda: pins.test_equilibration_reaches_its_fixed_point(),
    lambda: pins.test_rho_estimate_from_the_stacked_residuals(),
    lambda: pins.test_rho_update_rule(),
    lambda: pins.test_warm_start_round_trip(),
]


def _load(text):
    spec = importlib.util.spec_from_loader("oracle._scaling_mutant", loader=None)
    mod = importlib.util.module_from_spec(spec)
    mod.__package__ = "oracle"
    exec(compile(text, SRC, "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_scaling_pins_catch_mutant(name, old, new, monkeypatch):
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation site not unique/present: {name}"
    monkeypatch.setattr(pins, "scaling", _load(text.replace(old, new)))
    caught = False
    for chk in CHECKS:
        try:
            chk()
        except Exception:
            caught = True
            break
    assert caught, f"no pin failed for mutant: {name}"


def test_unmutated_copy_passes_every_check(monkeypatch):
    monkeypatch.setattr(pins, "scaling", _load(open(SRC).read()))
    for chk in CHECKS:
        chk()
