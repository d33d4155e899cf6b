"""The pins catch plausible mistakes: each case plants one error in a copy of
the oracle's C source (a dropped term, a wrong sign or index, a transposed
operand), builds it, and checks that at least one pin fails."""
import os
import shutil
import tempfile

import pytest

import oracle
import test_oracle_contacts as contacts
import test_oracle_limits as limits
import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "mpc_oracle.c")

# (name, text in the source, replacement)
MUTANTS = [
    ("drop s_k in back-sweep", "pp[i] = p[i] + sv[(size_t)k * nx + i];", "pp[i] = p[i];"),
    ("transposed A in back-sweep", "acc += Ak[t * nx + i] * pp[t];", "acc += Ak[i * nx + t] * pp[t];"),
    ("wrong sign of d", "for (int j = 0; j < nu; ++j) dk[j] = -hv[j];",
     "for (int j = 0; j < nu; ++j) dk[j] = hv[j];"),
    ("K' h dropped from p", "for (int t = 0; t < nu; ++t) acc += Kk[t * nx + i] * hv[t];", ""),
    ("sigma sign in qt", "x_ref[(size_t)k * nx + i] - sigma * x[(size_t)k * nx + i];",
     "x_ref[(size_t)k * nx + i] + sigma * x[(size_t)k * nx + i];"),
    ("dual update sign", "y[idx] = y[idx] + rho[idx] * (w - zn);", "y[idx] = y[idx] - rho[idx] * (w - zn);"),
    ("no relaxation of z", "const double w = alpha * zeta + (1.0 - alpha) * z[idx];",
     "const double w = zeta;"),
    ("rho_eq not applied", "rr = st->rho_eq_scale * st->rho;", "rr = st->rho;"),
    ("pyramid facet sign", "C[(p + 1) * nu + fx] = -1.0;", "C[(p + 1) * nu + fx] = 1.0;"),
    ("G'K dropped from P", "for (int t = 0; t < nu; ++t) acc += G[t * nx + i] * Kk[t * nx + j];", ""),
    ("P_{k+1} c instead of c in s", "acc += Pn[i * nx + t] * ck[t];", "acc += Pn[i * nx + t] * ck[i];"),
    ("dual residual sign", "for (int row = 0; row < m; ++row) acc += C[row * nu + j] * yk[row];",
     "for (int row = 0; row < m; ++row) acc -= C[row * nu + j] * yk[row];"),
    ("plant step without c_0", "double acc = c[o[a].c + i] + noise[o[a].x0 + i];",
     "double acc = noise[o[a].x0 + i];"),
    ("plant step with A_0 transposed", "acc += A0[i * nx + t] * x0[o[a].x0 + t];",
     "acc += A0[t * nx + i] * x0[o[a].x0 + t];"),
    ("complementarity signs swapped", "const double yp = yy > 0.0 ? yy : 0.0, ym = yy < 0.0 ? -yy : 0.0;",
     "const double yp = yy < 0.0 ? -yy : 0.0, ym = yy > 0.0 ? yy : 0.0;"),
    ("complementarity without the lower bound", "const double b = isinf(lo) ? ym : fmin(ym, zz - lo);",
     "const double b = 0.0;"),
    ("complementarity against the wrong bound", "const double a = isinf(hi) ? yp : fmin(yp, hi - zz);",
     "const double a = isinf(lo) ? yp : fmin(yp, zz - lo);"),
    ("state penalty missing from P_N",
     "Pn[i * nx + j] = ((i == j) ? q[i] + st->sigma + (qx ? qx[i] : 0.0) : 0.0) +",
     "Pn[i * nx + j] = ((i == j) ? q[i] + st->sigma : 0.0) +"),
    ("state rows' linear term with the wrong sign",
     "if (x_lo && k >= 1) acc += yx[(size_t)(k - 1) * nx + i] -",
     "if (x_lo && k >= 1) acc += -yx[(size_t)(k - 1) * nx + i] -"),
    ("state rows projected on the wrong stage",
     "const double w = alpha * xt[(size_t)k * nx + i] + (1.0 - alpha) * zx[idx];",
     "const double w = alpha * xt[(size_t)(k - 1) * nx + i] + (1.0 - alpha) * zx[idx];"),
    ("state multipliers left out of the costates", "      if (x_lo) acc += yx[(size_t)(k - 1) * nx + i];\n", ""),
    ("state rows left out of the primal residual",
     "rp = maxabs(x[(size_t)(k + 1) * nx + i] - zx[idx], rp);", ""),
    ("equality state rows with the inequality penalty", "      rho_x[i] = st->rho_eq_scale * st->rho;",
     "      rho_x[i] = st->rho;"),
    ("no-slip weight dropped from P_k", "                     (Qadd ? Qadd[((size_t)k * nx + i) * nx + j] : 0.0);",
     "                     0.0;"),
    ("no-slip rows with the stance of the previous stage",
     "const int sk = k < s->N ? k : s->N - 1;", "const int sk = k - 1;"),
    ("no-slip weight with a repeated index",
     "acc += Jc[row * nx + i] * rho_c[(size_t)(k - 1) * nc + row] * Jc[row * nx + j];",
     "acc += Jc[row * nx + i] * rho_c[(size_t)(k - 1) * nc + row] * Jc[row * nx + i];"),
    ("no-slip linear term with the wrong sign", "acc += Jc[row * nx + i] * (yc[idx] - rho_c[idx] * zc[idx]);",
     "acc += Jc[row * nx + i] * (yc[idx] + rho_c[idx] * zc[idx]);"),
    ("no-slip rows projected from the relaxed state",
     "zeta += Jc[row * nx + t] * xt[(size_t)k * nx + t];", "zeta += Jc[row * nx + t] * x[(size_t)k * nx + t];"),
    ("no-slip multipliers left out of the costates",
     "        for (int row = 0; row < nc; ++row) acc += Jc[row * nx + i] * yc[(size_t)(k - 1) * nc + row];\n", ""),
    ("no-slip rows left out of the primal residual", "rp = maxabs(acc - zc[idx], rp);", ""),
]

CHECKS = [
    lambda: pins.test_xupdate_equals_dense_kkt(pins.tiny_shape(5, 4), 1),
    lambda: pins.test_xupdate_equals_dense_kkt(pins.synth.quadruped(4), 2),
    lambda: pins.test_fixed_iterates_equal_dense_admm(pins.tiny_shape(3, 3), 4, 7),
    lambda: pins.test_fixed_iterates_equal_dense_admm(pins.synth.quadruped(3), 5, 5),
    lambda: pins.test_constraint_rows_and_bounds_match_statement(pins.synth.quadruped(3)),
    lambda: pins.test_residuals_match_lagrangian_gradient(),
    lambda: pins.test_converged_equals_brute_force_active_set(2, 2),
    lambda: pins.test_plant_step_is_the_solved_first_transition(),
    lambda: pins.test_complementarity_residual_is_the_projection_residual(),
    lambda: limits.test_xupdate_with_state_rows_equals_dense_kkt(limits.synth.quadruped(3), 2),
    lambda: limits.test_fixed_iterates_with_limits_equal_dense_admm(limits.synth.quadruped(3), 5, 6),
    lambda: limits.test_residuals_with_state_multipliers(),
    lambda: contacts.test_row_table_and_state_weight(contacts.TINY),
    lambda: contacts.test_xupdate_with_contact_rows_equals_dense_kkt(contacts.synth.quadruped(3), 2),
    lambda: contacts.test_fixed_iterates_with_contacts_equal_dense_admm(contacts.synth.quadruped(3), 5, 6, False),
    lambda: contacts.test_residuals_with_contact_multipliers(),
]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(name, old, new):
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation site not unique/present: {name}"
    tmp = tempfile.mkdtemp()
    try:
        src = os.path.join(tmp, "mpc_oracle.c")
        open(src, "w").write(text.replace(old, new))
        so = oracle.build(force=True, src=src, out=os.path.join(tmp, "libmutant.so"))
        oracle.use_library(so)
        caught = []
        for chk in CHECKS:
            try:
                chk()
            except (AssertionError, Exception):  # a failing pin (or a crash of the broken copy)
                caught.append(chk)
                break
        assert caught, f"no pin failed for mutant: {name}"
    finally:
        oracle.use_library(None)
        shutil.rmtree(tmp, ignore_errors=True)


def test_unmutated_copy_passes_every_check():
    """Control: the same build-and-load path with the source unchanged passes."""
    tmp = tempfile.mkdtemp()
    try:
        src = os.path.join(tmp, "mpc_oracle.c")
        shutil.copy(SRC, src)
        so = oracle.build(force=True, src=src, out=os.path.join(tmp, "libcopy.so"))
        oracle.use_library(so)
        for chk in CHECKS:
            chk()
    finally:
        oracle.use_library(None)
        shutil.rmtree(tmp, ignore_errors=True)
