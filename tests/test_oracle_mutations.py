"""The pins must catch plausible mistakes in the oracle (CPU only).

Each case plants one mistake (a flipped sign, a dropped term, a transposed
operand, an off-by-one index, a different integrator) in a private copy of
the oracle's C sources, builds it, routes the oracle through that build and
runs the pin tests; at least one pin must fail.
"""
import os
import shutil
import subprocess

import pytest

import oracle as O
import test_oracle_contact as contact
import test_oracle_pgs as pgs
import test_oracle_pins as pins

SRC = os.path.dirname(os.path.abspath(O.__file__))

MUTATIONS = [
    ("aba_fwd.inc", "- s * ax[k] + (1.0 - c) * ax2[k]", "+ s * ax[k] + (1.0 - c) * ax2[k]", "joint rotation sign"),
    ("aba_fwd.inc", "J[3 * i + j] - m * cx2[3 * i + j]", "J[3 * i + j] + m * cx2[3 * i + j]", "inertia shift sign"),
    ("aba_fwd.inc", "w[j] = l->u[j] - Uap;", "w[j] = l->u[j] + Uap;", "pass-3 sign"),
    ("aba_fwd.inc", "S s_ = l->pA[r] + Iac[r];", "S s_ = l->pA[r];", "dropped I^a c term"),
    ("aba_fwd.inc", "FN(mat6_mul)(XT_, l->Ia, T1);\n      FN(mat6_mul)(T1, l->X, T2);",
     "FN(mat6_mul)(l->X, l->Ia, T1);\n      FN(mat6_mul)(T1, XT_, T2);", "transposed congruence"),
    ("aba_fwd.inc", "FN(integrate_pos)(m, q, qd1, dt, q1);", "FN(integrate_pos)(m, q, qd, dt, q1);",
     "explicit instead of semi-implicit Euler"),
    ("aba_fwd.inc", "l->abase[k + 3] = l->ap[k + 3] + Eg[k];", "l->abase[k + 3] = l->ap[k + 3] - Eg[k];",
     "free-root gravity sign"),
    ("aba_oracle.c", "b->U[6 * j + r] -= l->ap[r] * wb[j];", "b->U[6 * j + r] += l->ap[r] * wb[j];",
     "adjoint sign (U_bar)"),
    ("aba_oracle.c", "          b->Di[3 * k + j] += yb[k] * l->u[j];\n", "", "dropped D_bar term"),
    ("aba_oracle.c", "tvec_add(F, b->pA, b->h);", "vec_add(F, b->pA, b->h);", "transposed crf adjoint"),
    ("aba_oracle.c", "const double tot = qd1bar[vi[i]] + dt * q1bar[qi[i]];", "const double tot = qd1bar[vi[i]];",
     "dropped integrator coupling"),
    ("aba_oracle.c", "E0bar[3 * r + c] += ab[3 + r] * g[c];", "E0bar[3 * c + r] += ab[3 + r] * g[c];",
     "transposed gravity adjoint index"),
    ("aba_oracle.c", "qtb[k] += h * (cr[k] - w1[k] * ob[3]);", "qtb[k] += h * (cr[k] + w1[k] * ob[3]);",
     "quaternion product adjoint sign"),
    ("aba_oracle.c", "tau + (size_t)(t0 + j - 1) * nu, tape, qdd);", "tau + (size_t)(t0 + j) * nu, tape, qdd);",
     "off-by-one in the segment replay"),
    ("aba_oracle.c", "outer_add(b->ap, al, b->X);", "outer_add(al, b->ap, b->X);", "transposed X_bar outer product"),
    ("aba_oracle.c", "      outer_add(b->h, l->v, Ibar);\n", "", "dropped h = I v term of the inertia adjoint"),
    ("aba_oracle.c", "pbar[7] += Ibar[1] + Ibar[6];", "pbar[7] += Ibar[1];", "off-diagonal inertia counted once"),
    ("aba_oracle.c", "pbar[1] += P[3 * 2 + 1] - P[3 * 1 + 2];", "pbar[1] += P[3 * 1 + 2] - P[3 * 2 + 1];",
     "first-moment adjoint sign"),
    ("aba_oracle.c", "pbar[0] += Ibar[6 * 3 + 3] + Ibar[6 * 4 + 4] + Ibar[6 * 5 + 5];",
     "pbar[0] += Ibar[6 * 3 + 3] + Ibar[6 * 4 + 4];", "dropped mass-block term"),
    ("aba_oracle.c", "dXJ[6 * (3 + r) + cc] = -axx[3 * r + cc];", "dXJ[6 * (3 + r) + cc] = axx[3 * r + cc];",
     "prismatic joint-transform derivative sign"),
    ("aba_fwd.inc", "Sv[k] = prism ? 0.0 : ax[k];", "Sv[k] = ax[k];", "prismatic motion subspace with an angular part"),
    ("aba_fwd.inc", "l->vJ[k] = 0; l->vJ[k + 3] = m->axis[3 * i + k] * qd[vi[i]];",
     "l->vJ[k] = m->axis[3 * i + k] * qd[vi[i]]; l->vJ[k + 3] = 0;", "prismatic joint velocity as a rotation"),
    ("aba_oracle.c", "    for (int j = 0; j < 3; ++j) sw += Sbar[prism ? 3 + j : j] * da[j];\n", "",
     "dropped motion-subspace term of the axis gradient"),
    ("aba_oracle.c", "dEJ[j] = -sin(q) * dax[j] + (1.0 - cos(q)) * (t1[j] + t2[j]);",
     "dEJ[j] = sin(q) * dax[j] + (1.0 - cos(q)) * (t1[j] + t2[j]);", "joint-rotation axis derivative sign"),
    ("aba_oracle.c", "mat3_mul_r(ET, ekx, Ee);", "mat3_mul_r(ekx, ET, Ee);", "transposed joint-origin derivative"),
    ("aba_oracle.c", "        dXT[6 * (3 + r) + c] = -dErx[3 * r + c];\n", "",
     "dropped translation term of the frame-rotation derivative"),
    ("aba_oracle.c", "          b->S[6 * k + c] += l->IA[6 * r + c] * b->U[6 * k + r];\n", "",
     "dropped U = IA S term of the motion-subspace adjoint"),
    ("pgs_oracle.c", "        if (j != i) d += A[(size_t)i * n + j] * x[j];\n      const double y = -(b[i] + d)",
     "        if (j != i) d += A[(size_t)i * n + i] * x[j];\n      const double y = -(b[i] + d)",
     "PGS row sum with the diagonal entry (as the printed listing reads)"),
    ("pgs_oracle.c", "      if (st < 0) lobar[i] += xb[i];\n      else if (st > 0) hibar[i] += xb[i];",
     "      if (st < 0) hibar[i] += xb[i];\n      else if (st > 0) lobar[i] += xb[i];", "PGS bound adjoints swapped"),
    ("pgs_oracle.c", "      xb[i] = 0;\n", "", "PGS adjoint keeps the overwritten row's adjoint"),
    ("pgs_oracle.c", "for (int j = 0; j < n; ++j) cur[j] = (j < i) ? xe[j] : xs[j];",
     "for (int j = 0; j < n; ++j) cur[j] = (j > i) ? xe[j] : xs[j];", "PGS adjoint with old and new values swapped"),
    ("pgs_oracle.c", "Abar[(size_t)i * n + i] += db * y;", "Abar[(size_t)i * n + i] -= db * y;", "PGS diagonal adjoint sign"),
    ("aba_oracle.c", "    *dq = -L[2];", "    *dq = L[2];", "joint-limit stiffness adjoint sign"),
    ("aba_oracle.c", "    *dqd = -L[3];", "    *dqd = 0;", "dropped joint-limit damping adjoint"),
    ("aba_fwd.inc", "if (SREAL(q) < L[0]) return -L[2] * (q - L[0]) - L[3] * qd;",
     "if (SREAL(q) < L[0]) return -L[2] * (q - L[1]) - L[3] * qd;", "lower joint limit measured from the upper one"),
    ("aba_fwd.inc", "for (int b = 0; b < 3; ++b) EJ[3 * a + b] = R[3 * b + a];",
     "for (int b = 0; b < 3; ++b) EJ[3 * a + b] = R[3 * a + b];", "ball-joint rotation not transposed"),
    ("aba_fwd.inc", "for (int k = 0; k < 3; ++k) { l->vJ[k] = qd[vi[i] + k]; l->vJ[k + 3] = 0; }",
     "for (int k = 0; k < 3; ++k) { l->vJ[k] = 0; l->vJ[k + 3] = qd[vi[i] + k]; }", "ball-joint velocity as a translation"),
    ("aba_fwd.inc", "Di[1] = -(b * k - c * h) / det;", "Di[1] = (b * k - c * h) / det;", "3x3 inverse cofactor sign"),
    ("aba_fwd.inc", "FN(quat_step)(q + qi[i], qd1 + vi[i], dt, q1 + qi[i]);",
     "FN(quat_step)(q + qi[i], qd1 + vi[i], 0.5 * dt, q1 + qi[i]);", "ball joint turned by half a step"),
    ("aba_oracle.c", "Rbar[3 * c + r] = XJb[6 * r + c] + XJb[6 * (3 + r) + 3 + c];",
     "Rbar[3 * r + c] = XJb[6 * r + c] + XJb[6 * (3 + r) + 3 + c];", "ball-joint rotation adjoint transposed"),
    ("aba_oracle.c", "quat_step_vjp(qt, w1, dt, q1bar + qi[i], qbar + qi[i], w1bar);",
     "quat_step_vjp(qt, qd + vi[i], dt, q1bar + qi[i], qbar + qi[i], w1bar);",
     "ball-joint orientation adjoint at the old angular velocity"),
    ("aba_oracle.c", "qddbar[vi[i] + k] = dt * w1bar[k];", "qddbar[vi[i] + k] = w1bar[k];",
     "ball-joint integrator adjoint without dt"),
    ("contact.inc", "dirs[3] = {1, 0, 2};", "dirs[3] = {0, 1, 2};", "contact normal along x"),
    ("contact.inc", "cl[3 * na + a] = c[a] - C->radius[k] * Ew[9 * l + 3 * a + 1];",
     "cl[3 * na + a] = c[a] + C->radius[k] * Ew[9 * l + 3 * a + 1];", "contact point at the sphere's top"),
    ("contact.inc", "fe[0] = cl[3 * c + 1] * f[2] - cl[3 * c + 2] * f[1];",
     "fe[0] = cl[3 * c + 2] * f[1] - cl[3 * c + 1] * f[2];", "contact moment arm sign"),
    ("contact.inc", "C->beta / dt * phi[i / 3]", "-C->beta / dt * phi[i / 3]", "Baumgarte sign"),
    ("contact.inc", "lok[i] = -mu * lamn[ri / 3];\n        hik[i] = mu * lamn[ri / 3];",
     "lok[i] = -mu;\n        hik[i] = mu;", "friction box not scaled by the normal impulse"),
    ("contact.inc", "lok[i] = -mu * lamn[ri / 3];", "lok[i] = -C->mu * lamn[ri / 3];",
     "friction gradient misses the lower bound"),
    ("contact.inc", "s_ += J[(size_t)i * nv + k] * qd1[k];", "s_ += J[(size_t)i * nv + k] * qd[k];",
     "contact velocity before the smooth update"),
    ("contact.inc", "> 1e-12 * dmax) keep[nk++] = i;", ">= 0) keep[nk++] = i;", "zero rows kept in the solve"),
    ("aba_oracle.c", "    const double *cur = xs + (size_t)t * nx;\n    for (int j = 0; j < nx + nu; ++j) {",
     "    const double *cur = xs + (size_t)(t + 1) * nx;\n    for (int j = 0; j < nx + nu; ++j) {",
     "contact step Jacobian at the step's output state"),
]

PINS = [
    pins.test_aba_equals_dense_solve_every_tree_up_to_4_links,
    pins.test_free_base_dense_solve_and_momentum_balance,
    pins.test_single_pendulum_closed_form,
    pins.test_semi_implicit_euler_step_and_no_secular_energy_growth,
    pins.test_single_step_tau_bar_is_Minv_qdd_bar,
    pins.test_single_step_state_adjoint_matches_inverse_dynamics_jacobian,
    pins.test_free_base_single_step_adjoint_matches_inverse_dynamics_jacobian,
    pins.test_rollout_gradient_complex_step_chain,
    pins.test_free_base_rollout_gradient_complex_step,
    lambda: pins.test_checkpoint_interval_changes_no_arithmetic("quad"),
    lambda: pins.test_inertial_parameter_gradient_scaling_identity(0),
    lambda: pins.test_inertial_parameter_gradient_central_differences(0),
    lambda: pins.test_inertial_parameter_gradient_central_differences(1),
    pins.test_cartpole_closed_form,
    pins.test_rollout_gradient_complex_step_with_prismatic_joints,
    pins.test_frame_gradient_invariances_of_a_fixed_base_tree,
    lambda: pins.test_frame_and_axis_gradients_central_differences(0),
    pins.test_joint_limit_torque_is_added_to_the_control,
    pins.test_rollout_gradient_with_joint_limits_complex_step,
    pins.test_aba_equals_dense_solve_every_tree_with_spherical_joints,
    pins.test_single_body_on_a_ball_joint_obeys_eulers_equations,
    lambda: pins.test_rollout_gradient_complex_step_with_spherical_joints(0),
    pgs.test_unbounded_converges_to_the_linear_solve,
    pgs.test_one_sweep_by_hand,
    lambda: pgs.test_adjoint_against_complex_step(3, 12),
    lambda: pgs.test_adjoint_against_complex_step(9, 2),
    pgs.test_adjoint_of_the_converged_linear_solve,
    contact.test_frictionless_ball_impact_closed_form,
    lambda: contact.test_sliding_point_mass_friction(2.0, 0.001),
    contact.test_assembly_against_newton_euler_kinematics_and_mass_matrix,
    contact.test_struck_pendulum_impulse_is_the_effective_mass_law,
    contact.test_baumgarte_pushes_out_at_beta_phi_over_dt,
    lambda: contact.test_rollout_gradient_with_contact_central_differences(0.8),
    contact.test_friction_gradient_of_a_sliding_point_mass_closed_form,
]


@pytest.mark.parametrize("fname,old,new,what", MUTATIONS, ids=[m[3] for m in MUTATIONS])
def test_pins_catch_planted_mistake(tmp_path, fname, old, new, what):
    for f in ("aba_oracle.c", "aba_fwd.inc", "contact.inc", "oracle.h", "pgs_oracle.c"):
        shutil.copy(os.path.join(SRC, f), tmp_path / f)
    path = tmp_path / fname
    text = path.read_text()
    assert text.count(old) == 1, f"mutation site for '{what}' not found exactly once"
    path.write_text(text.replace(old, new))
    so = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", str(so),
                           str(tmp_path / "aba_oracle.c"), str(tmp_path / "pgs_oracle.c"), "-lm"])
    caught = None
    with O.use_library(str(so)):
        for pin in PINS:
            try:
                pin()
            except (AssertionError, RuntimeError, FloatingPointError, ValueError) as e:
                caught = getattr(pin, "__name__", "checkpoint invariance")
                break
    assert caught is not None, f"no pin caught the planted mistake: {what}"
