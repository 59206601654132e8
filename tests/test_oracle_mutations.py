"""Plants plausible mistakes in a copy of the oracle (on the CPU) and checks
that the pins catch every one: each mutant must fail at least one pin."""
import os

import pytest

import oracle as oracle_pkg
from oracle import TAG_DIR, Oracle, load

from . import test_oracle_chord as chord
from . import test_oracle_dikin as dikin
from . import test_oracle_flags as flags
from . import test_oracle_precond as precond
from . import test_oracle_projection as proj
from . import test_oracle_rng as rng
from . import test_oracle_sampler as sampler

PINS = [
    rng.test_philox_published_kat,
    lambda o: rng.test_stream_layout(o, 12345678901234, TAG_DIR, 77, 3, 5),
    rng.test_uniforms_open_and_uniform,
    rng.test_gauss_distribution,
    lambda o: chord.test_interval_worked_example(o, 2.0, 7.5, 6.9),
    chord.test_hypercube_closed_form,
    chord.test_bisection_brute_force,
    proj.test_simplex_closed_form,
    lambda o: proj.test_projector_invariants(o, 40, 5, 1),
    sampler.test_simplex_stationary_from_exact_start,
    sampler.test_simplex_cut_small_feasible,
    precond.test_nll_matches_scipy,
    precond.test_gradient_finite_differences,
    precond.test_adam_closed_form,
    precond.test_direction_covariance,
    precond.test_train_step_gradient_finite_differences,
    precond.test_train_step_scale_equivariance,
    dikin.test_hessian_is_barrier_second_difference,
    dikin.test_objective_minimum_is_closed_form,
    dikin.test_objective_gradient_finite_differences,
    dikin.test_train_step_axis_box_closed_form,
    lambda o: dikin.test_train_step_reaches_closed_form_optimum(o, 8, 2, 1.0),
    lambda o: dikin.test_train_step_reaches_closed_form_optimum(o, 10, 3, 0.3),
    flags.test_facet_chord_end_is_zero,
    flags.test_rounding_below_facet_is_clamped,
    flags.test_past_facet_is_infeasible_and_clamped,
    flags.test_vertex_leaving_through_two_facets_is_degenerate,
    flags.test_nan_coordinate_is_nonfinite,
]

MUTANTS = {
    "philox_multiplier": ("0xD2511F53u", "0xD2511F55u"),
    "philox_rounds": ("round < 10", "round < 9"),
    "uniform_bits": (">> 12;", ">> 11;"),
    "box_muller_radius": ("sqrt(-2.0 * log(ua))", "sqrt(-log(ua))"),
    "box_muller_pairing": ("(j & 1) ? radius * sin(angle) : radius * cos(angle)",
                           "(j & 1) ? radius * cos(angle) : radius * sin(angle)"),
    "counter_words": ("ctr[1] = (uint32_t)chain;", "ctr[1] = (uint32_t)block;"),
    "chord_min_as_max": ("if (r < hi) hi = r;", "if (r > lo) hi = r;"),
    "chord_sign_sets": ("if (g > 0.0) {", "if (g < 0.0) {"),
    "theta_formula": ("theta = lo + u * (hi - lo);", "theta = lo + u * hi;"),
    "update_sign": ("x[j] = x[j] + theta * d[j];", "x[j] = x[j] - theta * d[j];"),
    "projection_sign": ("P[i * n + j] -= v;", "P[i * n + j] += v;"),
    "projection_no_inverse": ("cholesky_solve(m_eq, L, col);", ";"),
    "projection_skipped": ("d[i] = v;", "d[i] = h[i];"),
    "precond_scale": ("h[j] = v + exp(log_sigma[j]) * h[j];",
                      "h[j] = v + exp(2.0 * log_sigma[j]) * h[j];"),
    "nll_grad_factor": ("* U[k * r + a];\n                grad_U[i * r + a] = v;",
                        "* U[k * r + a];\n                grad_U[i * r + a] = 0.5 * v;"),
    "nll_logdet": ("\n    for (int64_t i = 0; i < n; ++i) logdet += 2.0 * log(L[i * n + i]);",
                   "\n    for (int64_t i = 0; i < n; ++i) logdet += log(L[i * n + i]);"),
    "dikin_logdet": ("\n        for (int64_t i = 0; i < n; ++i) logdet += 2.0 * log(L[i * n + i]);",
                     "\n        for (int64_t i = 0; i < n; ++i) logdet += log(L[i * n + i]);"),
    "adam_bias": ("double mh = m1[i] / c1;", "double mh = m1[i];"),
    "train_chain_scale": ("gV[i * r + a] = gU[i * r + a] * exp(log_sigma[i]);",
                          "gV[i * r + a] = gU[i * r + a];"),
    "train_chain_rowsum": ("gl[i] += gU[i * r + a] * U[i * r + a];", ";"),
    "slack_not_clamped": ("if (s < 0.0) s = 0.0;", ";"),
    "infeasible_no_tolerance": ("if (s < -tol) f |= MHAR_REF_CHAIN_INFEASIBLE;",
                                "if (s < 0.0) f |= MHAR_REF_CHAIN_INFEASIBLE;"),
    "degenerate_strict": ("} else if (!(hi > lo)) {", "} else if (!(hi >= lo)) {"),
    "nonfinite_unchecked": ("if (!finite) flags |= MHAR_REF_CHAIN_NONFINITE;", ";"),
    "dikin_weight_power": ("w[i] = 1.0 / (s * s);", "w[i] = 1.0 / s;"),
    "dikin_row_index": ("v += w[i] * A[i * n + p] * A[i * n + q];",
                        "v += w[i] * A[i * n + p] * A[i * n + p];"),
    "dikin_kl_half": ("*K = 0.5 * tr - 0.5 * logdet;", "*K = 0.5 * tr - logdet;"),
    "dikin_grad_sign": ("v += (H[i * n + k] - Sinv[i * n + k]) * U[k * r + a];",
                        "v += (H[i * n + k] + Sinv[i * n + k]) * U[k * r + a];"),
    "dikin_grad_l_scale": ("(H[i * n + i] - Sinv[i * n + i]) * exp(2.0 * log_sigma[i]);",
                           "(H[i * n + i] - Sinv[i * n + i]) * exp(log_sigma[i]);"),
    "dikin_not_inscribed": ("log_sigma[i] = log(kappa) - 0.5 * log(lam * H[i * n + i]);",
                            "log_sigma[i] = log(kappa) - 0.5 * log(H[i * n + i]);"),
    "dikin_kappa_power": ("log_sigma[i] = log(kappa) - 0.5 * log(lam * H[i * n + i]);",
                          "log_sigma[i] = 0.5 * log(kappa) - 0.5 * log(lam * H[i * n + i]);"),
    "dikin_no_newton": ("U[i * r + a] -= eta * col[i];", "U[i * r + a] -= eta * gU[i * r + a];"),
    "dikin_power_unscaled": ("lam += v[i] * t;", "lam += t;"),
}


def _fails(o, pin):
    try:
        pin(o)
    except AssertionError:
        return True
    except Exception:  # a crash or error also counts as caught
        return True
    return False


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(oracle_pkg.SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} must be unique"
    mutated = tmp_path / "mhar_ref.c"
    mutated.write_text(src.replace(old, new))
    (tmp_path / "mhar_ref.h").write_text(open(os.path.join(oracle_pkg.HERE, "mhar_ref.h")).read())
    lib_path = str(tmp_path / "libmut.so")
    import subprocess
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC", "-o",
                    lib_path, str(mutated), "-lm"], check=True)
    o = Oracle(load(lib_path))
    assert any(_fails(o, pin) for pin in PINS), f"no pin caught mutant {name}"


def test_unmutated_oracle_passes_all_pins():
    o = Oracle()
    assert not any(_fails(o, pin) for pin in PINS)
