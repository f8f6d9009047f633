"""The pins are strong enough: altered copies of the oracle fail them.

Each mutant is a plausible slip (a dropped term, a wrong sign or index, a
missing weight).  It is compiled from a modified copy of the oracle source in
a temporary directory, and at least one pin must fail against it.
"""

import os

import pytest

import oracle
from tests import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "podcg_oracle.c")

MUTANTS = {
    "drop_beta": ("double s = z[i] + beta * p[i];", "double s = z[i];"),
    "projection_sign": ("for (int32_t j = 0; j < yk; ++j) s -= W[j * n + i] * mu[j];",
                        "for (int32_t j = 0; j < yk; ++j) s += W[j * n + i] * mu[j];"),
    "no_preconditioner_in_loop": ("            z[i] = dinv[i] * r[i];\n        }",
                                  "            z[i] = r[i];\n        }"),
    "transposed_triangular_solve": ("for (int32_t k = 0; k < i; ++k) s -= R[k * m + i] * u[k];",
                                    "for (int32_t k = 0; k < i; ++k) s -= R[i * m + k] * u[k];"),
    "alpha_from_rr": ("double alpha = rho / gamma;", "double alpha = rr / gamma;"),
    "pod_missing_weight": ("coef[k] = w[k] * V[k * s + i] * inv_sigma;",
                           "coef[k] = V[k * s + i] * inv_sigma;"),
    "pod_missing_inv_sigma": ("coef[k] = w[k] * V[k * s + i] * inv_sigma;",
                              "coef[k] = w[k] * V[k * s + i];"),
    "pod_gram_unweighted": ("w[i] * dot(n, S + (size_t)i * n, AS + (size_t)j * n) * w[j];",
                            "dot(n, S + (size_t)i * n, AS + (size_t)j * n);"),
    "stage1_skips_A_d0": ("        for (int64_t i = 0; i < n; ++i) r[i] -= q[i];\n    }",
                          "        for (int64_t i = 0; i < n; ++i) r[i] -= 0.0 * q[i];\n    }"),
    "jacobi_rotation_sign": ("a[k * m + p] = c * akp - s * akq;", "a[k * m + p] = c * akp + s * akq;"),
    "beta_inverted": ("double beta = rho_new / rho;", "double beta = rho / rho_new;"),
}

PINS = [
    pins.test_cholesky_matches_library,
    pins.test_sym_eig_matches_library,
    pins.test_T1_solution_matches_dense_solve,
    pins.test_T2_stage1_is_the_A_projection_and_galerkin,
    pins.test_T3_directions_A_orthogonal_to_W_and_each_other,
    pins.test_T4_exact_recovery_when_solution_in_span,
    lambda o: pins.test_T6_iterates_minimise_A_norm_over_augmented_krylov_space(o, True),
    lambda o: pins.test_T6_iterates_minimise_A_norm_over_augmented_krylov_space(o, False),
    pins.test_T9_pod_basis_is_A_orthonormal_and_nested,
    pins.test_T10_pod_attains_eckart_young_optimum,
    pins.test_T11_pod_evd_equals_pod_svd,
]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) >= 1, f"mutation site for {name} not found"
    src = tmp_path / "mutant.c"
    src.write_text(text.replace(old, new, 1))
    so = oracle.build(src=str(src), out=str(tmp_path / "mutant.so"))
    failures = 0
    try:
        oracle.use_library(so)
        for pin in PINS:
            try:
                pin(oracle)
            except AssertionError:
                failures += 1
            except (ValueError, ZeroDivisionError, FloatingPointError, IndexError, TypeError,
                    __import__("numpy").linalg.LinAlgError):
                failures += 1
    finally:
        oracle.use_library(None)
    assert failures >= 1, f"no pin caught mutant {name}"
