"""The oracle's pins catch plausible slips.

Each case plants one mistake in a private copy of the oracle's source (a
dropped term, a flipped sign, a wrong index, a transposed operand), loads
it as a separate module, points the pin tests at it and checks that at
least one of the pins named for the case fails.  Nothing here touches the
real oracle module or the GPU path.
"""
import os
import sys
import types

import pytest

import test_oracle_pins as P

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "oracle", "sstep_gmres.py")


def mutant(old, new):
    with open(SRC) as f:
        text = f.read()
    assert text.count(old) == 1, f"mutation anchor not unique: {old!r}"
    text = text.replace(old, new)
    name = "oracle_mutant"
    mod = types.ModuleType(name)
    mod.__file__ = SRC
    sys.modules[name] = mod            # dataclasses look their module up
    exec(compile(text, SRC, "exec"), mod.__dict__)
    return mod


# (case, old source, new source, pins of which at least one must fail)
CASES = [
    ("hessenberg_sign",
     "M[:i, :] -= Hraw[:i, :i - 1] @ X",
     "M[:i, :] += Hraw[:i, :i - 1] @ X",
     [(P.test_arnoldi_relation_and_hessenberg_structure, ())]),
    ("givens_sine_sign",
     "cc, ss = a / rr, b / rr",
     "cc, ss = a / rr, -b / rr",
     [(P.test_givens_least_squares_vs_lstsq, ())]),
    ("cholesky_pivot_drops_last_term",
     "piv = G[j, j] - R[:j, j] @ R[:j, j]",
     "piv = G[j, j] - R[:j - 1, j] @ R[:j - 1, j]",
     [(P.test_partial_cholesky_against_numpy_and_truncation, ())]),
    ("ice_unsquared_pivot",
     "lam, (s, c) = _top_eig_2x2(self.smax2 + a * a, a * g, g * g)",
     "lam, (s, c) = _top_eig_2x2(self.smax2 + a * a, a * g, g)",
     [(P.test_ice_brackets_true_condition, ())]),
    ("leja_minimises_product",
     "scores.append(-np.inf if np.any(d == 0.0) else float(np.sum(np.log(d))))",
     "scores.append(-np.inf if np.any(d == 0.0) else float(-np.sum(np.log(d))))",
     [(P.test_leja_order_bruteforce, ())]),
    ("complex_pair_delta_sign",
     "delta[j + 1] = -beta * beta / g[j]",
     "delta[j + 1] = beta * beta / g[j]",
     [(P.test_complex_pair_recurrence, ())]),
    ("combine_transposed_Z",
     "R_top = W[:, :p].astype(np.float64) + R2[:, :p].astype(np.float64) @ Zp",
     "R_top = W[:, :p].astype(np.float64) + R2[:, :p].astype(np.float64) @ Zp.T",
     [(P.test_arnoldi_relation_and_hessenberg_structure, ()),
      (P.test_sstep_iterates_are_gmres_minimisers, ("scaled_newton", 5))]),
    ("rkk_operand_order",
     "R_kk = Zt @ Zp",
     "R_kk = Zp @ Zt",
     [(P.test_arnoldi_relation_and_hessenberg_structure, ()),
      (P.test_sstep_iterates_are_gmres_minimisers, ("scaled_newton", 5))]),
    ("mpk_multiplies_by_gamma",
     "V[:, j + 1] = w / wt(ga)",
     "V[:, j + 1] = w * wt(ga)",
     [(P.test_arnoldi_relation_and_hessenberg_structure, ()),
      (P.test_sstep_iterates_are_gmres_minimisers, ("scaled_newton", 3))]),
    ("change_of_basis_shift_sign",
     "B[j, j] = th",
     "B[j, j] = -th",
     [(P.test_arnoldi_relation_and_hessenberg_structure, ()),
      (P.test_sstep_iterates_are_gmres_minimisers, ("scaled_newton", 3))]),
    ("single_bcgs_pass",
     "R2 = Qi.T @ Qk                                   # second BCGS",
     "R2 = 0.0 * (Qi.T @ Qk)                           # second BCGS",
     [(P.test_loss_of_orthogonality, ())]),
    ("estimator_diagonal_without_eps",
     "L[i, j] = lr[i, :j].sum() + le",
     "L[i, j] = lr[i, :j].sum()",
     [(P.test_estimator_matrix_small_closed_form, ()),
      (P.test_E8_estimator_prediction, ())]),
    ("jacobi_scales_instead_of_unscaling",
     "xo = x / dscale if dscale is not None else x\n        if trace",
     "xo = x * dscale if dscale is not None else x\n        if trace",
     [(P.test_jacobi_right_preconditioning, ())]),
    ("refinement_drops_residual_norm",
     "x = x + beta * d",
     "x = x + d",
     [(P.test_fp32_inner_refinement_reaches_fp64_accuracy, ())]),
    ("gradient_sign",
     "return -np.asarray(lam)[rows] * np.asarray(x)[np.asarray(col)]",
     "return np.asarray(lam)[rows] * np.asarray(x)[np.asarray(col)]",
     [(P.test_adjoint_gradients_fd_and_dense, ())]),
    ("breakdown_wrong_coefficients",
     "return BlockQR(0, V[:, :0], W[:, :1].astype(np.float64),",
     "return BlockQR(0, V[:, :0], 0.5 * W[:, :1].astype(np.float64),",
     [(P.test_happy_breakdown_eigenvector_rhs, ())]),
    ("pythagorean_gram_sign",
     "G2 = (Qk.T @ Qk).astype(np.float64) - R2d.T @ R2d",
     "G2 = (Qk.T @ Qk).astype(np.float64) + R2d.T @ R2d",
     [(P.test_pythagorean_second_pass_block, (1e-12,))]),
    ("pythagorean_gram_drops_projection",
     "G2 = (Qk.T @ Qk).astype(np.float64) - R2d.T @ R2d",
     "G2 = (Qk.T @ Qk).astype(np.float64) - 0.0 * (R2d.T @ R2d)",
     [(P.test_pythagorean_second_pass_block, (1e-12,))]),
    ("fp32_model_with_fp64_roundoff",
     "self.u = U32 if self.wd == np.float32 else U64",
     "self.u = U64",
     [(P.test_fp32_partial_cholqr_stops_at_single_precision_bound, ()),
      (P.test_fp32_estimator_tracks_single_precision_basis_growth, ())]),
    ("fp32_block_bound_from_fp64",
     "self.omega = opts.omega if opts.omega > 0 else default_omega(self.u)",
     "self.omega = opts.omega if opts.omega > 0 else default_omega(U64)",
     [(P.test_fp32_partial_cholqr_stops_at_single_precision_bound, ())]),
    ("fp32_model_runs_in_fp64",
     "self.wd = np.dtype(opts.work_dtype)",
     "self.wd = np.dtype(np.float64)",
     [(P.test_fp32_inner_cycle_is_the_gmres_minimiser, ())]),
    ("ilu0_no_division_by_pivot",
     "v[e] = v[e] / piv",
     "v[e] = v[e]",
     [(P.test_ilu0_reproduces_A_on_its_pattern, ("laplace2d_12",)),
      (P.test_ilu0_five_point_closed_form, ())]),
    ("ilu0_eliminates_with_the_lower_part",
     "for f in range(dpos[k] + 1, rp[k + 1]):",
     "for f in range(rp[k], dpos[k]):",
     [(P.test_ilu0_reproduces_A_on_its_pattern, ("random_90",)),
      (P.test_ilu0_of_tridiagonal_is_the_exact_lu, ())]),
    ("ilu0_update_without_preconditioner",
     "x = x + (dx if prec is None else prec.solve(dx))",
     "x = x + dx",
     [(P.test_ilu0_right_preconditioned_iterates_are_gmres_minimisers,
       ("scaled_newton",))]),
    ("ilu0_shift_on_the_preconditioned_vector",
     "w = self.Aw @ z - wt(th) * V[:, j]",
     "w = self.Aw @ z - wt(th) * z",
     [(P.test_ilu0_right_preconditioned_iterates_are_gmres_minimisers,
       ("scaled_newton",))]),
    ("givens_rhs_not_rotated",
     "self.g[col + 1] = -ss * gc",
     "self.g[col + 1] = ss * gc",
     [(P.test_residual_monotone_and_true_residual, ()),
      (P.test_s1_equals_mgs_gmres, ("scaled_newton",))]),
]


@pytest.mark.parametrize("case,old,new,pins", CASES, ids=[c[0] for c in CASES])
def test_mutation_is_caught(monkeypatch, case, old, new, pins):
    mod = mutant(old, new)
    monkeypatch.setattr(P, "o", mod)
    caught = []
    for pin, args in pins:
        try:
            pin(*args)
        except Exception as e:          # an assertion or a crash
            caught.append((pin.__name__, type(e).__name__))
    sys.modules.pop("oracle_mutant", None)
    assert caught, f"{case} escaped every pin it names"


def test_unmutated_copy_passes_the_same_pins(monkeypatch):
    """Control: the loader itself changes nothing."""
    mod = mutant("def loo(Q):", "def loo(Q):")
    monkeypatch.setattr(P, "o", mod)
    for _, _, _, pins in CASES:
        for pin, args in pins:
            pin(*args)
    sys.modules.pop("oracle_mutant", None)
