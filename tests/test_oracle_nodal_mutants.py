"""Planted mistakes in copies of the nodal-projection oracle must fail a pin.

Each case copies `oracle/nodal_oracle.c`, replaces one exact piece of text by a
plausible mistake, compiles the copy with gcc on the CPU, routes the nodal
oracle wrappers through it and checks that the named pin of
tests/test_oracle_nodal.py now fails.  The oracle source itself is never
modified.
"""
import pytest

from oracle import compile_variant
from oracle import nodal as nd
from tests import test_oracle_nodal as T


def _passes(fn, *args):
    try:
        fn(*args)
        return True
    except AssertionError:
        return False


def pin_symbol():
    return _passes(T.test_symbol_of_the_constant_coefficient_operator, (6, 10, 4))


def pin_operator():
    return all(_passes(T.test_operator_equals_the_quadrature_assembly, s, b) for s, b in T.CASES)


def pin_div_grad_load():
    return all(_passes(T.test_divergence_gradient_and_load_equal_the_quadrature, s, b) for s, b in T.CASES)


def pin_transfers():
    return all(_passes(T.test_transfers_are_interpolation_and_its_scaled_transpose, s, b)
               for s, b in [((8, 8, 8), (0, 0, 0)), ((8, 4, 6), (1, 0, 1))])


def pin_rhs():
    return _passes(T.test_right_hand_side_is_the_weak_form_and_sums_to_zero)


def pin_lu():
    return all(_passes(T.test_solve_matches_a_sparse_lu_of_the_bordered_system, s, b)
               for s, b in [((16, 16, 16), (0, 0, 1)), ((16, 8, 12), (1, 1, 1))])


def pin_smooth():
    return _passes(T.test_smooth_flow_is_projected_at_second_order)


def pin_sigma():
    return _passes(T.test_sigma_coarsening_is_the_mean_of_the_children) and pin_lu()


MUTANTS = [
    ("lumped 1D mass matrix", "return a == b ? 1.0 / 3.0 : 1.0 / 6.0;", "return a == b ? 0.5 : 0.0;", pin_symbol),
    ("stiffness term scaled by h instead of 1/h", "double t = stiff1(bit(A, d), bit(B, d)) / h;",
     "double t = stiff1(bit(A, d), bit(B, d)) * h;", pin_operator),
    ("one axis dropped from the element stiffness", "for (int d = 0; d < 3; d++) {\n        double t = stiff1",
     "for (int d = 0; d < 2; d++) {\n        double t = stiff1", pin_operator),
    ("gradient integral sign flipped", "return a ? 1.0 : -1.0; }", "return a ? -1.0 : 1.0; }", pin_div_grad_load),
    ("y component dropped from the divergence", " + vy[cq[e]] * elem_grad(A, 1, h)", "", pin_div_grad_load),
    ("corner bits of the node in its cells mirrored", "corner[cnt] = (ox ? 1 : 0) | (oy ? 2 : 0) | (oz ? 4 : 0);",
     "corner[cnt] = (ox ? 0 : 1) | (oy ? 2 : 0) | (oz ? 4 : 0);", pin_operator),
    ("restriction without the 1/8", "rc[node(&c, I, J, K)] = 0.125 * s;", "rc[node(&c, I, J, K)] = s;",
     pin_transfers),
    ("odd fine nodes take one coarse node", "    w[0] = w[1] = 0.5;\n    return 2;", "    w[0] = 1.0;\n    return 1;",
     pin_transfers),
    ("source mean not removed", "for (long q = 0; q < n; q++) src[q] -= m;", "", pin_rhs),
    ("sign of the source in the right-hand side", "for (long q = 0; q < nn; q++) out[q] -= ld[q];",
     "for (long q = 0; q < nn; q++) out[q] += ld[q];", pin_rhs),
    ("Gauss-Seidel update with the wrong sign of the right-hand side",
     "(-h3 * lv->rhs[node(g, i, j, k)] - of) / dg", "(h3 * lv->rhs[node(g, i, j, k)] - of) / dg", pin_lu),
    ("convergence test on a mis-scaled norm", "rel = sqrt(node_dot(&lv[0].g, lv[0].res, lv[0].res)) / nb;",
     "rel = sqrt(node_dot(&lv[0].g, lv[0].res, lv[0].res)) / (1e6 * nb);", pin_lu),
    ("coarse sigma summed, not averaged", "sc[((long)K * NY + J) * NX + I] = 0.125 * s;",
     "sc[((long)K * NY + J) * NX + I] = s;", pin_sigma),
    ("velocity correction added", "ux[q] -= w * gx[q];\n        uy[q] -= w * gy[q];\n        uz[q] -= w * gz[q];",
     "ux[q] += w * gx[q];\n        uy[q] += w * gy[q];\n        uz[q] += w * gz[q];", pin_smooth),
]


def test_pins_pass_on_the_oracle():
    for _, _, _, pin in MUTANTS:
        assert pin(), pin.__name__


@pytest.mark.parametrize("case", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(case, tmp_path):
    name, old, new, pin = case
    src = nd.source_text()
    assert old in src, f"mutation site for '{name}' not found in the nodal oracle source"
    lib = compile_variant(src.replace(old, new), str(tmp_path / "mutant.so"))
    with nd.use_library(lib):
        assert not pin(), f"pin {pin.__name__} did not catch: {name}"
