"""Plants plausible mistakes in copies of the oracle source (on the CPU only)
and checks that each one fails at least one pin.  This shows that the pins in
``pins.py`` constrain every step of the oracle: a dropped term, a wrong sign, a
wrong or transposed index, a wrong factor or a wrong derivative rule is caught.
"""
import os

import pytest

import oracle
import pins
from oracle import build as obuild

SRC = open(obuild.SRC).read()

# (id, text in the oracle source, replacement)
MUTANTS = [
    ("cofactor_sign", "a[i1][j1] * a[i2][j2] - a[i1][j2] * a[i2][j1]",
     "a[i1][j1] * a[i2][j2] + a[i1][j2] * a[i2][j1]"),
    ("cofactor_index", "a[i1][j1] * a[i2][j2] - a[i1][j2] * a[i2][j1]",
     "a[i1][j1] * a[i2][j2] - a[i1][j1] * a[i2][j1]"),
    ("det_term", "a[0][1] * cof[0][1] + a[0][2] * cof[0][2]",
     "a[0][1] * cof[1][1] + a[0][2] * cof[0][2]"),
    ("det_dropped", "a[0][1] * cof[0][1] + a[0][2] * cof[0][2]", "a[0][1] * cof[0][1]"),
    ("sym_table", "{1, 3, 4}, {2, 4, 5}", "{1, 3, 5}, {2, 4, 5}"),
    ("gamma_sign", "- D(l, j, k))", "+ D(l, j, k))"),
    ("gamma_dropped_term", "((D(k, j, l) + D(j, l, k)) - D(l, j, k))", "(D(k, j, l) - D(l, j, k))"),
    ("gamma_deriv_index", "((D(k, j, l) + D(j, l, k))", "((D(j, k, l) + D(j, l, k))"),
    ("gamma_inverse_index", "G(i, l) * ((D", "G(j, l) * ((D"),
    ("gamma_half", "T(0.5) * sum", "sum"),
    ("gamma_dg_layout", "dg[k * 6 + sym(i, j)]", "dg[i * 6 + sym(k, j)]"),
    ("nabla_sign", "dbeta[j * 3 + i] - sum", "dbeta[j * 3 + i] + sum"),
    ("nabla_transposed_dbeta", "dbeta[j * 3 + i] - sum", "dbeta[i * 3 + j] - sum"),
    ("nabla_gamma_index", "gam27[(k * 3 + i) * 3 + j] * beta[k]", "gam27[(i * 3 + k) * 3 + j] * beta[k]"),
    ("nabla_stored_gamma", "g27[(i * 3 + j) * 3 + k] = Gs[i * 6 + sym(j, k)]",
     "g27[(i * 3 + j) * 3 + k] = Gs[j * 6 + sym(i, k)]"),
    ("dtg_sign", "T(-2.0) * alpha", "T(2.0) * alpha"),
    ("dtg_dropped_term", "+ nb[i * 3 + j] + nb[j * 3 + i]", "+ nb[i * 3 + j] + nb[i * 3 + j]"),
    ("dtg_factor", "T(-2.0) * alpha * K", "alpha * K"),
    ("tape_mul_partials", "make(a.v * b.v, a.id, b.v, b.id, a.v)", "make(a.v * b.v, a.id, a.v, b.id, b.v)"),
    ("tape_div_sign", "-q / b.v);", "q / b.v);"),
    ("tape_sub_sign", "make(a.v - b.v, a.id, 1.0, b.id, -1.0)", "make(a.v - b.v, a.id, 1.0, b.id, 1.0)"),
    ("dual_div", "(a.d - q * b.d) / b.v", "(a.d + q * b.d) / b.v"),
    ("dual_mul", "a.d * b.v + a.v * b.d", "a.d * b.v + a.v * b.v"),
    ("add3_dropped_term", "in[0][i] + in[1][i] + in[2][i] + in[3][i]",
     "in[0][i] + in[1][i] + in[3][i] + in[3][i]"),
    ("mult2_index", "in[0][i] * in[1][j] * in[2][k]", "in[0][i] * in[1][k] * in[2][j]"),
    ("mult3_index", "in[0][i] * in[1][j] * in[2][k] * in[3][l]",
     "in[0][i] * in[1][j] * in[2][l] * in[3][k]"),
    ("contract1_transposed_b", "sum += B[i * 3 + m] * E[((m * 3 + j) * 3 + k) * 3 + l]",
     "sum += B[m * 3 + i] * E[((m * 3 + j) * 3 + k) * 3 + l]"),
    ("contract1_e_index", "sum += B[i * 3 + m] * E[((m * 3 + j) * 3 + k) * 3 + l]",
     "sum += B[i * 3 + m] * E[((m * 3 + k) * 3 + j) * 3 + l]"),
    ("contract2_c_index", "sum += C[j * 3 + n] * B[i * 3 + m] * E[((m * 3 + n) * 3 + k) * 3 + l]",
     "sum += C[n * 3 + j] * B[i * 3 + m] * E[((m * 3 + n) * 3 + k) * 3 + l]"),
    ("contract3_e_index", "E[((m * 3 + n) * 3 + o) * 3 + l]", "E[((n * 3 + m) * 3 + o) * 3 + l]"),
    ("contract3_d_index", "sum += D[k * 3 + o] * C[j * 3 + n]", "sum += D[o * 3 + k] * C[j * 3 + n]"),
    ("kij_factor", "out[sym(i, j)] = 2.0 * alpha * in[1][sym(i, j)]",
     "out[sym(i, j)] = alpha * in[1][sym(i, j)]"),
    ("kij_outer", "+ in[2][i] * in[2][j]", "+ in[2][i] * in[2][i]"),
    ("expr_table", "{9, 81}, {9, 9, 81}", "{9, 81}, {9, 81, 9}"),
    ("sym4_table", "{1, 4, 5, 6}, {2, 5, 7, 8}", "{1, 4, 5, 6}, {2, 5, 8, 7}"),
    ("lst_contract_order", "sum += in[0][a * 4 + c] * in[1][c * 4 + b]",
     "sum += in[0][c * 4 + a] * in[1][c * 4 + b]"),
    ("lst_ascending_member", "for (int b = 0; b < 4; ++b)\n        for (int a = b; a < 4; ++a) {",
     "for (int a = 0; a < 4; ++a)\n        for (int b = a; b < 4; ++b) {"),
    ("lst_offset", "in[0][(i + 1) * 4 + c]", "in[0][i * 4 + c]"),
    ("lst_fixed", "in[1][c * 4 + 0]", "in[1][0 * 4 + c]"),
    ("spacetime_offset", "out[sym(i, j)] = in[0][sym4(i + 1, j + 1)]",
     "out[sym(i, j)] = in[0][sym4(i, j + 1)]"),
    ("spacetime_shift", "out[i] = in[0][sym4(i + 1, 0)]", "out[i] = in[0][sym4(i + 1, 1)]"),
]


def _run_all_pins(orc):
    failed = []
    for pin in pins.ALL_PINS:
        try:
            pin(orc)
        except Exception as e:           # a wrong result or a rejected shape
            failed.append(f"{pin.__name__}: {type(e).__name__}: {e}")
    return failed


@pytest.mark.parametrize("mid,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, mid, old, new):
    assert SRC.count(old) >= 1, f"mutation site for {mid} not found in oracle source"
    src = tmp_path / f"mut_{mid}.cpp"
    src.write_text(SRC.replace(old, new))
    lib = obuild.build(str(src), str(tmp_path / f"libmut_{mid}.so"))
    failed = _run_all_pins(oracle.Oracle(lib))
    assert failed, f"mutant {mid} passes every pin"


def test_unmutated_source_passes(tmp_path):
    lib = obuild.build(obuild.SRC, str(tmp_path / "libclean.so"))
    assert _run_all_pins(oracle.Oracle(lib)) == []
    assert os.path.exists(lib)
