"""Plant plausible mistakes in a copy of the oracle and check the pins catch each.

The mistakes are planted on the CPU, in a temporary copy of ``pwa_oracle.c``
compiled next to the test; the real oracle is never modified.  A mutation
that every pin let through would mean the pins do not fix that part of the
oracle.
"""
import pytest

import oracle
import pins

# (name, text in pwa_oracle.c, replacement)
MUTATIONS = [
    ("table_drops_conj",
     "A[i * W + a] * conj(A[i * W + ap]);", "A[i * W + a] * A[i * W + ap];"),
    ("hermitian_completion_no_conj",
     "return conj(Ti[packed_index(W, ap, a)]);", "return Ti[packed_index(W, ap, a)];"),
    ("packed_index_off_by_row",
     "- (int64_t)a * (a - 1) / 2", "- (int64_t)a * (a + 1) / 2"),
    ("intensity_conj_on_wrong_v",
     "s += V[a] * conj(V[ap]) * table_entry(Ti, W, a, ap);",
     "s += conj(V[a]) * V[ap] * table_entry(Ti, W, a, ap);"),
    ("amplitude_intensity_conj_v",
     "for (int32_t a = 0; a < W; ++a) s += V[a] * A[i * W + a];\n        Iout",
     "for (int32_t a = 0; a < W; ++a) s += conj(V[a]) * A[i * W + a];\n        Iout"),
    ("mc_matrix_conj_wrong_side",
     "cplx x = B[j * W + a] * conj(B[j * W + ap]);", "cplx x = conj(B[j * W + a]) * B[j * W + ap];"),
    ("mc_matrix_divides_by_accepted",
     "/ (double)n_gen;", "/ (double)n_acc;"),
    ("mc_term_transposed",
     "cplx x = V[a] * conj(V[ap]) * M[a * W + ap];", "cplx x = V[a] * conj(V[ap]) * M[ap * W + a];"),
    ("data_term_sign",
     "*nll = -sum_ln +", "*nll = sum_ln +"),
    ("amp_data_term_sign",
     "*nll = -nsum_value(&d) +", "*nll = nsum_value(&d) +"),
    ("gradient_missing_factor_two",
     "g *= 2.0;", "g *= 1.0;"),
    ("gradient_transposed_matrix",
     "g += V[a] * (M[a * W + b] - U[a * W + b]);", "g += V[a] * (M[b * W + a] - U[b * W + a]);"),
    ("gradient_sign_of_data_part",
     "g += V[a] * (M[a * W + b] - U[a * W + b]);", "g += V[a] * (M[a * W + b] + U[a * W + b]);"),
    ("amp_gradient_drops_conj",
     "cplx x = s * conj(A[i * W + b]) / Ii;", "cplx x = s * A[i * W + b] / Ii;"),
    ("amp_gradient_mc_part_transposed",
     "mv += V[a] * M[a * W + b];", "mv += V[a] * M[b * W + a];"),
    ("log_base_ten",
     "nsum_add(&dpart[c], log(Ii));\n            if (!upart)", "nsum_add(&dpart[c], log10(Ii));\n            if (!upart)"),
    ("degenerate_clamped",
     "if (!(Ii > 0.0) || !isfinite(Ii)) { bad[c]++; continue; }\n            nsum_add(&dpart[c], log(Ii));\n            if (!gpart)",
     "if (!(Ii > 0.0) || !isfinite(Ii)) { Ii = 1e-300; }\n            nsum_add(&dpart[c], log(Ii));\n            if (!gpart)"),
    ("fumili_im_sign",
     "J[2 * b + 1] = -2.0 * cimag(z) / Ii;", "J[2 * b + 1] = 2.0 * cimag(z) / Ii;"),
    ("fumili_drops_conj",
     "cplx z = conj(s) * A[i * W + b];", "cplx z = s * A[i * W + b];"),
    ("fumili_factor_two",
     "J[2 * b] = 2.0 * creal(z) / Ii;", "J[2 * b] = creal(z) / Ii;"),
    ("fumili_drops_last_chunk",
     "for (int64_t c = 0; c < nc; ++c) nsum_add(&t, nsum_value(&hpart[c * P * P + p * P + q]));",
     "for (int64_t c = 0; c + 1 < nc; ++c) nsum_add(&t, nsum_value(&hpart[c * P * P + p * P + q]));"),
    ("chunk_partials_dropped",
     "for (int64_t c = 0; c < nc; ++c) { nsum_add(&d, nsum_value(&dpart[c])); nbad += bad[c]; }\n    cplx* U",
     "for (int64_t c = 0; c + 1 < nc; ++c) { nsum_add(&d, nsum_value(&dpart[c])); nbad += bad[c]; }\n    cplx* U"),
]


def _mutant(tmp_path, name, old, new):
    src = open(oracle.SOURCE).read()
    assert src.count(old) == 1, "mutation %s does not match exactly once" % name
    path = tmp_path / ("%s.c" % name)
    path.write_text(src.replace(old, new))
    lib = tmp_path / ("lib_%s.so" % name)
    oracle.build(str(path), str(lib))
    return oracle.Oracle(oracle.load(str(lib)))


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_mutation_is_caught(tmp_path, name, old, new):
    o = _mutant(tmp_path, name, old, new)
    caught = []
    for pin in pins.ALL_PINS:
        try:
            pin(o)
        except AssertionError:
            caught.append(pin.__name__)
    assert caught, "no pin catches the planted mistake %r" % name


def test_unmutated_copy_passes(tmp_path):
    """Control: the copy-and-compile route itself does not break the pins."""
    src = open(oracle.SOURCE).read()
    path = tmp_path / "copy.c"
    path.write_text(src)
    lib = tmp_path / "lib_copy.so"
    oracle.build(str(path), str(lib))
    o = oracle.Oracle(oracle.load(str(lib)))
    for pin in pins.ALL_PINS:
        pin(o)
