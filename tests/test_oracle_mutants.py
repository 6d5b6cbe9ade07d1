"""Planted mistakes in a copy of the oracle must fail its pins.

Each mutant is a plausible slip (a transposed operand, a dropped term, a wrong
sign, a wrong index, a lost NIL rule). The copy is compiled on the CPU into a
temporary directory; the pins of ``test_oracle_pins`` (dense product,
boolean pattern, hand-derived counts) are run against it and at least one
must fail.
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as wl
from tests._util import norm_thresholded_by_definition, positions, random_pattern, tau_in_gap, to_dense

MUTANTS = {
    "B child index transposed": ("const qo_node *x = B->child[2 * k + n];",
                                 "const qo_node *x = B->child[2 * n + k];"),
    "second product of C_mn dropped": ("qo_node *s = qt_add(ctx, level + 1, Y[q][0], Y[q][1]);",
                                       "tree_free(Y[q][1], ctx->lb, 1); "
                                       "qo_node *s = qt_add(ctx, level + 1, Y[q][0], NULL);"),
    "last inner leaf index skipped": ("for (int k = 0; k < lb; ++k) {",
                                      "for (int k = 0; k + 1 < lb || (lb == 1 && k < 1); ++k) {"),
    "block product B transposed": ("x = B[t * b + c];", "x = B[c * b + t];"),
    "leaf add sign": ("X->blk[q][e] += Y->blk[q][e];", "X->blk[q][e] -= Y->blk[q][e];"),
    "leaf block placement transposed": ("n->blk[i * lb + j] = (double *)(V",
                                        "n->blk[j * lb + i] = (double *)(V"),
    "empty leaf product kept": ("if (!any) { tree_free(X, lb, 1); return NULL; }\n    return X;",
                                "return X;"),
    "local block sum restarts per t": ("s += a * x;", "s = a * x;"),
    "abs mode drops B's absolute value": ("if (use_abs) { a = fabs(a); x = fabs(x); }",
                                          "if (use_abs) { a = fabs(a); }"),
    "task norm rule reads A twice": ("if (A->n2 * B->n2 < ctx->tau2) {", "if (A->n2 * A->n2 < ctx->tau2) {"),
    "block norm rule transposes B's block": ("if (A->bn2[i * lb + k] * B->bn2[k * lb + j] < ctx->tau2)",
                                             "if (A->bn2[i * lb + k] * B->bn2[j * lb + k] < ctx->tau2)"),
    "block norm not squared": ("for (int e = 0; e < b * b; ++e) s += x[e] * x[e];",
                               "for (int e = 0; e < b * b; ++e) s += fabs(x[e]);"),
    "node norm keeps only the last child": ("if (n->child[q]) n->n2 += n->child[q]->n2;",
                                            "if (n->child[q]) n->n2 = n->child[q]->n2;"),
}


def _graded(rng, nbr, nbc, fill, b):
    M = random_pattern(rng, nbr, nbc, fill, b)
    scale = 10.0 ** rng.uniform(-6, 0, size=M.nnz)
    return wl.BlockMatrix(M.n_rows, M.n_cols, b, M.I, M.J, M.V * scale[:, None, None])


def _battery(lib):
    """Return True if every pin passes for this compiled oracle."""
    try:
        return _run_pins(lib)
    except Exception:          # a mutant may also produce blocks outside the matrix
        return False


def _run_pins(lib):
    rng = np.random.default_rng(2024)
    ok = True
    for b, lb in ((3, 1), (3, 2), (2, 4), (4, 8)):
        A = random_pattern(rng, 9, 13, 0.4, b)
        B = random_pattern(rng, 13, 7, 0.4, b)
        C, st = oracle.multiply(A, B, lb * b, lib=lib)
        Ad, Bd = to_dense(A), to_dense(B)
        ref = Ad @ Bd
        bound = np.abs(Ad) @ np.abs(Bd)
        ok &= bool(np.all(np.abs(to_dense(C) - ref) <= 1e-13 * bound))
        ok &= np.array_equal(positions(C), oracle.pattern_by_definition(A, B))
        Cabs, _ = oracle.multiply(A, B, lb * b, use_abs=True, lib=lib)
        ok &= bool(np.all(np.abs(to_dense(Cabs) - bound) <= 1e-13 * bound))
    # the norm-thresholded product against its definition (graded block norms)
    for b, lb, q in ((4, 2, 0.3), (2, 4, 0.6), (4, 8, 0.8)):
        A = _graded(rng, 20, 24, 0.3, b)
        B = _graded(rng, 24, 18, 0.3, b)
        tau = tau_in_gap(A, B, q)
        ref, kept, _, _ = norm_thresholded_by_definition(A, B, tau)
        C, st = oracle.multiply(A, B, lb * b, tau=tau, lib=lib)
        ok &= np.array_equal(positions(C), positions(ref)) and st.block_products == kept
        if np.array_equal(positions(C), positions(ref)):
            ok &= bool(np.allclose(C.V, ref.V, rtol=1e-12, atol=1e-300))
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "banded1024_counts.json")))
    A = wl.config("banded1024")
    C, st = oracle.multiply(A, A, 256, lib=lib)
    ok &= (st.block_products == g["block_products"] and C.nnz == g["nnz_C"]
           and st.mul_tasks.tolist() == g["mul_tasks_per_level"]
           and st.c_nodes.tolist() == g["c_nodes_per_level"])
    return bool(ok)


def test_unmutated_copy_passes(tmp_path):
    src = open(oracle._SRC).read()
    p = tmp_path / "o.c"
    p.write_text(src)
    lib = oracle.load(oracle.build(str(p), str(tmp_path / "o.so")))
    assert _battery(lib)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    src = open(oracle._SRC).read()
    assert src.count(old) == 1, name
    p = tmp_path / "m.c"
    p.write_text(src.replace(old, new))
    lib = oracle.load(oracle.build(str(p), str(tmp_path / "m.so")))
    assert not _battery(lib), name
