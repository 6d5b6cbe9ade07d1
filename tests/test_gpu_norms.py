"""GPU: per-submatrix Frobenius norms and the norm-thresholded product, through the C ABI.

qt_norms is checked against numpy's sums of squares; qt_multiply_tau against
the oracle's norm-thresholded product (pattern exact, values within the fp64
bound, the same number of block products) at thresholds that no block
product's norm lies near, against the plain product at tau = 0 (bitwise), and
against the bound sum of the dropped products' norms.
"""
import numpy as np
import pytest

import oracle
import workloads as wl
from tests._util import compare, norm_thresholded_by_definition, random_pattern, tau_in_gap

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1501_07800_amd as q
    return q


def _say(*a):
    print(*a, flush=True)


def _graded(rng, nbr, nbc, fill, b):
    M = random_pattern(rng, nbr, nbc, fill, b)
    scale = 10.0 ** rng.uniform(-6, 0, size=M.nnz)
    return wl.BlockMatrix(M.n_rows, M.n_cols, b, M.I, M.J, M.V * scale[:, None, None])


def _blocks(h, A, B):
    I, J, V = h.to_blocks("f64")
    return wl.BlockMatrix(A.n_rows, B.n_cols, A.b, I, J, V)


@pytest.mark.parametrize("b", [16, 32, 64])
def test_norms_match_numpy(qt, b):
    rng = np.random.default_rng(60 + b)
    A = _graded(rng, 23, 17, 0.3, b)
    h = qt.from_blockmatrix(A, 4 * b)
    bn, tot = h.norms()
    o = np.lexsort((A.J, A.I))
    ref = (A.V[o].reshape(A.nnz, -1) ** 2).sum(axis=1)
    assert np.allclose(bn, ref, rtol=1e-14, atol=0)
    assert tot == pytest.approx(float((A.V ** 2).sum()), rel=1e-13)
    # an fp32 multiply result: the norms of its fp32 values
    C = qt.multiply(h, qt.from_blockmatrix(_graded(rng, 17, 9, 0.4, b), 4 * b), "f32")
    I, J, V = C.to_blocks("f32")
    cb, ct = C.norms()
    ref = (V.astype(np.float64).reshape(len(I), -1) ** 2).sum(axis=1)
    assert np.allclose(cb, ref, rtol=1e-13, atol=0)
    assert ct == pytest.approx(float(ref.sum()), rel=1e-12)
    # all NIL
    E = qt.build(4 * b, 4 * b, b, b, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros((0, b, b)))
    eb, et = E.norms()
    assert len(eb) == 0 and et == 0.0


@pytest.mark.parametrize("b,lb,q", [(16, 2, 0.3), (32, 4, 0.6), (32, 1, 0.5), (64, 2, 0.8), (16, 8, 0.9)])
def test_multiply_tau_matches_oracle(qt, b, lb, q):
    rng = np.random.default_rng(70 + lb + b)
    A = _graded(rng, 40, 48, 0.12, b)
    B = _graded(rng, 48, 36, 0.12, b)
    tau = tau_in_gap(A, B, q)
    leaf = lb * b
    _say("multiply_tau b", b, "leaf", leaf, "tau", tau)
    ref, st = oracle.multiply(A, B, leaf, tau=tau)
    absAB, _ = oracle.multiply(A, B, leaf, use_abs=True, tau=tau)
    hA, hB = qt.from_blockmatrix(A, leaf), qt.from_blockmatrix(B, leaf)
    hC = qt.multiply_tau(hA, hB, tau)
    got = _blocks(hC, A, B)
    same, _, _, e_cw = compare(ref, got, absAB)
    assert same, (ref.nnz, got.nnz)
    assert e_cw <= 1e-12
    stats = hC.stats()
    assert stats["products"] == st.block_products
    full = qt.multiply(hA, hB).stats()
    assert 0 < stats["products"] < full["products"]
    assert sum(stats["pairs"]) <= sum(full["pairs"])
    # C = A*B minus the dropped products, within the sum of their norms
    _, _, _, bound = norm_thresholded_by_definition(A, B, tau)
    Cx, _ = oracle.multiply(A, B, leaf)
    from tests._util import to_dense
    assert np.linalg.norm(to_dense(Cx) - to_dense(got)) <= bound * (1 + 1e-9)


def test_multiply_tau_lifted_operand(qt):
    """A tall A (70 x 9 blocks) times a small B (9 x 12): B's quadtree is
    lifted by several levels, where its root norm stands for every level
    above it."""
    rng = np.random.default_rng(75)
    A = _graded(rng, 70, 9, 0.3, 16)
    B = _graded(rng, 9, 12, 0.5, 16)
    tau = tau_in_gap(A, B, 0.5)
    ref, st = oracle.multiply(A, B, 32, tau=tau)
    C = qt.multiply_tau(qt.from_blockmatrix(A, 32), qt.from_blockmatrix(B, 32), tau)
    got = _blocks(C, A, B)
    same, _, e_f, _ = compare(ref, got)
    assert same and e_f <= 1e-13
    assert C.stats()["products"] == st.block_products
    # and the other way round: B^T A^T with the lifted operand on the left
    from tests._util import transpose
    At, Bt = transpose(A), transpose(B)
    ref2, st2 = oracle.multiply(Bt, At, 32, tau=tau)
    C2 = qt.multiply_tau(qt.from_blockmatrix(Bt, 32), qt.from_blockmatrix(At, 32), tau)
    same, _, e_f, _ = compare(ref2, _blocks(C2, Bt, At))
    assert same and e_f <= 1e-13 and C2.stats()["products"] == st2.block_products == st.block_products


def test_multiply_tau_zero_is_the_product_and_large_tau_empties(qt):
    rng = np.random.default_rng(80)
    A = _graded(rng, 30, 30, 0.15, 32)
    h = qt.from_blockmatrix(A, 128)
    I0, J0, V0 = qt.multiply(h, h).to_blocks()
    I1, J1, V1 = qt.multiply_tau(h, h, 0.0).to_blocks()
    assert np.array_equal(I0, I1) and np.array_equal(J0, J1) and np.array_equal(V0, V1)
    big = 2.0 * float((A.V ** 2).sum())
    E = qt.multiply_tau(h, h, big)
    assert E.info()["nblocks"] == 0 and E.stats()["products"] == 0 and E.levels().sum() == 0
    with pytest.raises(qt.QtError):
        qt.multiply_tau(h, h, float("nan"))


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
def test_multiply_tau_reduced_precision(qt, prec):
    rng = np.random.default_rng(81)
    A = _graded(rng, 36, 36, 0.15, 32)
    tau = tau_in_gap(A, A, 0.5)
    ref, st = oracle.multiply(A, A, 128, tau=tau)
    h = qt.from_blockmatrix(A, 128)
    C = qt.multiply_tau(h, h, tau, prec)
    got = _blocks(C, A, A)
    same, _, e_f, _ = compare(ref, got)
    assert same
    assert e_f <= (1e-5 if prec == "f32" else 1e-4)
    assert C.stats()["products"] == st.block_products


def test_multiply_tau_decay_workload(qt):
    """On a decay matrix (entries exp(-d^2/2) of atom distances) a small
    threshold drops the many products of far-apart blocks and keeps C's
    large entries: the oracle's rule, pattern exact."""
    A = wl.decay3d(768, 18.0, 16, 32, seed=21)
    nrm = np.linalg.norm(A.V.reshape(A.nnz, -1), axis=1)
    tau = tau_in_gap(A, A, 0.4)
    ref, st = oracle.multiply(A, A, 256, tau=tau)
    h = qt.from_blockmatrix(A, 256)
    C = qt.multiply_tau(h, h, tau)
    got = _blocks(C, A, A)
    absAB, _ = oracle.multiply(A, A, 256, use_abs=True, tau=tau)
    same, _, _, e_cw = compare(ref, got, absAB)
    assert same and e_cw <= 1e-12
    full = qt.multiply(h, h).stats()["products"]
    _say("decay tau", tau, "max block norm", nrm.max(), "products", st.block_products, "of", full)
    assert C.stats()["products"] == st.block_products < full
