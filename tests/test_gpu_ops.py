"""GPU: transposed products, upper-triangle products and the symmetric
square (the task types of Sec. 3.2 and 3.3), through the C ABI, against the
CPU oracle run on the transposed / mirrored inputs built by definition."""
import numpy as np
import pytest

import oracle
import workloads as wl
from tests._util import (compare, identity, positions, random_pattern, symmetric_from_upper, transpose,
                         upper_blocks)

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


def _blocks(h, n_rows, n_cols, b):
    I, J, V = h.to_blocks("f64")
    return wl.BlockMatrix(n_rows, n_cols, b, I, J, V)


def _check(C, ref, absref, tol):
    same, _, e_f, e_cw = compare(ref, C, absref)
    assert same, (ref.nnz, C.nnz)
    assert e_cw <= tol, e_cw
    return e_cw


@pytest.mark.parametrize("ta,tb", [(False, False), (True, False), (False, True), (True, True)])
@pytest.mark.parametrize("b,lb", [(32, 4), (64, 2), (16, 8)])
def test_transposed_products_f64(qt, ta, tb, b, lb):
    rng = np.random.default_rng(100 + 2 * ta + tb + b)
    m, k, n = 19, 27, 13
    A = random_pattern(rng, k if ta else m, m if ta else k, 0.15, b)   # op(A) is m x k blocks
    B = random_pattern(rng, n if tb else k, k if tb else n, 0.15, b)   # op(B) is k x n blocks
    opA = transpose(A) if ta else A
    opB = transpose(B) if tb else B
    _say("transposes", ta, tb, "b", b)
    ref, st = oracle.multiply(opA, opB, lb * b)
    absref, _ = oracle.multiply(opA, opB, lb * b, use_abs=True)
    hA, hB = qt.from_blockmatrix(A, lb * b), qt.from_blockmatrix(B, lb * b)
    hC = qt.multiply_ex(hA, hB, trans_a=ta, trans_b=tb)
    inf = hC.info()
    assert (inf["n_rows"], inf["n_cols"]) == (m * b, n * b)
    _check(_blocks(hC, m * b, n * b, b), ref, absref, 1e-12)
    assert hC.stats()["products"] == st.block_products
    assert hC.stats()["pairs"].tolist() == st.mul_tasks.tolist()


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
def test_transposed_products_reduced(qt, prec):
    rng = np.random.default_rng(7)
    b = 32
    A = random_pattern(rng, 30, 20, 0.2, b)
    B = random_pattern(rng, 30, 25, 0.2, b)
    ref, _ = oracle.multiply(transpose(A), B, 4 * b)
    absref, _ = oracle.multiply(transpose(A), B, 4 * b, use_abs=True)
    hC = qt.multiply_ex(qt.from_blockmatrix(A, 4 * b), qt.from_blockmatrix(B, 4 * b), trans_a=True, prec=prec)
    kmax = int(np.bincount(A.J, minlength=20).max())
    tol = (kmax * b + 2) * 2.0 ** -24 if prec == "f32" else 3 * 2.0 ** -16 + (3 * b + 4) * 2.0 ** -24
    _check(_blocks(hC, 20 * b, 25 * b, b), ref, absref, tol)


def test_upper_only_product(qt):
    rng = np.random.default_rng(8)
    b = 32
    A = random_pattern(rng, 45, 45, 0.08, b)
    B = random_pattern(rng, 45, 45, 0.08, b)
    full, _ = oracle.multiply(A, B, 8 * b)
    absfull, _ = oracle.multiply(A, B, 8 * b, use_abs=True)
    for leaf in (b, 4 * b, 8 * b):
        hC = qt.multiply_ex(qt.from_blockmatrix(A, leaf), qt.from_blockmatrix(B, leaf), upper=True)
        _check(_blocks(hC, A.n_rows, B.n_cols, b), upper_blocks(full), upper_blocks(absfull), 1e-12)
    with pytest.raises(qt.QtError) as e:
        R = random_pattern(rng, 5, 7, 0.5, b)
        qt.multiply_ex(qt.from_blockmatrix(R, b), qt.from_blockmatrix(random_pattern(rng, 7, 4, 0.5, b), b),
                       upper=True)
    assert e.value.status == qt.QT_ERR_SHAPE


def _sym_upper(rng, nb, fill, b):
    X = random_pattern(rng, nb, nb, fill, b)
    U = upper_blocks(X)
    V = U.V.copy()
    d = U.I == U.J
    V[d] = 0.5 * (V[d] + V[d].transpose(0, 2, 1))          # symmetric diagonal blocks
    return wl.BlockMatrix(U.n_rows, U.n_cols, b, U.I, U.J, V)


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3"])
def test_sysq(qt, prec):
    rng = np.random.default_rng(9)
    b = 32
    U = _sym_upper(rng, 50, 0.06, b)
    S = symmetric_from_upper(U)
    full, st = oracle.multiply(S, S, 4 * b)
    absfull, _ = oracle.multiply(S, S, 4 * b, use_abs=True)
    h = qt.from_blockmatrix(U, 4 * b)
    _say("sysq", prec)
    C = qt.sysq(h, prec)
    kmax = int(np.bincount(S.I, minlength=50).max())
    tol = {"f64": 1e-12, "f32": (kmax * b + 2) * 2.0 ** -24,
           "bf16x3": 3 * 2.0 ** -16 + (3 * b + 4) * 2.0 ** -24}[prec]
    _check(_blocks(C, U.n_rows, U.n_cols, b), upper_blocks(full), upper_blocks(absfull), tol)
    # about half the block products of the full square (Sec. 6.1: the expected speedup of 2)
    ratio = C.stats()["products"] / st.block_products
    assert 0.45 < ratio < 0.65, ratio


@pytest.mark.parametrize("ta,tb", [(True, False), (False, True), (True, True)])
@pytest.mark.parametrize("prec,b", [("f64", 32), ("f64", 16), ("f64", 64), ("f32", 32), ("f32", 64),
                                    ("bf16x3", 32), ("bf16x3", 64)])
def test_transposed_read_equals_explicit_transpose_bitwise(qt, prec, b, ta, tb):
    """op(A) op(B) read straight from the stored blocks (no transposed copy)
    is bitwise the plain product of operands transposed on the host: the
    transposed loads feed the MFMAs the same inner indices in the same order."""
    rng = np.random.default_rng(50 + b)
    nb = 23 if b < 64 else 11
    A = random_pattern(rng, nb, nb + 3, 0.12, b)            # op(A) is nb x (nb+3), or its transpose
    if ta and not tb:
        B = random_pattern(rng, nb, nb + 1, 0.12, b)
    elif tb and not ta:
        B = random_pattern(rng, nb + 2, nb + 3, 0.12, b)
    else:
        B = random_pattern(rng, nb + 1, nb, 0.12, b)
    leaf = 4 * b
    got = qt.multiply_ex(qt.from_blockmatrix(A, leaf), qt.from_blockmatrix(B, leaf), ta, tb, prec=prec)
    At = transpose(A) if ta else A
    Bt = transpose(B) if tb else B
    ref = qt.multiply(qt.from_blockmatrix(At, leaf), qt.from_blockmatrix(Bt, leaf), prec)
    I1, J1, V1 = got.to_blocks("f64")
    I2, J2, V2 = ref.to_blocks("f64")
    assert np.array_equal(I1, I2) and np.array_equal(J1, J2)
    assert np.array_equal(V1, V2)


@pytest.mark.parametrize("prec,b", [("f64", 16), ("f64", 64), ("f32", 64), ("bf16x3", 64)])
def test_sysq_block_sizes(qt, prec, b):
    rng = np.random.default_rng(60 + b)
    nb = 40 if b < 64 else 18
    U = _sym_upper(rng, nb, 0.08, b)
    S = symmetric_from_upper(U)
    full, st = oracle.multiply(S, S, 2 * b)
    absfull, _ = oracle.multiply(S, S, 2 * b, use_abs=True)
    C = qt.sysq(qt.from_blockmatrix(U, 2 * b), prec)
    kmax = int(np.bincount(S.I, minlength=nb).max())
    tol = {"f64": 1e-12, "f32": (kmax * b + 2) * 2.0 ** -24,
           "bf16x3": 3 * 2.0 ** -16 + (3 * b + 4) * 2.0 ** -24}[prec]
    _check(_blocks(C, U.n_rows, U.n_cols, b), upper_blocks(full), upper_blocks(absfull), tol)


def test_sysq_of_fp32_values_and_no_value_copy(qt):
    """The symmetric operand is structure only: its blocks are read from the
    triangle's own values (transposed for the mirrored ones), so the first
    qt_sysq of a handle obtains a few bytes per block, not a copy of the
    values; and an fp32 triangle (an fp32 multiply's result) works too."""
    import paper_1501_07800_amd as q
    rng = np.random.default_rng(61)
    b = 32
    U = _sym_upper(rng, 48, 0.08, b)
    h = qt.from_blockmatrix(U, 4 * b)
    qt.prepare(h, "f64")
    seen = []
    base = q.TorchAllocator()

    def alloc(n, st):
        seen.append(n)
        return base.alloc(n, st)
    q.set_allocator(alloc, base.free)
    try:
        C = qt.sysq(h, "f64")
    finally:
        if q.ALLOCATOR is not None:
            q.set_allocator(q.ALLOCATOR.alloc, q.ALLOCATOR.free)
        else:
            q.use_hip_pool()
    value_bytes = U.nnz * b * b * 8
    c_bytes = C.nblocks * b * b * 8
    # everything obtained beyond C's values: structure, scratch and product lists
    assert sum(seen) - c_bytes < 0.25 * value_bytes, (sum(seen), c_bytes, value_bytes)
    # an fp32 upper triangle: (U32)^2 through the f32 path
    Id = identity(48, b)
    h32 = qt.multiply(h, qt.from_blockmatrix(Id, 4 * b), "f32")     # U with fp32 values
    C32 = qt.sysq(h32, "f32")
    S = symmetric_from_upper(U)
    full, _ = oracle.multiply(S, S, 4 * b)
    absfull, _ = oracle.multiply(S, S, 4 * b, use_abs=True)
    kmax = int(np.bincount(S.I, minlength=48).max())
    _check(_blocks(C32, U.n_rows, U.n_cols, b), upper_blocks(full), upper_blocks(absfull),
           (kmax * b + 4) * 2.0 ** -24)


def test_sysq_decay_and_errors(qt):
    A = wl.decay3d(512, 16.0, 16, 32, seed=11)
    S = wl.BlockMatrix(A.n_rows, A.n_cols, 32, A.I, A.J, A.V)
    U = upper_blocks(S)
    Sm = symmetric_from_upper(U)
    full, _ = oracle.multiply(Sm, Sm, 256)
    absfull, _ = oracle.multiply(Sm, Sm, 256, use_abs=True)
    C = qt.sysq(qt.from_blockmatrix(U, 256))
    _check(_blocks(C, U.n_rows, U.n_cols, 32), upper_blocks(full), upper_blocks(absfull), 1e-12)
    with pytest.raises(qt.QtError) as e:
        qt.sysq(qt.from_blockmatrix(S, 256))               # holds blocks below the diagonal
    assert e.value.status == qt.QT_ERR_ARG
    rng = np.random.default_rng(0)
    with pytest.raises(qt.QtError) as e:
        qt.sysq(qt.from_blockmatrix(random_pattern(rng, 4, 6, 0.5, 32), 32))
    assert e.value.status == qt.QT_ERR_SHAPE


def test_add_matches_algorithm2_bitwise(qt):
    rng = np.random.default_rng(12)
    for b, leaf in ((32, 128), (16, 16), (64, 512)):
        A = random_pattern(rng, 30, 22, 0.2, b)
        B = random_pattern(rng, 30, 22, 0.2, b)
        ref, _ = oracle.add(A, B, leaf)
        hC = qt.add(qt.from_blockmatrix(A, leaf), qt.from_blockmatrix(B, leaf))
        C = _blocks(hC, A.n_rows, A.n_cols, b)
        assert np.array_equal(positions(C), positions(ref))
        assert np.array_equal(C.V, ref.V)                 # one fp64 addition per shared entry: exact
        # the sum is a full matrix handle: it multiplies like any other
        D = qt.multiply(hC, qt.from_blockmatrix(transpose(A), leaf))
        refD, _ = oracle.multiply(ref, transpose(A), leaf)
        absD, _ = oracle.multiply(wl.BlockMatrix(ref.n_rows, ref.n_cols, b, ref.I, ref.J, np.abs(ref.V)),
                                  wl.BlockMatrix(A.n_cols, A.n_rows, b, transpose(A).I, transpose(A).J,
                                                 np.abs(transpose(A).V)), leaf)
        _check(_blocks(D, A.n_rows, A.n_rows, b), refD, absD, 1e-12)
    empty = random_pattern(rng, 4, 4, 0.0, 32)
    X = random_pattern(rng, 4, 4, 0.5, 32)
    C = qt.add(qt.from_blockmatrix(empty, 64), qt.from_blockmatrix(X, 64))
    assert np.array_equal(_blocks(C, X.n_rows, X.n_cols, 32).V, X.V)


@pytest.mark.parametrize("a", [0.25, 0.6, 0.9])
def test_rmat_pair_counts_match_oracle(qt, a):
    """Per-level multiply pairs (the task counts of Sec. 5) on R-MAT patterns."""
    A = wl.rmat(9, 5, a, 16, seed=61)
    for leaf in (16, 64, 128):
        ref, st = oracle.multiply(A, A, leaf)
        h = qt.from_blockmatrix(A, leaf)
        C = qt.multiply(h, h)
        assert C.stats()["pairs"].tolist() == st.mul_tasks.tolist()
        assert C.stats()["products"] == st.block_products
        assert np.array_equal(positions(_blocks(C, A.n_rows, A.n_cols, 16)), positions(ref))


def test_truncate_matches_definition(qt):
    rng = np.random.default_rng(13)
    b = 32
    M = random_pattern(rng, 40, 40, 0.1, b)
    M.V *= np.exp(rng.uniform(-12, 0, size=(M.nnz, 1, 1)))      # well separated block norms
    n2 = np.sort((M.V.reshape(M.nnz, -1) ** 2).sum(1))
    cums = np.cumsum(n2)
    h = qt.from_blockmatrix(M, 4 * b)
    for k_target in (0, 1, 7, M.nnz // 2, M.nnz - 1, M.nnz):
        # eps between the cumulative sums, far from either
        lo = cums[k_target - 1] if k_target > 0 else 0.0
        hi = cums[k_target] if k_target < M.nnz else 2 * cums[-1] + 1.0
        eps = float(np.sqrt(0.5 * (lo + hi))) if k_target > 0 else float(np.sqrt(0.5 * cums[0]))
        ref, k = oracle.truncate(M, eps)
        T, removed, e2 = qt.truncate(h, eps)
        assert removed == k == k_target
        got = _blocks(T, M.n_rows, M.n_cols, b)
        assert np.array_equal(positions(got), positions(wl.BlockMatrix(M.n_rows, M.n_cols, b, *_sorted(ref))))
        assert np.array_equal(got.V, _sorted(ref)[2])
        assert e2 < eps * eps and abs(e2 - lo) <= 1e-12 * max(lo, 1e-300)


def test_truncate_equal_norms_follow_z_order(qt):
    """All blocks of equal norm: which ones go is decided by the tie rule
    (quadtree Z order first), the same on the GPU as in the oracle."""
    rng = np.random.default_rng(14)
    b = 16
    M = random_pattern(rng, 64, 64, 0.2, b)
    M.V[:] = 0.0
    M.V[:, 0, 0] = 1.0
    h = qt.from_blockmatrix(M, 4 * b)
    for k_target in (1, 5, M.nnz // 3, M.nnz - 1):
        eps = float(np.sqrt(k_target + 0.5))
        ref, k = oracle.truncate(M, eps)
        T, removed, _ = qt.truncate(h, eps)
        assert removed == k == k_target
        got = _blocks(T, M.n_rows, M.n_cols, b)
        assert np.array_equal(positions(got), positions(wl.BlockMatrix(M.n_rows, M.n_cols, b, *_sorted(ref))))


def _sorted(M):
    o = np.lexsort((M.J, M.I))
    return M.I[o], M.J[o], M.V[o]


def test_probe_mfma_rates(qt):
    """The register-only MFMA loop runs and reports rates of the right order
    (published dense peaks: fp64 78.6, fp32 157.3, bf16 2516.6 TFLOP/s)."""
    f64 = qt.probe_mfma("f64")
    f32 = qt.probe_mfma("f32")
    bf = qt.probe_mfma("bf16x3")
    print("probe TFLOP/s", f64, f32, bf, flush=True)
    assert 10.0 < f64 < 80.0
    assert 20.0 < f32 < 160.0
    assert 200.0 < bf < 2600.0


@pytest.mark.parametrize("prec,b", [("f64", 16), ("f64", 32), ("f64", 64), ("f32", 16), ("f32", 32), ("f32", 64),
                                    ("bf16x3", 32), ("bf16x3", 64)])
def test_probe_batched_rates(qt, prec, b):
    """The batched-GEMM practical peak (64000 uniform products) runs through
    the numeric kernels at a rate below the published MFMA peak."""
    peak = {"f64": 78.6, "f32": 157.3, "bf16x3": 157.3}[prec]
    tf = qt.probe_batched(prec, b, 64000)
    print("batched", prec, b, tf, flush=True)
    assert 0.5 < tf <= 1.05 * peak


def test_probe_batched_errors(qt):
    import ctypes
    out = ctypes.c_double()
    L = qt.lib
    assert L.qt_probe_batched(0, 48, 100, None, ctypes.byref(out)) == qt.QT_ERR_SHAPE
    assert L.qt_probe_batched(0, 32, 0, None, ctypes.byref(out)) == qt.QT_ERR_ARG
    assert L.qt_probe_batched(2, 16, 100, None, ctypes.byref(out)) == qt.QT_ERR_UNSUPPORTED
    assert L.qt_probe_batched(7, 32, 100, None, ctypes.byref(out)) == qt.QT_ERR_ARG
