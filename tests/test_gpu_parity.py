"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Patterns must match exactly. FP64 values must be within 1e-12 of the oracle
componentwise, relative to |A||B|, and normwise. The FP32 and split-BF16
paths are held to a-priori bounds derived from their roundings:
  fp32:    (k*b + 2) * 2^-24 * (|A||B|)_ij   (k = products in the C block)
  bf16x3:  (3*2^-16 + (3b + 4) * 2^-24) * (|A||B|)_ij
"""
import numpy as np
import pytest

import oracle
import workloads as wl
from tests._util import compare, positions, random_pattern

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


@pytest.fixture(scope="module")
def qt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1501_07800_amd as q
    return q


def _say(*a):
    print(*a, flush=True)


def gpu_multiply(qt, A, B, leaf, prec="f64", same=False):
    hA = qt.from_blockmatrix(A, leaf)
    hB = hA if same else qt.from_blockmatrix(B, leaf)
    hC = qt.multiply(hA, hB, prec)
    I, J, V = hC.to_blocks("f64")
    st = hC.stats()
    C = wl.BlockMatrix(A.n_rows, B.n_cols, A.b, I, J, V)
    return C, st, hC


def check_f64(qt, A, B, leaf, same=False, check_counts=True):
    _say("f64", A.n_rows, A.n_cols, B.n_cols, "b", A.b, "leaf", leaf, "nnz", A.nnz, B.nnz)
    ref, ost = oracle.multiply(A, B, leaf)
    absAB, _ = oracle.multiply(A, B, leaf, use_abs=True)
    C, st, hC = gpu_multiply(qt, A, B, leaf, "f64", same)
    same_pat, e_max, e_f, e_cw = compare(ref, C, absAB)
    assert same_pat, (ref.nnz, C.nnz)
    assert e_cw <= TOL64, e_cw
    assert e_f <= TOL64, e_f
    assert st["products"] == ost.block_products
    # C's quadtree: the non-NIL nodes of every level, as Algorithm 1 forms them
    # with zero submatrices NIL at every level (Sec. 3.1)
    assert hC.levels().tolist() == ost.c_nodes.tolist()
    if check_counts:
        assert st["pairs"].tolist() == ost.mul_tasks.tolist()
    return ref, C


def test_round_trip_bit_exact(qt):
    rng = np.random.default_rng(0)
    for b, leaf, nbr, nbc in ((16, 64, 13, 21), (32, 256, 40, 9), (64, 64, 5, 5)):
        A = random_pattern(rng, nbr, nbc, 0.3, b)
        _say("round trip", b, leaf, nbr, nbc)
        h = qt.from_blockmatrix(A, leaf)
        I, J, V = h.to_blocks("f64")
        assert np.array_equal(I, A.I) and np.array_equal(J, A.J) and np.array_equal(V, A.V)
        I, J, V32 = h.to_blocks("f32")
        assert np.array_equal(V32, A.V.astype(np.float32))
        assert h.info()["nblocks"] == A.nnz


def test_round_trip_device_arrays(qt):
    import torch
    rng = np.random.default_rng(1)
    A = random_pattern(rng, 30, 30, 0.2, 32)
    perm = rng.permutation(A.nnz)            # any input order
    dev = torch.device("cuda")
    I = torch.from_numpy(A.I[perm].copy()).to(dev)
    J = torch.from_numpy(A.J[perm].copy()).to(dev)
    V = torch.from_numpy(A.V[perm].copy()).to(dev)
    h = qt.build(A.n_rows, A.n_cols, 32, 128, I, J, V)
    oI = torch.empty_like(I)
    oJ = torch.empty_like(J)
    oV = torch.empty_like(V)
    h.to_blocks_device(oI, oJ, oV)
    torch.cuda.synchronize()
    assert np.array_equal(oI.cpu().numpy(), A.I)
    assert np.array_equal(oJ.cpu().numpy(), A.J)
    assert np.array_equal(oV.cpu().numpy(), A.V)


def test_build_errors(qt):
    b = 16
    V = np.ones((2, b, b))
    with pytest.raises(qt.QtError) as e:
        qt.build(64, 64, b, 32, np.array([0, 4], np.int32), np.array([0, 0], np.int32), V)
    assert e.value.status == qt.QT_ERR_ARG
    with pytest.raises(qt.QtError) as e:
        qt.build(64, 64, b, 32, np.array([1, 1], np.int32), np.array([2, 2], np.int32), V)
    assert e.value.status == qt.QT_ERR_DUPLICATE
    A = qt.build(64, 48, b, 32, np.array([0], np.int32), np.array([0], np.int32), V[:1])
    B = qt.build(64, 64, b, 32, np.array([0], np.int32), np.array([0], np.int32), V[:1])
    with pytest.raises(qt.QtError) as e:
        qt.multiply(A, B)                     # 48 columns vs 64 rows
    assert e.value.status == qt.QT_ERR_SHAPE
    C = qt.build(48, 48, b, 16, np.array([0], np.int32), np.array([0], np.int32), V[:1])
    with pytest.raises(qt.QtError) as e:
        qt.multiply(A, C)                     # leaf sizes differ
    assert e.value.status == qt.QT_ERR_SHAPE


def test_banded1024_f64(qt):
    A = wl.config("banded1024")
    ref, C = check_f64(qt, A, A, 256, same=True)
    assert C.nnz == 374


def test_banded1024_c_tree_matches_golden(qt):
    """C's non-NIL nodes per level equal the hand-derived counts of the
    banded workload: 4 of its 14 leaf pair groups yield no block product and
    are NIL (golden file, derived by hand from the band structure)."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "banded1024_counts.json")))
    A = wl.config("banded1024")
    hA = qt.from_blockmatrix(A, 256)
    hC = qt.multiply(hA, hA)
    assert hC.levels().tolist() == g["c_nodes_per_level"]
    assert hC.stats()["pairs"].tolist() == g["mul_tasks_per_level"]
    assert hC.nblocks == g["nnz_C"]


@pytest.mark.parametrize("case", ["banded", "decay", "random"])
def test_chained_pair_counts_match_oracle(qt, case):
    """D = C*A with the multiply result C as an operand: the traversal of D
    walks C's tree, so its pairs per level (the multiply tasks of Algorithm 1
    at each level) equal the oracle's only if C's tree holds no empty node."""
    if case == "banded":
        A, leaf = wl.config("banded1024"), 256
    elif case == "decay":
        A, leaf = wl.decay3d(1024, 25.0, 16, 32, seed=17), 128
    else:
        A, leaf = wl.random_blocks(256, 256, 600, 32, seed=18), 128
    _say("chained pair counts", case, A.n_rows, A.nnz, leaf)
    ref_C, st_C = oracle.multiply(A, A, leaf)
    ref_D, st_D = oracle.multiply(ref_C, A, leaf)
    hA = qt.from_blockmatrix(A, leaf)
    hC = qt.multiply(hA, hA)
    assert hC.levels().tolist() == st_C.c_nodes.tolist()
    hD = qt.multiply(hC, hA)
    st = hD.stats()
    assert st["pairs"].tolist() == st_D.mul_tasks.tolist()
    assert st["products"] == st_D.block_products
    assert hD.levels().tolist() == st_D.c_nodes.tolist()
    I, J = hD.pattern()
    assert np.array_equal(I, ref_D.I) and np.array_equal(J, ref_D.J)


def test_exact_cancellation_keeps_block(qt):
    """A C block whose block products cancel exactly stays present with value
    zero: sparsity is detected from the structure only, never from values.
    C(0,0) = X Y + X (-Y) with small integer entries, so both the oracle's and
    the GPU's sums are exact zeros; C(0,1) = X Y' is an ordinary block."""
    b = 32
    rng = np.random.default_rng(19)
    X = rng.integers(-3, 4, (b, b)).astype(np.float64)
    Y = rng.integers(-3, 4, (b, b)).astype(np.float64)
    Y2 = rng.integers(-3, 4, (b, b)).astype(np.float64)
    n = 4 * b
    A = wl.BlockMatrix(n, n, b, np.array([0, 0], np.int32), np.array([0, 1], np.int32), np.stack([X, X]))
    B = wl.BlockMatrix(n, n, b, np.array([0, 0, 1], np.int32), np.array([0, 1, 0], np.int32),
                       np.stack([Y, Y2, -Y]))
    ref, st = oracle.multiply(A, B, 2 * b)
    assert ref.nnz == 2 and np.all(ref.V[0] == 0.0)
    for prec in ("f64", "f32", "bf16x3"):
        hA, hB = qt.from_blockmatrix(A, 2 * b), qt.from_blockmatrix(B, 2 * b)
        hC = qt.multiply(hA, hB, prec)
        I, J, V = hC.to_blocks("f64")
        assert I.tolist() == [0, 0] and J.tolist() == [0, 1], prec
        assert np.all(V[0] == 0.0), prec
        assert np.array_equal(V[1], X @ Y2), prec      # integers below 2^24: exact in every path
        assert hC.levels().tolist() == st.c_nodes.tolist()


@pytest.mark.parametrize("b", [16, 32, 64])
@pytest.mark.parametrize("lb", [1, 2, 8])
def test_random_shapes_f64(qt, b, lb):
    rng = np.random.default_rng(10 * b + lb)
    # rectangular, dimensions not multiples of the leaf (ragged tail)
    nbr, nbk, nbc = (37, 29, 45) if b < 64 else (19, 13, 23)
    for fill in (0.03, 0.25):
        A = random_pattern(rng, nbr, nbk, fill, b)
        B = random_pattern(rng, nbk, nbc, fill, b)
        check_f64(qt, A, B, lb * b)


def test_depth_mismatch_f64(qt):
    rng = np.random.default_rng(3)
    A = random_pattern(rng, 3, 70, 0.5, 32)      # wide: deeper tree than A's row count needs
    B = random_pattern(rng, 70, 2, 0.5, 32)      # tall: deeper than its column count needs
    check_f64(qt, A, B, 64)                      # C is 3 x 2 blocks, both operands deeper than C
    X = random_pattern(rng, 2, 3, 0.8, 32)       # shallow times deep
    check_f64(qt, X, A, 64)
    check_f64(qt, B, X, 64)                      # deep times shallow


def test_wide_levels(qt):
    """Levels wider than one workgroup per node allows: b = 16 blocks, one
    block per leaf, 2048 x 2048 blocks at 1 % fill (11 levels). The deepest
    tree levels and the leaf level hold 10^5 to 10^6 C nodes, so their
    kernels run four nodes per workgroup, the widest fall back from workgroup
    aggregates to a separate scan, and the level above the first wide one
    does not make the next level's counts in its fill. Pattern, values, pair
    counts and C's nodes per level against the oracle, for A*A and A^T*A."""
    from tests._util import transpose
    A = wl.random_blocks(2048, 2048, 41943, 16, seed=41)
    ref, C = check_f64(qt, A, A, 16, same=True)
    _say("wide levels: C blocks", C.nnz)
    assert C.nnz > 300000    # the leaf level is past the aggregate path
    At = transpose(A)
    ref_t, ost_t = oracle.multiply(At, A, 16)
    hA = qt.from_blockmatrix(A, 16)
    hCt = qt.multiply_ex(hA, hA, trans_a=True)
    I, J, V = hCt.to_blocks("f64")
    got = wl.BlockMatrix(A.n_cols, A.n_cols, 16, I, J, V)
    same_pat, _, e_f, _ = compare(ref_t, got)
    assert same_pat and e_f <= TOL64
    assert hCt.stats()["pairs"].tolist() == ost_t.mul_tasks.tolist()
    assert hCt.levels().tolist() == ost_t.c_nodes.tolist()


def test_leaf_size_independent_bitwise(qt):
    rng = np.random.default_rng(4)
    A = random_pattern(rng, 96, 96, 0.06, 32)
    outs = []
    for leaf in (32, 64, 128, 256):
        C, _, _ = gpu_multiply(qt, A, A, leaf, "f64", same=True)
        outs.append(C)
    for C in outs[1:]:
        assert np.array_equal(positions(C), positions(outs[0]))
        assert np.array_equal(C.V, outs[0].V)


def test_empty_and_degenerate(qt):
    rng = np.random.default_rng(5)
    A = random_pattern(rng, 8, 8, 0.3, 32)
    Z = random_pattern(rng, 8, 8, 0.0, 32)
    for X, Y in ((A, Z), (Z, A), (Z, Z)):
        C, st, h = gpu_multiply(qt, X, Y, 64)
        assert C.nnz == 0 and st["products"] == 0
    # no shared inner index: every pair of leaves is present but no block product exists
    A1 = wl.BlockMatrix(8 * 32, 8 * 32, 32, np.array([0], np.int32), np.array([1], np.int32), np.ones((1, 32, 32)))
    B1 = wl.BlockMatrix(8 * 32, 8 * 32, 32, np.array([0], np.int32), np.array([0], np.int32), np.ones((1, 32, 32)))
    C, st, _ = gpu_multiply(qt, A1, B1, 256)
    assert C.nnz == 0
    # a single block
    one = random_pattern(rng, 1, 1, 1.0, 64)
    check_f64(qt, one, one, 64)


def test_chained_product_f64(qt):
    """C = A*A, then D = C*A, with C used as an operand (its own tree)."""
    rng = np.random.default_rng(6)
    A = random_pattern(rng, 40, 40, 0.05, 32)
    ref_C, _ = oracle.multiply(A, A, 128)
    ref_D, _ = oracle.multiply(ref_C, A, 128)
    absC, _ = oracle.multiply(A, A, 128, use_abs=True)
    absD, _ = oracle.multiply(absC, A, 128, use_abs=True)
    hA = qt.from_blockmatrix(A, 128)
    hC = qt.multiply(hA, hA)
    hD = qt.multiply(hC, hA)
    I, J, V = hD.to_blocks()
    D = wl.BlockMatrix(A.n_rows, A.n_cols, 32, I, J, V)
    same, _, e_f, e_cw = compare(ref_D, D, absD)
    assert same and e_cw <= TOL64


def test_back_to_back_chain_on_streams(qt):
    """C_1 = A*A, C_{k+1} = C_k*A, issued back to back with no host sync
    between the calls, on the default stream and on a torch stream: each
    traversal overlaps the previous numeric kernel (it reads only C_k's
    structure) while each numeric kernel waits for the previous values. The
    earlier results are freed while later ones are still being computed."""
    import torch
    rng = np.random.default_rng(16)
    A = random_pattern(rng, 48, 48, 0.06, 32)
    refs, absrefs = [], []
    ref, absref = A, A
    absA = wl.BlockMatrix(A.n_rows, A.n_cols, 32, A.I, A.J, np.abs(A.V))
    for _ in range(4):
        ref, _ = oracle.multiply(ref, A, 128)
        absref, _ = oracle.multiply(absref if len(refs) else absA, absA, 128)
        refs.append(ref)
        absrefs.append(absref)
    for stream in (None, torch.cuda.Stream()):
        hA = qt.from_blockmatrix(A, 128, stream=stream)
        chain = [hA]
        for _ in range(4):
            chain.append(qt.multiply(chain[-1], hA, stream=stream))
            if len(chain) >= 4:
                chain[-3].free()     # C_{k-1}: freed in stream order, after the multiply that read it
        I, J, V = chain[-1].to_blocks(stream=stream)
        got = wl.BlockMatrix(A.n_rows, A.n_cols, 32, I, J, V)
        same, _, _, e_cw = compare(refs[-1], got, absrefs[-1])
        assert same and e_cw <= 4 * TOL64, e_cw


def test_decay_small_f64(qt):
    A = wl.decay3d(1024, 25.0, 16, 32, seed=7)
    check_f64(qt, A, A, 256, same=True)


def test_random_small_f64(qt):
    A = wl.random_blocks(512, 512, int(0.02 * 512 * 512), 32, seed=8)
    check_f64(qt, A, A, 128, same=True)


def _bound_check(C, ref, absAB, rel):
    same, e_max, e_f, e_cw = compare(ref, C, absAB)
    assert same
    return e_cw, e_f


def test_f32_random(qt):
    for b in (16, 32, 64):
        rng = np.random.default_rng(20 + b)
        A = random_pattern(rng, 40, 40, 0.1, b)
        B = random_pattern(rng, 40, 40, 0.1, b)
        _say("f32 b", b)
        ref, _ = oracle.multiply(A, B, 4 * b)
        absAB, _ = oracle.multiply(A, B, 4 * b, use_abs=True)
        C, st, h = gpu_multiply(qt, A, B, 4 * b, "f32")
        assert h.info()["value_type"] == "f32"
        kmax = int(np.bincount(A.I, minlength=40).max())
        same, e_max, e_f, e_cw = compare(ref, C, absAB)
        assert same
        assert e_cw <= (kmax * b + 2) * 2.0 ** -24, e_cw
        assert e_f < 1e-6


def test_bf16x3_random(qt):
    for b in (32, 64):
        rng = np.random.default_rng(30 + b)
        A = random_pattern(rng, 30, 30, 0.15, b)
        B = random_pattern(rng, 30, 30, 0.15, b)
        _say("bf16x3 b", b)
        ref, _ = oracle.multiply(A, B, 2 * b)
        absAB, _ = oracle.multiply(A, B, 2 * b, use_abs=True)
        C, st, h = gpu_multiply(qt, A, B, 2 * b, "bf16x3")
        assert h.info()["value_type"] == "f64"
        same, e_max, e_f, e_cw = compare(ref, C, absAB)
        assert same
        assert e_cw <= 3 * 2.0 ** -16 + (3 * b + 4) * 2.0 ** -24, e_cw
        assert e_f < 2e-5
    with pytest.raises(qt.QtError) as e:
        X = qt.from_blockmatrix(random_pattern(np.random.default_rng(0), 4, 4, 0.5, 16), 32)
        qt.multiply(X, X, "bf16x3")
    assert e.value.status == qt.QT_ERR_UNSUPPORTED


def test_bf16x3_split_form_is_what_is_computed(qt):
    """The split path equals the fp64 product of the split operands up to fp32
    accumulation inside one block product: dropping a cross term or a wrong
    split would exceed this much tighter bound."""
    from oracle.precision import split_bf16, with_values
    for b in (32, 64):
        rng = np.random.default_rng(41 + b)
        A = random_pattern(rng, 24, 24, 0.2, b)
        hi, lo = split_bf16(A.V)
        Ah, Al = with_values(A, hi), with_values(A, lo)
        hh, _ = oracle.multiply(Ah, Ah, 4 * b)
        hl, _ = oracle.multiply(Ah, Al, 4 * b)
        lh, _ = oracle.multiply(Al, Ah, 4 * b)
        absAB, _ = oracle.multiply(A, A, 4 * b, use_abs=True)
        ref = wl.BlockMatrix(A.n_rows, A.n_cols, b, hh.I, hh.J, hh.V + hl.V + lh.V)
        C, _, _ = gpu_multiply(qt, A, A, 4 * b, "bf16x3", same=True)
        same, e_max, e_f, e_cw = compare(ref, C, absAB)
        assert same
        assert e_cw <= 1.05 * (3 * b + 4) * 2.0 ** -24, e_cw


@pytest.mark.parametrize("prec,b", [("f64", 32), ("f64", 16), ("bf16x3", 64)])
def test_launch_order_shapes(qt, prec, b):
    """Products with several block products per C block (the split kernel at
    b = 64 launches their C blocks in leaf-row strips; fp64 keeps Morton
    order): rectangular, ragged and transposed shapes against the oracle."""
    from tests._util import transpose
    rng = np.random.default_rng(700 + b)
    m, k, n = (23, 41, 17) if b == 64 else (45, 61, 37)
    for ta, tb, lb in ((False, False, 2), (True, False, 4), (False, True, 1), (True, True, 2)):
        A = random_pattern(rng, k if ta else m, m if ta else k, 0.45, b)
        B = random_pattern(rng, n if tb else k, k if tb else n, 0.45, b)
        opA = transpose(A) if ta else A
        opB = transpose(B) if tb else B
        _say("launch order", prec, "b", b, "trans", ta, tb, "leaf", lb * b)
        ref, ost = oracle.multiply(opA, opB, lb * b)
        absref, _ = oracle.multiply(opA, opB, lb * b, use_abs=True)
        hC = qt.multiply_ex(qt.from_blockmatrix(A, lb * b), qt.from_blockmatrix(B, lb * b), trans_a=ta,
                            trans_b=tb, prec=prec)
        st = hC.stats()
        assert st["products"] == ost.block_products
        assert st["products"] >= 2 * ref.nnz      # where the split kernel uses the strips
        I, J, V = hC.to_blocks("f64")
        C = wl.BlockMatrix(m * b, n * b, b, I, J, V)
        same, e_max, e_f, e_cw = compare(ref, C, absref)
        assert same
        if prec == "f64":
            assert e_cw <= TOL64 and e_f <= TOL64, (e_cw, e_f)
        else:
            assert e_cw <= 3 * 2.0 ** -16 + (3 * b + 4) * 2.0 ** -24, e_cw


@pytest.mark.parametrize("prec,b", [("f64", 32), ("f64", 16), ("f64", 64), ("f32", 32), ("bf16x3", 64)])
def test_inner_index_order_shapes(qt, prec, b):
    """Products with fewer than two block products per C block (the C blocks
    are then launched grouped by the inner index of their first product):
    rectangular, ragged and transposed shapes against the oracle."""
    from tests._util import transpose
    rng = np.random.default_rng(900 + b)
    m, k, n = (29, 47, 23) if b == 64 else (53, 71, 43)
    for ta, tb, lb in ((False, False, 2), (True, False, 4), (False, True, 1), (True, True, 2)):
        A = random_pattern(rng, k if ta else m, m if ta else k, 0.07, b)
        B = random_pattern(rng, n if tb else k, k if tb else n, 0.07, b)
        opA = transpose(A) if ta else A
        opB = transpose(B) if tb else B
        _say("inner-index order", prec, "b", b, "trans", ta, tb, "leaf", lb * b)
        ref, ost = oracle.multiply(opA, opB, lb * b)
        absref, _ = oracle.multiply(opA, opB, lb * b, use_abs=True)
        hC = qt.multiply_ex(qt.from_blockmatrix(A, lb * b), qt.from_blockmatrix(B, lb * b), trans_a=ta,
                            trans_b=tb, prec=prec)
        st = hC.stats()
        assert st["products"] == ost.block_products
        assert 0 < st["products"] < 2 * ref.nnz   # where the inner-index order is used
        I, J, V = hC.to_blocks("f64")
        C = wl.BlockMatrix(m * b, n * b, b, I, J, V)
        same, e_max, e_f, e_cw = compare(ref, C, absref)
        assert same
        if prec == "f64":
            assert e_cw <= TOL64 and e_f <= TOL64, (e_cw, e_f)
        elif prec == "f32":
            assert e_cw <= (k * b + 2) * 2.0 ** -24, e_cw
        else:
            assert e_cw <= 3 * 2.0 ** -16 + (3 * b + 4) * 2.0 ** -24, e_cw


@pytest.mark.parametrize("kdim", [16384, 16385])
def test_inner_index_order_widest(qt, kdim):
    """The inner-index order counts C blocks per k in an LDS table of up to
    16384 entries (64 KiB): an inner dimension of exactly that many blocks
    uses the full table, one more keeps Morton order. Both against the
    oracle."""
    rng = np.random.default_rng(77)
    A = random_pattern(rng, 40, kdim, 0.004, 16)
    B = random_pattern(rng, kdim, 36, 0.004, 16)
    _say("inner-index order, inner dimension", kdim)
    ref, ost = oracle.multiply(A, B, 64)
    absref, _ = oracle.multiply(A, B, 64, use_abs=True)
    assert 0 < ost.block_products < 2 * ref.nnz
    C, st, _ = gpu_multiply(qt, A, B, 64, "f64")
    assert st["products"] == ost.block_products
    same, e_max, e_f, e_cw = compare(ref, C, absref)
    assert same
    assert e_cw <= TOL64 and e_f <= TOL64, (e_cw, e_f)


def test_inner_index_order_repeatable(qt):
    """Inside one inner index the launch slots are claimed by atomics and vary
    from call to call; every C block is still computed by one wave in
    ascending k, so repeated multiplies give bitwise equal results."""
    rng = np.random.default_rng(913)
    A = random_pattern(rng, 80, 96, 0.05, 32)
    B = random_pattern(rng, 96, 72, 0.05, 32)
    ref, ost = oracle.multiply(A, B, 128)
    assert ost.block_products < 2 * ref.nnz
    hA, hB = qt.from_blockmatrix(A, 128), qt.from_blockmatrix(B, 128)
    for prec in ("f64", "f32", "bf16x3"):
        first = None
        for rep in range(3):
            _say("inner-index order repeat", prec, rep)
            hC = qt.multiply(hA, hB, prec)
            out = hC.to_blocks("f64")
            hC.free()
            if first is None:
                first = out
                pos = np.sort(out[0].astype(np.int64) * B.nb_cols + out[1])
                assert np.array_equal(pos, np.sort(ref.I.astype(np.int64) * B.nb_cols + ref.J))
            else:
                for x, y in zip(first, out):
                    assert np.array_equal(x, y), prec
