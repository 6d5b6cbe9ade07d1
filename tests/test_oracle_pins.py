"""Pins of the CPU oracle against facts that do not come from the oracle.

Each test ties the oracle to something the paper or plain mathematics fixes:
dense products computed by a library routine, the boolean product of the
patterns, hand-derived closed forms, exact invariants, and the task-count
formulas of Sec. 5 (Eq. 1-3 and the banded bound).
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads as wl
from tests._util import (norm_thresholded_by_definition, tau_in_gap, block_permutation, compare, identity, make, positions,
                         random_pattern, to_dense)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _dense_check(A, B, leaf, tol=1e-13):
    C, st = oracle.multiply(A, B, leaf)
    Ad, Bd = to_dense(A), to_dense(B)
    ref = Ad @ Bd
    bound = np.abs(Ad) @ np.abs(Bd)
    Cd = to_dense(C)
    err = np.abs(Cd - ref)
    assert np.all(err <= tol * bound + 0.0), float((err - tol * bound).max())
    # structural pattern: exactly the boolean product of the block patterns
    assert np.array_equal(positions(C), oracle.pattern_by_definition(A, B))
    assert st.block_products == oracle.product_count(A, B)
    return C, st


@pytest.mark.parametrize("b", [1, 2, 4, 8, 32])
@pytest.mark.parametrize("lb", [1, 2, 8])
def test_dense_special_case(b, lb):
    """Sec. 3 Alg. 1 + Sec. 4.1 leaf multiply == dense matmul on tiny inputs."""
    rng = np.random.default_rng(100 + 10 * b + lb)
    nbr, nbk, nbc = (13, 11, 9) if b < 32 else (5, 6, 7)
    for fill in (0.05, 0.3, 1.0):
        A = random_pattern(rng, nbr, nbk, fill, b)
        B = random_pattern(rng, nbk, nbc, fill, b)
        _dense_check(A, B, lb * b)


def test_dense_nonsymmetric_operands_catch_transposes():
    """A non-square, non-symmetric pair: a transposed operand or swapped child
    index in the recursion would change the product."""
    rng = np.random.default_rng(7)
    A = random_pattern(rng, 6, 17, 0.5, 3)
    B = random_pattern(rng, 17, 4, 0.5, 3)
    for lb in (1, 2, 4, 8, 16, 32):
        _dense_check(A, B, lb * 3)


@pytest.mark.parametrize("b", [1, 4, 32])
@pytest.mark.parametrize("lb", [1, 2, 8])
def test_abs_mode_is_abs_product(b, lb):
    """The |A||B| mode, the denominator of every componentwise parity bound,
    equals numpy's product of the entrywise absolute values (a library routine
    on the dense forms). All terms are non-negative, so the oracle's sum and
    numpy's differ only by rounding: within (k+1) u of the value. Operands with
    mixed signs make a dropped fabs on either side (or a signed sum) fail."""
    rng = np.random.default_rng(300 + 10 * b + lb)
    nbr, nbk, nbc = (11, 9, 7) if b < 32 else (4, 5, 3)
    for fill in (0.1, 0.5, 1.0):
        A = random_pattern(rng, nbr, nbk, fill, b)
        B = random_pattern(rng, nbk, nbc, fill, b)
        C, _ = oracle.multiply(A, B, lb * b, use_abs=True)
        ref = np.abs(to_dense(A)) @ np.abs(to_dense(B))
        Cd = to_dense(C)
        k = nbk * b
        assert np.all(np.abs(Cd - ref) <= (k + 1) * 2.0 ** -53 * ref)
        assert np.array_equal(positions(C), oracle.pattern_by_definition(A, B))
        # every present block of |A||B| is non-negative, and positive wherever
        # some product term is nonzero (no cancellation is possible)
        assert (C.V >= 0).all()


def test_boolean_product_pattern_larger():
    """Pattern(C) is the boolean product of the block patterns (bit-exact)."""
    rng = np.random.default_rng(11)
    A = random_pattern(rng, 300, 300, 0.02, 1)
    B = random_pattern(rng, 300, 300, 0.02, 1)
    for leaf in (1, 4, 16):
        C, st = oracle.multiply(A, B, leaf)
        assert np.array_equal(positions(C), oracle.pattern_by_definition(A, B))
        assert st.block_products == oracle.product_count(A, B)


def test_banded1024_closed_form():
    """Hand-derived counts for the 1024 banded workload (golden fixture)."""
    g = json.load(open(os.path.join(GOLDEN, "banded1024_counts.json")))
    A = wl.config("banded1024")
    assert A.nnz == g["nnz_A"]
    C, st = oracle.multiply(A, A, 256)
    assert st.block_products == g["block_products"]
    assert 2 * A.b ** 3 * st.block_products == g["flops"]
    assert C.nnz == g["nnz_C"]
    assert st.mul_tasks.tolist() == g["mul_tasks_per_level"]
    assert st.c_nodes.tolist() == g["c_nodes_per_level"]
    assert np.all(np.abs(C.I.astype(int) - C.J.astype(int)) <= 6)


def test_identity_exact():
    rng = np.random.default_rng(3)
    A = random_pattern(rng, 24, 24, 0.1, 8)
    E = identity(24, 8)
    for leaf in (8, 32, 64):
        C1, _ = oracle.multiply(A, E, leaf)
        C2, _ = oracle.multiply(E, A, leaf)
        for C in (C1, C2):
            assert np.array_equal(positions(C), positions(A))
            assert np.array_equal(C.V, A.V)          # exact: one product per block, times 1


def test_permutation_invariants():
    rng = np.random.default_rng(5)
    nb, b = 20, 4
    A = random_pattern(rng, nb, nb, 0.15, b)
    B = random_pattern(rng, nb, nb, 0.15, b)
    sigma = rng.permutation(nb)
    P = block_permutation(sigma, b)
    Pt = block_permutation(np.argsort(sigma), b)
    # P A moves block row j to sigma[j], exactly
    PA, _ = oracle.multiply(P, A, 4 * b)
    ref = make(A.n_rows, A.n_cols, b, sigma[A.I], A.J, A.V)
    assert np.array_equal(positions(PA), positions(ref)) and np.array_equal(PA.V, ref.V)
    # (P A P^T)(P B P^T) = P (A B) P^T: pattern exact, values to rounding
    PAPt, _ = oracle.multiply(PA, Pt, 4 * b)
    PB, _ = oracle.multiply(P, B, 4 * b)
    PBPt, _ = oracle.multiply(PB, Pt, 4 * b)
    lhs, _ = oracle.multiply(PAPt, PBPt, 8 * b)
    AB, _ = oracle.multiply(A, B, 2 * b)
    rhs = make(AB.n_rows, AB.n_cols, b, sigma[AB.I], sigma[AB.J], AB.V)
    absAB, _ = oracle.multiply(A, B, 2 * b, use_abs=True)
    absr = make(AB.n_rows, AB.n_cols, b, sigma[absAB.I], sigma[absAB.J], absAB.V)
    same, _, _, e_cw = compare(rhs, lhs, absr)
    assert same and e_cw <= 1e-13


def test_power_of_two_scaling_exact():
    rng = np.random.default_rng(8)
    A = random_pattern(rng, 16, 16, 0.2, 8)
    B = random_pattern(rng, 16, 16, 0.2, 8)
    C, _ = oracle.multiply(A, B, 32)
    As = make(A.n_rows, A.n_cols, 8, A.I, A.J, A.V * 2.0 ** 7)
    Cs, _ = oracle.multiply(As, B, 32)
    assert np.array_equal(Cs.V, C.V * 2.0 ** 7)


def test_nil_operand():
    rng = np.random.default_rng(9)
    A = random_pattern(rng, 8, 8, 0.3, 4)
    Z = random_pattern(rng, 8, 8, 0.0, 4)
    for X, Y in ((A, Z), (Z, A), (Z, Z)):
        C, st = oracle.multiply(X, Y, 16)
        assert C.nnz == 0 and st.block_products == 0 and st.mul_tasks.sum() == 0


def test_leaf_size_does_not_change_result():
    """Sec. 5: a larger leaf only merges the lowest levels."""
    rng = np.random.default_rng(12)
    A = random_pattern(rng, 64, 64, 0.05, 4)
    B = random_pattern(rng, 64, 64, 0.05, 4)
    ref, _ = oracle.multiply(A, B, 4)
    absAB, _ = oracle.multiply(A, B, 4, use_abs=True)
    for leaf in (8, 16, 32, 64, 256):
        C, _ = oracle.multiply(A, B, leaf)
        same, _, _, e_cw = compare(ref, C, absAB)
        assert same and e_cw <= 1e-13


def _eq1(N, delta, l):
    L = int(round(math.log2(N)))
    n_l = 4 ** (L - l)
    return 8.0 ** l * (1.0 - (1.0 - delta) ** n_l) ** 2


def test_random_task_counts_eq1_eq2_eq3():
    """Sec. 5.1: tasks per level for a random pattern, block size 1.

    Eq. 1 gives the expectation (checked within 2% where the count is large),
    Eq. 2 and Eq. 3 are hard upper bounds on the expectation; the realised
    count must also respect the total bound (3 1/7)(delta N^2)^(3/2) of the
    summed Eq. 2/3 argument, up to sampling noise of the expectation.
    """
    N, delta = 512, 0.04
    rng = np.random.default_rng(21)
    A = random_pattern(rng, N, N, delta, 1)
    B = random_pattern(rng, N, N, delta, 1)
    _, st = oracle.multiply(A, B, 1)
    L = int(math.log2(N))
    assert len(st.mul_tasks) == L + 1
    for l in range(L + 1):
        exp = _eq1(N, delta, l)
        got = st.mul_tasks[l]
        assert got <= 8 ** l                                  # Eq. 2 (hard: at most N_l^3 pairs)
        if exp >= 1e4:
            assert abs(got - exp) <= 0.02 * exp, (l, got, exp)
        # Eq. 3 bounds the expectation; allow 3 sigma-ish sampling slack
        assert exp <= 16.0 ** L * delta ** 2 / 2 ** l * (1 + 1e-12)
        assert got <= 16.0 ** L * delta ** 2 / 2 ** l * 1.02 + 3 * math.sqrt(exp + 1)
    assert st.mul_tasks.sum() < (3 + 1 / 7) * (delta * N * N) ** 1.5
    assert st.block_products == st.mul_tasks[L]


def test_banded_task_bound():
    """Sec. 5.1: banded, bandwidth 2d+1 with d = 2^k, block size 1:
    C_l < 2^l (2 d_l + 1)^2 per level and the total bound on the sum."""
    N, k = 1024, 2
    d = 2 ** k
    L = int(math.log2(N))
    A = wl.banded(N, d, 1, seed=0)
    _, st = oracle.multiply(A, A, 1)
    for l in range(L + 1):
        d_l = 1 if l < L - k else 2 ** (l - (L - k))
        assert st.mul_tasks[l] < 2 ** l * (2 * d_l + 1) ** 2, (l, st.mul_tasks[l])
    assert st.mul_tasks.sum() < (4 + 4 / 7) * d * d * N + (5 + 1 / 3) * d * N + 2 * N + 9 * N / d


def test_additions_fewer_than_multiplications():
    """Sec. 5: add tasks are strictly fewer than multiply tasks."""
    rng = np.random.default_rng(31)
    for fill in (0.01, 0.1, 0.5):
        A = random_pattern(rng, 64, 64, fill, 2)
        for leaf in (2, 8, 32):
            C, st = oracle.multiply(A, A, leaf)
            if st.mul_tasks.sum() == 0:
                continue
            assert st.add_tasks.sum() < st.mul_tasks.sum()
            # every block addition merges two partial results
            assert st.leaf_block_adds <= st.block_products - C.nnz


def test_overlap_levels_grow():
    """Sec. 5.1, overlap pattern: tasks at least double from level to level
    on a decay matrix (checked on the levels below the root region)."""
    A = wl.decay3d(512, 20.0, 16, 16, seed=40)
    _, st = oracle.multiply(A, A, 16)
    m = st.mul_tasks
    assert all(m[l] >= 2 * m[l - 1] for l in range(1, len(m)))


def test_block_by_definition_agrees():
    A = wl.decay3d(256, 16.0, 16, 32, seed=41)
    C, _ = oracle.multiply(A, A, 128)
    idx = oracle.make_index(A, A)
    rng = np.random.default_rng(0)
    for t in rng.choice(C.nnz, size=min(40, C.nnz), replace=False):
        ref = oracle.block_by_definition(A, A, C.I[t], C.J[t], idx)
        assert np.allclose(ref, C.V[t], rtol=0, atol=1e-12 * (np.abs(ref).max() + 1))


def test_errors():
    rng = np.random.default_rng(1)
    A = random_pattern(rng, 4, 4, 0.5, 2)
    bad = make(8, 8, 2, [0, 5], [0, 0], np.ones((2, 2, 2)))
    with pytest.raises(oracle.OracleError) as e:
        oracle.multiply(bad, A, 4)                   # block row 5 outside a 4-row grid
    assert e.value.code == 1
    dup = make(8, 8, 2, [1, 1], [2, 2], np.ones((2, 2, 2)))
    with pytest.raises(oracle.OracleError) as e:
        oracle.multiply(dup, A, 4)
    assert e.value.code == 3
    B = random_pattern(rng, 3, 4, 0.5, 2)
    with pytest.raises(oracle.OracleError) as e:
        oracle.multiply(A, B, 4)                     # inner dimensions differ
    assert e.value.code == 2
    with pytest.raises(oracle.OracleError) as e:
        oracle.multiply(A, A, 6)                     # leaf/b = 3 is not a power of 2
    assert e.value.code == 2


def test_bf16_rounding_definition():
    """Round-to-nearest-even to bfloat16 from the IEEE definition."""
    from oracle.precision import bf16_rne, split_bf16
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, 1.0 + 2 ** -9, 1.0 + 3 * 2 ** -8,
                  -2.5, 0.0, 1e-40], np.float32)
    r = bf16_rne(x)
    assert r[0] == 1.0
    assert r[1] == 1.0 + 2 ** -7 or r[1] == 1.0           # tie: 1+2^-8 is halfway, even -> 1.0
    assert r[1] == 1.0
    assert r[2] == 1.0 + 2 ** -7                         # above halfway rounds up
    assert r[3] == 1.0                                    # below halfway rounds down
    assert r[4] == 1.0 + 2 ** -6                          # tie at odd -> up to even
    assert r[5] == -2.5 and r[6] == 0.0
    v = np.random.default_rng(0).standard_normal(10000)
    hi, lo = split_bf16(v)
    a32 = v.astype(np.float32)
    assert np.all(np.abs((hi.astype(np.float64) + lo) - a32) <= np.abs(a32) * 2.0 ** -16)


def test_add_algorithm2_dense_and_union():
    """Sec. 3, Algorithm 2: the sum's pattern is the union of the patterns and
    its values the dense sum (exact: one addition per entry at most)."""
    rng = np.random.default_rng(51)
    for b, lb in ((1, 1), (2, 4), (8, 2), (4, 8)):
        A = random_pattern(rng, 21, 17, 0.3, b)
        B = random_pattern(rng, 21, 17, 0.3, b)
        C, st = oracle.add(A, B, lb * b)
        assert np.array_equal(to_dense(C), to_dense(A) + to_dense(B))
        assert np.array_equal(positions(C), np.union1d(positions(A), positions(B)))
        # one leaf block addition per position present in both
        assert st.leaf_block_adds == np.intersect1d(positions(A), positions(B)).size
    Z = random_pattern(rng, 21, 17, 0.0, 2)
    A = random_pattern(rng, 21, 17, 0.3, 2)
    C, _ = oracle.add(A, Z, 8)
    assert np.array_equal(C.V, A.V) and np.array_equal(positions(C), positions(A))


def test_rmat_locality_moves_tasks_down():
    """Sec. 5.1, R-MAT matrices: a = 0.25 is the random case (Eq. 1 within a
    few percent at the populated levels), and raising a pushes the multiply
    tasks towards the lowest levels (the share of leaf-level tasks grows)."""
    scale = 10
    shares = []
    for a in (0.25, 0.5, 0.75, 0.9):
        A = wl.rmat(scale, 5, a, 1, seed=60)
        _, st = oracle.multiply(A, A, 1)
        m = st.mul_tasks.astype(float)
        shares.append(m[-1] / m.sum())
        if a == 0.25:
            N = 1 << scale
            delta = A.nnz / float(N * N)
            for l in range(scale + 1):
                e = _eq1(N, delta, l)
                if e >= 2e4:
                    assert abs(m[l] - e) <= 0.05 * e, (l, m[l], e)
    assert all(shares[i] < shares[i + 1] for i in range(len(shares) - 1)), shares


def test_truncation_definition():
    """Truncation of Sec. 6.2: ||M - T||_F < eps, the removed blocks are the
    smallest ones, and removing the next block would reach eps."""
    rng = np.random.default_rng(70)
    M = random_pattern(rng, 30, 30, 0.3, 4)
    M.V *= rng.uniform(1e-6, 1.0, size=(M.nnz, 1, 1))
    norms = np.sqrt((M.V.reshape(M.nnz, -1) ** 2).sum(1))
    for eps in (0.0, 1e-5, 1e-3, 0.5, 3.0, 1e9):
        T, k = oracle.truncate(M, eps)
        E = to_dense(M) - to_dense(T)
        assert np.linalg.norm(E) < eps or (k == 0 and eps == 0.0)
        kept = set(zip(T.I.tolist(), T.J.tolist()))
        removed = [t for t in range(M.nnz) if (int(M.I[t]), int(M.J[t])) not in kept]
        assert len(removed) == k
        if k and T.nnz:
            assert norms[removed].max() <= np.sort(norms[[t for t in range(M.nnz) if t not in removed]])[0]
        if T.nnz:
            nxt = np.sort(norms[[t for t in range(M.nnz) if t not in removed]])[0]
            assert np.sqrt(np.sum(norms[removed] ** 2) + nxt ** 2) >= eps
        assert np.array_equal(to_dense(T)[to_dense(T) != 0], to_dense(M)[to_dense(T) != 0])


def test_truncation_ties_follow_z_order():
    """Equal block norms are removed in quadtree (Z) order: on a 2 x 2 block
    grid of unit-norm blocks, eps^2 = 2.5 removes exactly two blocks, the
    top-left and then the top-right one (children 0 and 1 of the root)."""
    b = 2
    I = np.array([1, 1, 0, 0], np.int32)
    J = np.array([1, 0, 1, 0], np.int32)
    V = np.zeros((4, b, b))
    V[:, 0, 0] = 1.0                                   # every block has norm 1
    M = wl.BlockMatrix(2 * b, 2 * b, b, I, J, V)
    T, k = oracle.truncate(M, float(np.sqrt(2.5)))
    assert k == 2
    assert sorted(zip(T.I.tolist(), T.J.tolist())) == [(1, 0), (1, 1)]
    T, k = oracle.truncate(M, float(np.sqrt(3.5)))
    assert k == 3 and list(zip(T.I.tolist(), T.J.tolist())) == [(1, 1)]


# ------------------------------------------------- norm-thresholded product

def _graded(rng, nbr, nbc, fill, b):
    """Random pattern whose blocks are scaled over six decades, so that their
    norm products spread over twelve."""
    M = random_pattern(rng, nbr, nbc, fill, b)
    scale = 10.0 ** rng.uniform(-6, 0, size=M.nnz)
    return wl.BlockMatrix(M.n_rows, M.n_cols, b, M.I, M.J, M.V * scale[:, None, None])


@pytest.mark.parametrize("b,lb,q", [(4, 2, 0.3), (2, 4, 0.6), (3, 1, 0.5), (4, 8, 0.8)])
def test_norm_threshold_matches_definition(b, lb, q):
    """The oracle's norm-thresholded product (tasks dropped at every level by
    their node norms, block products by their block norms) equals the
    definition by block norms alone, and keeps exactly its products
    (Sec. 7: Frobenius norms per submatrix in the quadtree)."""
    rng = np.random.default_rng(31 + lb)
    A = _graded(rng, 20, 24, 0.3, b)
    B = _graded(rng, 24, 18, 0.3, b)
    tau = tau_in_gap(A, B, q)
    ref, kept, dropped, _ = norm_thresholded_by_definition(A, B, tau)
    C, st = oracle.multiply(A, B, lb * b, tau=tau)
    assert np.array_equal(positions(C), positions(ref))
    absAB, _ = oracle.multiply(A, B, lb * b, use_abs=True, tau=tau)
    assert np.all(np.abs(C.V - ref.V) <= 1e-13 * absAB.V + 1e-300)
    assert st.block_products == kept and kept + dropped == oracle.product_count(A, B)
    assert 0 < kept and 0 < dropped
    # the dropped block products are all that is missing, within their norm sum
    Cx, _ = oracle.multiply(A, B, lb * b)
    err = np.linalg.norm(to_dense(Cx) - to_dense(C))
    _, _, _, bound = norm_thresholded_by_definition(A, B, tau)
    assert err <= bound * (1 + 1e-12)


def test_norm_threshold_zero_is_exact_and_prunes_tasks():
    rng = np.random.default_rng(37)
    A = _graded(rng, 32, 32, 0.2, 4)
    C0, st0 = oracle.multiply(A, A, 16)
    Ct, stt = oracle.multiply(A, A, 16, tau=0.0)
    assert np.array_equal(positions(C0), positions(Ct)) and np.array_equal(C0.V, Ct.V)
    assert stt.pruned_products == 0 and not stt.pruned_tasks.any()
    # a threshold above every norm product leaves C empty, dropping the root task
    big = float(np.linalg.norm(A.V)) ** 2 * 2
    Cb, stb = oracle.multiply(A, A, 16, tau=big)
    assert Cb.nnz == 0 and stb.pruned_tasks[0] == 1 and stb.block_products == 0
    # tasks are dropped above the leaves too: with the lower-right quadrant of
    # A scaled down, its products with itself fall below tau as a whole
    low = (A.I >= 16) & (A.J >= 16)
    As = wl.BlockMatrix(A.n_rows, A.n_cols, 4, A.I, A.J, A.V * np.where(low, 1e-9, 1.0)[:, None, None])
    tau = tau_in_gap(As, As, 0.3)
    C, st = oracle.multiply(As, As, 16, tau=tau)
    assert st.pruned_tasks[1] >= 1
    ref, kept, _, _ = norm_thresholded_by_definition(As, As, tau)
    assert np.array_equal(positions(C), positions(ref)) and st.block_products == kept
    with pytest.raises(oracle.OracleError):
        oracle.multiply(A, A, 16, tau=-1.0)
