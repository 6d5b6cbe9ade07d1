"""Helpers shared by the tests (layout only: no multiply arithmetic)."""
from __future__ import annotations

import numpy as np

from workloads import BlockMatrix


def to_dense(M: BlockMatrix) -> np.ndarray:
    D = np.zeros((M.n_rows, M.n_cols), dtype=np.float64)
    b = M.b
    for t in range(M.nnz):
        i, j = int(M.I[t]), int(M.J[t])
        D[i * b:(i + 1) * b, j * b:(j + 1) * b] = M.V[t]
    return D


def positions(M: BlockMatrix) -> np.ndarray:
    """Row-major block positions I * nb_cols + J (int64)."""
    return M.I.astype(np.int64) * M.nb_cols + M.J.astype(np.int64)


def make(n_rows, n_cols, b, I, J, V) -> BlockMatrix:
    I = np.asarray(I, np.int32)
    J = np.asarray(J, np.int32)
    order = np.lexsort((J, I))
    V = np.asarray(V, np.float64).reshape(len(I), b, b)
    return BlockMatrix(n_rows, n_cols, b, I[order], J[order], np.ascontiguousarray(V[order]))


def identity(nb: int, b: int) -> BlockMatrix:
    I = np.arange(nb, dtype=np.int32)
    V = np.broadcast_to(np.eye(b), (nb, b, b)).copy()
    return BlockMatrix(nb * b, nb * b, b, I, I.copy(), V)


def block_permutation(sigma: np.ndarray, b: int) -> BlockMatrix:
    """P with identity blocks at (sigma[j], j): (P A) moves block row j to sigma[j]."""
    nb = len(sigma)
    I = np.asarray(sigma, np.int32)
    J = np.arange(nb, dtype=np.int32)
    V = np.broadcast_to(np.eye(b), (nb, b, b)).copy()
    return make(nb * b, nb * b, b, I, J, V)


def random_pattern(rng, nbr, nbc, fill, b, rect_ok=True) -> BlockMatrix:
    total = nbr * nbc
    cnt = int(round(fill * total))
    pos = np.sort(rng.choice(total, size=cnt, replace=False)) if cnt else np.zeros(0, np.int64)
    I = (pos // nbc).astype(np.int32)
    J = (pos % nbc).astype(np.int32)
    V = rng.standard_normal((cnt, b, b))
    return BlockMatrix(nbr * b, nbc * b, b, I, J, V)


def compare(C_ref: BlockMatrix, C: BlockMatrix, absAB: BlockMatrix | None = None):
    """Pattern equality (bool) and componentwise / normwise errors of C vs C_ref.

    Componentwise error is |C - C_ref| / (|A||B|) (0/0 := 0); normwise is
    ||C - C_ref||_F / ||C_ref||_F.
    """
    same = (C_ref.nnz == C.nnz and np.array_equal(positions(C_ref), positions(C)))
    if not same:
        return False, np.inf, np.inf, np.inf
    d = C.V - C_ref.V
    e_max = float(np.abs(d).max()) if d.size else 0.0
    nrm = float(np.linalg.norm(C_ref.V))
    e_f = float(np.linalg.norm(d)) / nrm if nrm > 0 else float(np.linalg.norm(d))
    e_cw = 0.0
    if absAB is not None and d.size:
        den = absAB.V
        num = np.abs(d)
        with np.errstate(divide="ignore", invalid="ignore"):
            r = np.where(den > 0, num / np.where(den > 0, den, 1.0), np.where(num > 0, np.inf, 0.0))
        e_cw = float(r.max())
    return True, e_max, e_f, e_cw


def transpose(M: BlockMatrix) -> BlockMatrix:
    """M^T by definition: block (I, J) -> (J, I), each block transposed."""
    return make(M.n_cols, M.n_rows, M.b, M.J, M.I, np.ascontiguousarray(M.V.transpose(0, 2, 1)))


def upper_blocks(M: BlockMatrix) -> BlockMatrix:
    """The blocks of M with I <= J."""
    k = M.I <= M.J
    return BlockMatrix(M.n_rows, M.n_cols, M.b, M.I[k], M.J[k], np.ascontiguousarray(M.V[k]))


def symmetric_from_upper(U: BlockMatrix) -> BlockMatrix:
    """S with S(I,J) = U(I,J) for I <= J and S(J,I) = U(I,J)^T for I < J."""
    k = U.I < U.J
    I = np.concatenate([U.I, U.J[k]])
    J = np.concatenate([U.J, U.I[k]])
    V = np.concatenate([U.V, U.V[k].transpose(0, 2, 1)])
    return make(U.n_rows, U.n_cols, U.b, I, J, V)


def norm_thresholded_by_definition(A, B, tau):
    """C(I,J) = sum over K with ||A(I,K)||_F ||B(K,J)||_F >= tau of A(I,K) B(K,J),
    straight from the definition (numpy block norms, a loop over all block
    pairs): returns (C as BlockMatrix, kept products, dropped products, sum
    of ||A(I,K)|| ||B(K,J)|| over the dropped ones)."""
    na = np.linalg.norm(A.V.reshape(A.nnz, -1), axis=1)
    nb = np.linalg.norm(B.V.reshape(B.nnz, -1), axis=1)
    rows = {}
    for t, (i, k) in enumerate(zip(A.I.tolist(), A.J.tolist())):
        rows.setdefault(k, []).append((i, t))
    acc = {}
    kept = dropped = 0
    dropped_norm = 0.0
    for u, (k, j) in enumerate(zip(B.I.tolist(), B.J.tolist())):
        for i, t in rows.get(k, []):
            if na[t] * nb[u] >= tau:
                kept += 1
                key = (i, j)
                acc[key] = acc.get(key, 0.0) + A.V[t] @ B.V[u]
            else:
                dropped += 1
                dropped_norm += na[t] * nb[u]
    keys = sorted(acc)
    I = np.array([k[0] for k in keys], np.int32)
    J = np.array([k[1] for k in keys], np.int32)
    V = np.array([acc[k] for k in keys]).reshape(len(keys), A.b, B.b) if keys else np.zeros((0, A.b, A.b))
    return BlockMatrix(A.n_rows, B.n_cols, A.b, I, J, V), kept, dropped, dropped_norm


def tau_in_gap(A, B, quantile, rel_gap=1e-6):
    """A threshold near the given quantile of the block products' norm
    products, placed in the middle of a gap between two of them that is at
    least rel_gap wide (relative), so that no product's norm lies within
    rounding of it whatever the order its norms were summed in."""
    na = np.linalg.norm(A.V.reshape(A.nnz, -1), axis=1)
    nb = np.linalg.norm(B.V.reshape(B.nnz, -1), axis=1)
    cols = {}
    for t, k in enumerate(A.J.tolist()):
        cols.setdefault(k, []).append(na[t])
    prods = []
    for u, k in enumerate(B.I.tolist()):
        prods.extend(x * nb[u] for x in cols.get(k, []))
    prods = np.sort(np.array(prods))
    start = int(quantile * (len(prods) - 1))
    for m in range(start, len(prods) - 1):
        lo, hi = prods[m], prods[m + 1]
        if hi > lo * (1 + rel_gap):
            return float(np.sqrt(lo * hi))
    raise ValueError("no gap")
