"""CPU oracle for the quadtree block-sparse multiply C = A*B.

TEST INFRASTRUCTURE. Only ``tests/``, the smoke check in ``__graft_entry__``
and the CPU-baseline leg of ``bench.py`` import this package. The GPU library
never imports, links or calls it, and the two share no code.

``multiply`` runs the plain C implementation in ``qt_oracle.c``: the
quadtree multiply of Rubensson & Rudberg, Sec. 3 (Algorithms 1 and 2), with
block-sparse leaves multiplied by plain triple loops (Sec. 4.1, Fig. 2), in
fp64. ``block_by_definition`` computes one block of C straight from the
definition C(I,J) = sum_K A(I,K) B(K,J), for sampled checks at sizes the full
oracle would take too long on.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

from workloads import BlockMatrix

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qt_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ERRORS = {0: "ok", 1: "invalid argument", 2: "shape", 3: "duplicate block", 4: "out of memory"}


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle error {code}: {ERRORS.get(code, '?')}")
        self.code = code


def build(src: str = _SRC, out: str = _LIB) -> str:
    """Compile the oracle with gcc (no FMA contraction, OpenMP tasks)."""
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared",
           "-fPIC", "-std=c99", "-Wall", "-Wno-unknown-pragmas", "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


_lib_handle = None


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib_handle = load(_LIB)
    return _lib_handle


def load(path: str):
    """Load a compiled oracle library and declare its entry points."""
    lib = ctypes.CDLL(path)
    i64, i32p, f64p = ctypes.c_int64, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)
    lib.qo_multiply.restype = ctypes.c_int
    lib.qo_multiply.argtypes = [i64, i64, i64, i32p, i32p, f64p,
                                i64, i64, i64, i32p, i32p, f64p,
                                ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                ctypes.POINTER(ctypes.c_void_p)]
    lib.qo_result_nnz.restype = i64
    lib.qo_result_nnz.argtypes = [ctypes.c_void_p]
    lib.qo_result_levels.restype = ctypes.c_int
    lib.qo_result_levels.argtypes = [ctypes.c_void_p]
    lib.qo_result_copy.restype = None
    lib.qo_result_copy.argtypes = [ctypes.c_void_p, i32p, i32p, f64p]
    lib.qo_result_stats.restype = None
    lib.qo_result_stats.argtypes = [ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_int64)] * 4
    lib.qo_result_pruned.restype = None
    lib.qo_result_pruned.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
    lib.qo_result_free.restype = None
    lib.qo_result_free.argtypes = [ctypes.c_void_p]
    lib.qo_add.restype = ctypes.c_int
    lib.qo_add.argtypes = [i64, i64, i64, i32p, i32p, f64p, i64, i32p, i32p, f64p, ctypes.c_int, ctypes.c_int,
                           ctypes.POINTER(ctypes.c_void_p)]
    lib.qo_threads.restype = ctypes.c_int
    lib.qo_threads.argtypes = [ctypes.c_int]
    return lib


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


@dataclass
class OracleStats:
    """Counters of one oracle multiply (levels 0 = root .. L = leaf level)."""
    mul_tasks: np.ndarray      # multiply tasks with both operands present, per level
    add_tasks: np.ndarray      # add tasks with both operands present, per level
    c_nodes: np.ndarray        # non-NIL nodes of C per level
    block_products: int        # leaf block products A(i,k) B(k,j)
    leaf_block_adds: int       # block additions inside leaf adds
    pruned_tasks: np.ndarray = None    # multiply tasks dropped by the norm threshold, per level
    pruned_products: int = 0           # block products dropped by it


def multiply(A: BlockMatrix, B: BlockMatrix, leaf: int, use_abs: bool = False,
             par_levels: int = 3, threads: int | None = None, lib=None, tau: float = 0.0):
    """C = A*B (or |A|*|B|) by the quadtree algorithm; returns (C, stats).

    C lists its blocks in row-major (I, J) order. ``threads`` caps the OpenMP
    thread count for this call (None: the OpenMP default). ``lib`` selects
    another compiled copy of the oracle (see ``load``). ``tau`` > 0 drops every
    multiply task and block product whose operands' Frobenius norms multiply
    to less than tau (the norm-thresholded product; tau = 0 is exact).
    """
    lib = _lib() if lib is None else lib
    if A.b != B.b:
        raise OracleError(2)
    b = A.b
    Ia, Ja = np.ascontiguousarray(A.I, np.int32), np.ascontiguousarray(A.J, np.int32)
    Ib, Jb = np.ascontiguousarray(B.I, np.int32), np.ascontiguousarray(B.J, np.int32)
    Va = np.ascontiguousarray(A.V, np.float64)
    Vb = np.ascontiguousarray(B.V, np.float64)
    out = ctypes.c_void_p()
    if threads is not None:
        lib.qo_threads(int(threads))
    rc = lib.qo_multiply(A.n_rows, A.n_cols, A.nnz, _ptr(Ia, ctypes.c_int32), _ptr(Ja, ctypes.c_int32),
                         _ptr(Va, ctypes.c_double),
                         B.n_rows, B.n_cols, B.nnz, _ptr(Ib, ctypes.c_int32), _ptr(Jb, ctypes.c_int32),
                         _ptr(Vb, ctypes.c_double),
                         b, leaf, 1 if use_abs else 0, float(tau), par_levels if threads != 1 else 0,
                         ctypes.byref(out))
    if rc != 0:
        raise OracleError(rc)
    try:
        nnz = lib.qo_result_nnz(out)
        nl = lib.qo_result_levels(out)
        I = np.empty(nnz, np.int32)
        J = np.empty(nnz, np.int32)
        V = np.empty((nnz, b, b), np.float64)
        lib.qo_result_copy(out, _ptr(I, ctypes.c_int32), _ptr(J, ctypes.c_int32), _ptr(V, ctypes.c_double))
        mul = np.zeros(nl, np.int64)
        add = np.zeros(nl, np.int64)
        nodes = np.zeros(nl, np.int64)
        st = np.zeros(2, np.int64)
        lib.qo_result_stats(out, *[_ptr(x, ctypes.c_int64) for x in (mul, add, nodes, st)])
        ptasks = np.zeros(nl, np.int64)
        pprods = np.zeros(1, np.int64)
        lib.qo_result_pruned(out, _ptr(ptasks, ctypes.c_int64), _ptr(pprods, ctypes.c_int64))
    finally:
        lib.qo_result_free(out)
    C = BlockMatrix(A.n_rows, B.n_cols, b, I, J, V, {"from": "oracle", "leaf": leaf})
    stats = OracleStats(mul, add, nodes, int(st[0]), int(st[1]), ptasks, int(pprods[0]))
    return C, stats


def _take(lib, out, rows, cols, b, meta):
    try:
        nnz = lib.qo_result_nnz(out)
        nl = lib.qo_result_levels(out)
        I = np.empty(nnz, np.int32)
        J = np.empty(nnz, np.int32)
        V = np.empty((nnz, b, b), np.float64)
        lib.qo_result_copy(out, _ptr(I, ctypes.c_int32), _ptr(J, ctypes.c_int32), _ptr(V, ctypes.c_double))
        mul = np.zeros(nl, np.int64)
        add = np.zeros(nl, np.int64)
        nodes = np.zeros(nl, np.int64)
        st = np.zeros(2, np.int64)
        lib.qo_result_stats(out, *[_ptr(x, ctypes.c_int64) for x in (mul, add, nodes, st)])
    finally:
        lib.qo_result_free(out)
    return BlockMatrix(rows, cols, b, I, J, V, meta), OracleStats(mul, add, nodes, int(st[0]), int(st[1]))


def add(A: BlockMatrix, B: BlockMatrix, leaf: int, lib=None):
    """C = A + B by Algorithm 2 (structural union; both-present blocks summed)."""
    lib = _lib() if lib is None else lib
    if A.b != B.b or A.n_rows != B.n_rows or A.n_cols != B.n_cols:
        raise OracleError(2)
    b = A.b
    arrs = [np.ascontiguousarray(x, t) for x, t in ((A.I, np.int32), (A.J, np.int32), (A.V, np.float64),
                                                     (B.I, np.int32), (B.J, np.int32), (B.V, np.float64))]
    out = ctypes.c_void_p()
    rc = lib.qo_add(A.n_rows, A.n_cols, A.nnz, _ptr(arrs[0], ctypes.c_int32), _ptr(arrs[1], ctypes.c_int32),
                    _ptr(arrs[2], ctypes.c_double), B.nnz, _ptr(arrs[3], ctypes.c_int32),
                    _ptr(arrs[4], ctypes.c_int32), _ptr(arrs[5], ctypes.c_double), b, leaf, ctypes.byref(out))
    if rc != 0:
        raise OracleError(rc)
    return _take(lib, out, A.n_rows, A.n_cols, b, {"from": "oracle add", "leaf": leaf})


def _morton(I, J):
    """Bit-interleaved position of block (I, J): column bits at even, row bits
    at odd positions (the Z order of the quadtree's children 2m + n)."""
    key = np.zeros(len(I), np.uint64)
    I = np.asarray(I, np.uint64)
    J = np.asarray(J, np.uint64)
    for bit in range(32):
        one = np.uint64(1)
        key |= ((J >> np.uint64(bit)) & one) << np.uint64(2 * bit)
        key |= ((I >> np.uint64(bit)) & one) << np.uint64(2 * bit + 1)
    return key


def truncate(M: BlockMatrix, eps: float):
    """Drop blocks in order of increasing Frobenius norm (equal norms: quadtree
    Z order first) while the norm of all removed blocks stays below eps
    (||M - T||_F < eps). Returns (T, removed)."""
    n2 = (M.V.reshape(M.nnz, -1) ** 2).sum(axis=1)
    order = np.lexsort((_morton(M.I, M.J), n2))
    run = np.cumsum(n2[order])
    k = int(np.count_nonzero(run < eps * eps))
    keep = np.ones(M.nnz, bool)
    keep[order[:k]] = False
    return BlockMatrix(M.n_rows, M.n_cols, M.b, M.I[keep], M.J[keep], M.V[keep], dict(M.meta)), k


def threads() -> int:
    """OpenMP threads the oracle's multiply uses."""
    return int(_lib().qo_threads(0))


def block_by_definition(A: BlockMatrix, B: BlockMatrix, I: int, J: int, index=None):
    """C(I,J) = sum over K ascending of A(I,K) B(K,J), straight from the definition.

    Returns None when no K has both A(I,K) and B(K,J) present (a NIL block).
    ``index`` may carry (rowsA, colsB) dictionaries from ``make_index`` to
    avoid rebuilding them for every sampled block.
    """
    rowsA, colsB = index if index is not None else make_index(A, B)
    ra = rowsA.get(int(I), {})
    cb = colsB.get(int(J), {})
    ks = sorted(set(ra) & set(cb))
    if not ks:
        return None
    acc = np.zeros((A.b, A.b), np.float64)
    for k in ks:
        acc += A.V[ra[k]] @ B.V[cb[k]]
    return acc


def make_index(A: BlockMatrix, B: BlockMatrix):
    """Block lookup tables: A's blocks by row (K -> position) and B's by column."""
    rowsA: dict = {}
    for t, (i, k) in enumerate(zip(A.I.tolist(), A.J.tolist())):
        rowsA.setdefault(i, {})[k] = t
    colsB: dict = {}
    for t, (k, j) in enumerate(zip(B.I.tolist(), B.J.tolist())):
        colsB.setdefault(j, {})[k] = t
    return rowsA, colsB


def pattern_by_definition(A: BlockMatrix, B: BlockMatrix) -> np.ndarray:
    """Block pattern of A*B as sorted row-major positions I*nb_cols(B) + J.

    (I, J) is present iff some K has A(I,K) and B(K,J) present: the boolean
    product of the two block patterns, by sparse matrix product of 0/1
    indicators (counts are exact small integers).
    """
    import scipy.sparse as sp
    a = sp.csr_matrix((np.ones(A.nnz), (A.I, A.J)), shape=(A.nb_rows, A.nb_cols))
    b = sp.csr_matrix((np.ones(B.nnz), (B.I, B.J)), shape=(B.nb_rows, B.nb_cols))
    c = (a @ b).tocoo()
    pos = c.row.astype(np.int64) * B.nb_cols + c.col.astype(np.int64)
    pos.sort()
    return pos


def product_count(A: BlockMatrix, B: BlockMatrix) -> int:
    """Number of block products: sum over K of (#A blocks in column K)(#B blocks in row K)."""
    ca = np.bincount(A.J, minlength=A.nb_cols).astype(np.int64)
    rb = np.bincount(B.I, minlength=B.nb_rows).astype(np.int64)
    return int((ca * rb).sum())
