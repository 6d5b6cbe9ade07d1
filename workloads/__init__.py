"""Seeded synthetic inputs for the quadtree block-sparse multiply.

This module only draws matrices. It holds none of the multiply's arithmetic,
and both the CPU oracle (through the tests) and the GPU library (through the
tests, the smoke check and the benchmark) take their inputs from here.

A block-sparse matrix is held as a ``BlockMatrix``: the block grid position
(I, J) of every nonzero b x b block, and its values, row-major inside the
block. Blocks are listed in row-major (I, then J) order.

Patterns (Rubensson & Rudberg, Sec. 5.1 and Sec. 6):

* ``banded``: every block with |I - J| <= w (the banded case of Sec. 5.1).
* ``random_blocks``: an exact number of distinct block positions drawn
  uniformly without replacement (the random case of Sec. 5.1 and the
  uniformly random leaf benchmark of Sec. 6.1).
* ``decay3d``: an overlap-like matrix of atoms in a cube, ordered by a
  recursive divide-space bisection (Sec. 5.1, overlap pattern; Sec. 6.2).
  The paper builds its overlap matrices with an electronic structure code
  from water clusters, which are not available here; this generator stands
  in for them with the same kind of distance-decay sparsity.
* ``rmat``: R-MAT graph patterns with a tunable degree of locality (Sec. 5.1).
* ``batch_mix``: many independent problems of uneven size and fill, mixing
  the banded, random and decay patterns.

Random streams are numpy's PCG64 ``default_rng(seed)``; block values are
drawn in row-major block order.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "BlockMatrix",
    "banded",
    "random_blocks",
    "decay3d",
    "divide_space_order",
    "rmat",
    "batch_mix",
    "config",
    "CONFIGS",
]


@dataclass
class BlockMatrix:
    """A block-sparse matrix given by its nonzero blocks.

    n_rows, n_cols: scalar dimensions (multiples of b).
    b: block size.
    I, J: int32 block row / column of each stored block.
    V: float64 array of shape (nnz, b, b), row-major inside each block.
    meta: free-form description of how the matrix was drawn.
    """

    n_rows: int
    n_cols: int
    b: int
    I: np.ndarray
    J: np.ndarray
    V: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.I.shape[0])

    @property
    def nb_rows(self) -> int:
        return self.n_rows // self.b

    @property
    def nb_cols(self) -> int:
        return self.n_cols // self.b


def _finish(n_rows, n_cols, b, I, J, V, meta) -> BlockMatrix:
    I = np.ascontiguousarray(I, dtype=np.int32)
    J = np.ascontiguousarray(J, dtype=np.int32)
    V = np.ascontiguousarray(V, dtype=np.float64).reshape(len(I), b, b)
    return BlockMatrix(int(n_rows), int(n_cols), int(b), I, J, V, dict(meta))


def banded(nb: int, w: int, b: int, seed: int, rng=None) -> BlockMatrix:
    """Square block-banded matrix: all blocks with |I - J| <= w, entries N(0,1)."""
    rng = np.random.default_rng(seed) if rng is None else rng
    I, J = [], []
    for i in range(nb):
        lo, hi = max(0, i - w), min(nb - 1, i + w)
        I.extend([i] * (hi - lo + 1))
        J.extend(range(lo, hi + 1))
    I = np.array(I, dtype=np.int32)
    J = np.array(J, dtype=np.int32)
    V = rng.standard_normal((len(I), b, b))
    return _finish(nb * b, nb * b, b, I, J, V,
                   {"pattern": "banded", "w": w, "seed": seed})


def random_blocks(nb_rows: int, nb_cols: int, count: int, b: int, seed: int,
                  rng=None, values: str = "normal") -> BlockMatrix:
    """Exactly ``count`` distinct block positions, uniform without replacement.

    values: "normal" for N(0,1) entries, "ones" for all-one blocks (pattern
    studies where the values do not matter).
    """
    rng = np.random.default_rng(seed) if rng is None else rng
    total = nb_rows * nb_cols
    count = int(min(count, total))
    pos = rng.choice(total, size=count, replace=False)
    pos.sort()
    I = (pos // nb_cols).astype(np.int32)
    J = (pos % nb_cols).astype(np.int32)
    if values == "normal":
        V = rng.standard_normal((count, b, b))
    else:
        V = np.ones((count, b, b))
    return _finish(nb_rows * b, nb_cols * b, b, I, J, V,
                   {"pattern": "random", "count": count, "seed": seed})


def divide_space_order(xyz: np.ndarray) -> np.ndarray:
    """Recursive divide-space ordering of points.

    Each box of points is cut at the median along the longest side of its
    bounding box, and the two halves are ordered one after the other,
    recursively, down to single points (Sec. 5.1 names the procedure but
    does not spell it out; this is the reading used here).
    Returns the permutation as an int64 array.
    """
    n = xyz.shape[0]
    out = np.empty(n, dtype=np.int64)
    pos = 0
    stack = [np.arange(n)]
    while stack:
        idx = stack.pop()
        if idx.size == 1:
            out[pos] = idx[0]
            pos += 1
            continue
        pts = xyz[idx]
        axis = int(np.argmax(pts.max(axis=0) - pts.min(axis=0)))
        srt = idx[np.argsort(pts[:, axis], kind="stable")]
        half = srt.size // 2
        # push the upper half first so the lower half is emitted first
        stack.append(srt[half:])
        stack.append(srt[:half])
    return out


def decay3d(natoms: int, side: float, bf_per_atom: int, b: int, seed: int,
            threshold: float = 1e-10, rng=None, chunk: int = 4096) -> BlockMatrix:
    """3D distance-decay matrix standing in for an overlap matrix.

    natoms atoms uniform in [0, side]^3, ordered by ``divide_space_order``,
    bf_per_atom contiguous basis functions per atom, entry
    a_ij = exp(-0.5 * d_ij^2) * U_ij with U_ij ~ U(0.5, 1) drawn per entry
    (so the matrix is not symmetric; functions of one atom have d = 0).
    Blocks whose largest entry is below ``threshold`` are dropped; entries
    inside kept blocks are never truncated.
    """
    from scipy.spatial import cKDTree

    if b % bf_per_atom != 0:
        raise ValueError("block size must be a multiple of the functions per atom")
    rng = np.random.default_rng(seed) if rng is None else rng
    xyz = rng.uniform(0.0, side, size=(natoms, 3))
    xyz = xyz[divide_space_order(xyz)]
    apb = b // bf_per_atom                      # atoms per block
    n = natoms * bf_per_atom
    if n % b != 0:
        raise ValueError("matrix dimension must be a multiple of the block size")
    nb = n // b
    # exp(-0.5 d^2) * U < threshold for every U < 1 once d exceeds this radius
    cutoff = math.sqrt(-2.0 * math.log(threshold))
    pairs = cKDTree(xyz).query_pairs(r=cutoff, output_type="ndarray")
    bi = pairs[:, 0] // apb
    bj = pairs[:, 1] // apb
    cand = np.concatenate([
        bi * nb + bj, bj * nb + bi, np.arange(nb, dtype=np.int64) * (nb + 1)])
    cand = np.unique(cand)                      # sorted: row-major block order
    cI = cand // nb
    cJ = cand % nb
    keep = np.zeros(cand.size, dtype=bool)
    vals = []
    rep = bf_per_atom
    for s in range(0, cand.size, chunk):
        e = min(cand.size, s + chunk)
        ai = xyz[(cI[s:e, None] * apb + np.arange(apb)[None, :])]   # (m, apb, 3)
        aj = xyz[(cJ[s:e, None] * apb + np.arange(apb)[None, :])]
        d2 = ((ai[:, :, None, :] - aj[:, None, :, :]) ** 2).sum(-1)  # (m, apb, apb)
        g = np.exp(-0.5 * d2)
        g = np.repeat(np.repeat(g, rep, axis=1), rep, axis=2)        # (m, b, b)
        u = 0.5 + 0.5 * rng.random((e - s, b, b))
        blk = g * u
        k = blk.reshape(e - s, -1).max(axis=1) >= threshold
        keep[s:e] = k
        vals.append(blk[k])
    V = np.concatenate(vals, axis=0) if vals else np.zeros((0, b, b))
    return _finish(n, n, b, cI[keep], cJ[keep], V, {
        "pattern": "decay3d", "natoms": natoms, "side": side,
        "bf_per_atom": bf_per_atom, "threshold": threshold, "seed": seed})


def rmat(scale: int, edges_per_row: float, a: float, b: int, seed: int, rng=None) -> BlockMatrix:
    """R-MAT graph pattern on a 2^scale x 2^scale block grid (Sec. 5.1, Fig. 4).

    Each edge picks, level by level from the top, one quadrant with
    probabilities (a, q, q, q), q = (1 - a) / 3; repeated edges coincide, so
    the matrix holds at most round(edges_per_row * 2^scale) blocks. a = 0.25
    is the uniformly random case; larger a concentrates the pattern (more
    locality). Block values N(0,1), drawn in row-major block order.
    """
    rng = np.random.default_rng(seed) if rng is None else rng
    n = 1 << scale
    m = int(round(edges_per_row * n))
    q = (1.0 - a) / 3.0
    quad = rng.choice(4, size=(m, scale), p=[a, q, q, q])   # 0: (0,0) 1: (0,1) 2: (1,0) 3: (1,1)
    w = (1 << np.arange(scale - 1, -1, -1)).astype(np.int64)
    I = ((quad >> 1) * w).sum(axis=1)
    J = ((quad & 1) * w).sum(axis=1)
    pos = np.unique(I * n + J)
    I, J = pos // n, pos % n
    V = rng.standard_normal((pos.size, b, b))
    return _finish(n * b, n * b, b, I, J, V, {"pattern": "rmat", "a": a, "seed": seed})


def _decay_with_fill(n: int, b: int, fill: float, rng) -> BlockMatrix:
    """Decay matrix of dimension n with block fill ``fill`` (to one block).

    n/16 atoms in a cube whose side keeps the density of the 32768-function
    decay workload, divide-space ordered as in ``decay3d``. Instead of a
    fixed entry threshold, the kept blocks are the round(fill * nb^2) block
    pairs whose closest atom pair is nearest -- equivalently, the blocks with
    the largest bound exp(-0.5 d_min^2) on their entries, so the threshold is
    the value that gives the wanted fill. Entries exp(-0.5 d^2) * U(0.5, 1).
    """
    from scipy.spatial import cKDTree

    natoms = n // 16
    side = 40.0 * (n / 32768.0) ** (1.0 / 3.0)
    xyz = rng.uniform(0.0, side, size=(natoms, 3))
    xyz = xyz[divide_space_order(xyz)]
    apb = b // 16
    nb = n // b
    K = int(min(nb * nb, max(nb, round(fill * nb * nb))))
    tree = cKDTree(xyz)
    R = side / max(1.0, nb ** 0.5)
    while True:
        pairs = tree.query_pairs(r=R, output_type="ndarray")
        d = np.sqrt(((xyz[pairs[:, 0]] - xyz[pairs[:, 1]]) ** 2).sum(-1))
        bi, bj = pairs[:, 0] // apb, pairs[:, 1] // apb
        key = np.concatenate([bi * nb + bj, bj * nb + bi, np.arange(nb, dtype=np.int64) * (nb + 1)])
        dd = np.concatenate([d, d, np.zeros(nb)])
        o = np.lexsort((dd, key))
        key, dd = key[o], dd[o]
        first = np.concatenate([[True], key[1:] != key[:-1]])
        ukey, dmin = key[first], dd[first]
        if ukey.size >= K or R > 2 * side:
            break
        R *= 1.4
    sel = np.lexsort((ukey, dmin))[:K]
    keys = np.sort(ukey[sel])                   # row-major block order
    I = keys // nb
    J = keys % nb
    ai = xyz[(I[:, None] * apb + np.arange(apb)[None, :])]
    aj = xyz[(J[:, None] * apb + np.arange(apb)[None, :])]
    d2 = ((ai[:, :, None, :] - aj[:, None, :, :]) ** 2).sum(-1)
    g = np.repeat(np.repeat(np.exp(-0.5 * d2), 16, axis=1), 16, axis=2)
    V = g * (0.5 + 0.5 * rng.random((keys.size, b, b)))
    return _finish(n, n, b, I, J, V, {"pattern": "decay3d-fill", "fill": fill})


def batch_mix(count: int, seed: int, b: int = 32, n_lo: int = 2048,
              n_hi: int = 32768, fill_lo: float = 0.005, fill_hi: float = 0.05):
    """``count`` independent (A, B) problems of uneven size and fill.

    n = 32 * floor(exp(U(ln n_lo, ln n_hi)) / 32); the pattern is uniform over
    {banded, decay, random}; the block fill f is log-uniform in
    [fill_lo, fill_hi]; A and B are independent draws of the same kind.
    Returns a list of (A, B) BlockMatrix pairs.
    """
    rng = np.random.default_rng(seed)
    probs = []
    for _ in range(count):
        n = 32 * int(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi))) // 32)
        n = max(n, b)
        n -= n % b
        kind = ("banded", "decay", "random")[int(rng.integers(0, 3))]
        f = math.exp(rng.uniform(math.log(fill_lo), math.log(fill_hi)))
        nb = n // b
        pair = []
        for _side in range(2):
            if kind == "banded":
                w = max(0, int(round((f * nb - 1) / 2)))
                pair.append(banded(nb, w, b, 0, rng=rng))
            elif kind == "random":
                pair.append(random_blocks(nb, nb, max(1, int(round(f * nb * nb))), b, 0, rng=rng))
            else:
                pair.append(_decay_with_fill(n, b, f, rng))
        probs.append(tuple(pair))
    return probs


# The benchmark workloads, by name.
CONFIGS = {
    "banded1024": dict(kind="banded", nb=32, w=3, b=32, leaf=256, seed=1),
    "decay32768": dict(kind="decay3d", natoms=2048, side=40.0, bf=16, b=32, leaf=256, seed=2),
    "random65536": dict(kind="random", nb=2048, fill=0.01, b=32, leaf=256, seed=3),
    "decay131072": dict(kind="decay3d", natoms=8192, side=40.0, bf=16, b=64, leaf=512, seed=4),
}


def config(name: str) -> BlockMatrix:
    """Draw the named workload's matrix A (every named workload computes A*A)."""
    c = CONFIGS[name]
    if c["kind"] == "banded":
        return banded(c["nb"], c["w"], c["b"], c["seed"])
    if c["kind"] == "random":
        nb = c["nb"]
        return random_blocks(nb, nb, int(round(c["fill"] * nb * nb)), c["b"], c["seed"])
    return decay3d(c["natoms"], c["side"], c["bf"], c["b"], c["seed"])
