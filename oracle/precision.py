"""Reduced-precision input forms for checking the FP32 and split-BF16 paths.

TEST INFRASTRUCTURE (see the package docstring). The paper computes in fp64
and fp32 only; the split-bf16 form is an extension whose exact rounded result
has no plain definition, so these helpers give the inputs' rounded forms and
the tests bound the GPU result against the fp64 oracle run on them.

* ``to_fp32``: round every entry to the nearest binary32 value, ties to even
  (numpy's float64 -> float32 conversion).
* ``bf16_rne``: round binary32 values to bfloat16 (8 significand bits), ties
  to even, written from the IEEE-754 definition on the bit pattern.
* ``split_bf16``: hi = bf16(a32), lo = bf16(a32 - hi); the difference is exact
  in binary32, so a32 = hi + lo + (rounding error of lo).
"""
from __future__ import annotations

import numpy as np

from workloads import BlockMatrix


def to_fp32(x: np.ndarray) -> np.ndarray:
    return np.asarray(x, dtype=np.float64).astype(np.float32)


def bf16_rne(x32: np.ndarray) -> np.ndarray:
    """Round binary32 values to bfloat16 (returned as binary32 values)."""
    x32 = np.ascontiguousarray(x32, dtype=np.float32)
    u = x32.view(np.uint32).astype(np.uint64)
    nan = np.isnan(x32)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    out = r.view(np.float32).copy()
    out[nan] = np.float32(np.nan)
    return out


def split_bf16(x: np.ndarray):
    a32 = to_fp32(x)
    hi = bf16_rne(a32)
    lo = bf16_rne((a32 - hi).astype(np.float32))
    return hi, lo


def with_values(M: BlockMatrix, V: np.ndarray) -> BlockMatrix:
    """Same pattern as M, new values (converted to float64)."""
    return BlockMatrix(M.n_rows, M.n_cols, M.b, M.I, M.J,
                       np.ascontiguousarray(V, dtype=np.float64).reshape(M.V.shape), dict(M.meta))
