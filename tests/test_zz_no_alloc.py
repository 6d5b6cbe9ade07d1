"""qt_to_blocks_noalloc: the allocation-free copy-out, through the C ABI.

Its output must equal qt_to_blocks' (device arrays) bit for bit, on two
calls in a row where the second matrix is smaller than the first (the shared
scratch keeps the first call's contents), for both output types and for the
pattern alone; during those calls the installed allocator must not be
called at all. Sizes beyond QT_NOALLOC_MAX_BLOCKS are refused.
"""
import numpy as np
import pytest

from tests._util import random_pattern

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


class Counting:
    """Allocator over torch's that counts its calls; with refuse=True it
    returns no memory at all."""

    def __init__(self, base):
        self.base, self.calls, self.refuse = base, 0, False

    def alloc(self, n, stream):
        self.calls += 1
        return None if self.refuse else self.base.alloc(n, stream)

    def free(self, p, stream):
        self.calls += 1
        self.base.free(p, stream)


def _restore(qt):
    if qt.ALLOCATOR is not None:
        qt.set_allocator(qt.ALLOCATOR.alloc, qt.ALLOCATOR.free)
    else:
        qt.use_hip_pool()


def _device_out(n, b, dtype):
    import torch
    I = torch.full((max(n, 1),), -7, dtype=torch.int32, device="cuda")
    J = torch.full((max(n, 1),), -7, dtype=torch.int32, device="cuda")
    V = torch.full((max(n, 1), b, b), float("nan"), dtype=dtype, device="cuda")
    return I, J, V


def _copy_both(qt, M, dtype_name, counter, with_values=True):
    """(reference, allocation-free) outputs of one matrix as torch tensors."""
    import torch
    dt = torch.float64 if dtype_name == "f64" else torch.float32
    inf = M.info()
    n, b = inf["nblocks"], inf["b"]
    stream = torch.cuda.current_stream()
    rI, rJ, rV = _device_out(n, b, dt)
    M.to_blocks_device(rI, rJ, rV, dtype_name)
    gI, gJ, gV = _device_out(n, b, dt)
    torch.cuda.synchronize()
    counter.calls = 0
    counter.refuse = True
    st = qt.lib.qt_to_blocks_noalloc(M.handle, gI.data_ptr(), gJ.data_ptr(),
                                     gV.data_ptr() if with_values else None, qt.PREC[dtype_name],
                                     stream.cuda_stream)
    counter.refuse = False
    assert st == qt.QT_OK, qt.lib.qt_last_error()
    assert counter.calls == 0, f"the allocation-free copy-out called the allocator {counter.calls} times"
    torch.cuda.synchronize()
    return (rI[:n], rJ[:n], rV[:n]), (gI[:n], gJ[:n], gV[:n])


@pytest.mark.parametrize("dtype_name", ["f64", "f32"])
def test_noalloc_matches_to_blocks_twice_second_smaller(qt, dtype_name):
    import torch
    rng = np.random.default_rng(90)
    big = random_pattern(rng, 96, 80, 0.12, 32)        # ~920 blocks: several sort tiles
    A = random_pattern(rng, 40, 40, 0.1, 32)
    hBig = qt.from_blockmatrix(big, 128)
    hA = qt.from_blockmatrix(A, 64)
    hC = qt.multiply(hA, hA, "f64" if dtype_name == "f64" else "f32")   # a multiply result, smaller than big
    counter = Counting(qt.TorchAllocator())
    qt.set_allocator(counter.alloc, counter.free)
    try:
        sizes = []
        for M in (hBig, hC):
            n = M.info()["nblocks"]
            sizes.append(n)
            _say("noalloc copy-out:", dtype_name, "blocks", n)
            (rI, rJ, rV), (gI, gJ, gV) = _copy_both(qt, M, dtype_name, counter)
            assert torch.equal(rI, gI) and torch.equal(rJ, gJ)
            assert torch.equal(rV.view(torch.int64 if dtype_name == "f64" else torch.int32),
                               gV.view(torch.int64 if dtype_name == "f64" else torch.int32))
        assert sizes[1] < sizes[0]
        # the second matrix again, pattern only (values NULL)
        (rI, rJ, _), (gI, gJ, gV) = _copy_both(qt, hC, dtype_name, counter, with_values=False)
        assert torch.equal(rI, gI) and torch.equal(rJ, gJ)
        assert bool(torch.isnan(gV).all()), "values written although NULL was passed"
    finally:
        _restore(qt)


def test_noalloc_small_and_empty(qt):
    """One block, two blocks (below one sort tile) and an all-NIL matrix."""
    import torch
    counter = Counting(qt.TorchAllocator())
    rng = np.random.default_rng(91)
    cases = []
    for I, J in (([3], [1]), ([5, 0], [2, 7])):
        I = np.array(I, np.int32)
        J = np.array(J, np.int32)
        V = rng.standard_normal((len(I), 16, 16))
        cases.append(qt.build(128, 128, 16, 32, I, J, V))
    cases.append(qt.build(128, 128, 16, 32, np.zeros(0, np.int32), np.zeros(0, np.int32),
                          np.zeros((0, 16, 16))))
    qt.set_allocator(counter.alloc, counter.free)
    try:
        for M in cases:
            (rI, rJ, rV), (gI, gJ, gV) = _copy_both(qt, M, "f64", counter)
            assert torch.equal(rI, gI) and torch.equal(rJ, gJ) and torch.equal(rV, gV)
    finally:
        _restore(qt)


def test_noalloc_refuses_beyond_its_scratch(qt):
    """A matrix with QT_NOALLOC_MAX_BLOCKS + 1 blocks is refused with
    UNSUPPORTED (and nothing written); the regular copy-out still works."""
    import torch
    n = qt.NOALLOC_MAX_BLOCKS + 1
    nb = 2048
    t = torch.arange(n, dtype=torch.int64, device="cuda")
    I = (t // nb).to(torch.int32)
    J = (t % nb).to(torch.int32)
    V = torch.zeros((n, 16, 16), dtype=torch.float64, device="cuda")
    M = qt.build(16 * nb, 16 * nb, 16, 128, I, J, V)
    del V
    assert M.info()["nblocks"] == n
    gI = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    gJ = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    st = qt.lib.qt_to_blocks_noalloc(M.handle, gI.data_ptr(), gJ.data_ptr(), None, qt.PREC["f64"],
                                     torch.cuda.current_stream().cuda_stream)
    assert st == qt.QT_ERR_UNSUPPORTED
    assert b"at most" in qt.lib.qt_last_error()
    torch.cuda.synchronize()
    assert bool((gI == -7).all())
    del M


def test_noalloc_argument_errors(qt):
    import torch
    rng = np.random.default_rng(92)
    A = random_pattern(rng, 8, 8, 0.3, 16)
    M = qt.from_blockmatrix(A, 32)
    I = torch.zeros(A.nnz, dtype=torch.int32, device="cuda")
    L = qt.lib
    assert L.qt_to_blocks_noalloc(None, I.data_ptr(), I.data_ptr(), None, 0, None) == qt.QT_ERR_ARG
    assert L.qt_to_blocks_noalloc(M.handle, None, None, None, 0, None) == qt.QT_ERR_ARG
    assert L.qt_to_blocks_noalloc(M.handle, I.data_ptr(), I.data_ptr(), None, 2, None) == qt.QT_ERR_UNSUPPORTED
