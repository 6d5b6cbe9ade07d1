"""Quadtree block-sparse matrix multiply on AMD MI355X (gfx950).

A thin ctypes binding over ``libqt.so``; every step of the multiply runs in
the library's HIP kernels. The entry points mirror ``include/qt.h``:

    build(n_rows, n_cols, b, leaf, I, J, V)  -> Matrix      (qt_build)
    multiply(A, B, prec="f64")               -> Matrix      (qt_multiply)
    Matrix.to_blocks(dtype)                  -> (I, J, V)   (qt_to_blocks)
    Matrix.info(), Matrix.stats(), prepare(M, prec)

Block lists may be numpy arrays (host memory) or torch tensors on the GPU
(device memory); streams are torch streams (the current stream by default).
Importing the package loads the library and raises if it is missing: there is
no other implementation to fall back to.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqt.so")

QT_OK, QT_ERR_ARG, QT_ERR_SHAPE, QT_ERR_DUPLICATE, QT_ERR_OOM, QT_ERR_DEVICE, QT_ERR_UNSUPPORTED = range(7)
PREC = {"f64": 0, "f32": 1, "bf16x3": 2}
PREC_NAME = {v: k for k, v in PREC.items()}
MEM_HOST, MEM_DEVICE = 0, 1

STATUS = {0: "ok", 1: "invalid argument", 2: "shape", 3: "duplicate block", 4: "out of memory",
          5: "device error", 6: "unsupported"}


class QtError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_1501_07800_amd/csrc/build.py`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    i64p, i32p = ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)
    lib.qt_build.restype = ctypes.c_int
    lib.qt_build.argtypes = [i64, i64, i32, i32, i64, vp, vp, vp, ctypes.c_int, vp, ctypes.POINTER(vp)]
    lib.qt_multiply.restype = ctypes.c_int
    lib.qt_multiply.argtypes = [vp, vp, ctypes.c_int, vp, ctypes.POINTER(vp)]
    lib.qt_multiply_ex.restype = ctypes.c_int
    lib.qt_multiply_ex.argtypes = [vp, vp, i32, ctypes.c_int, vp, ctypes.POINTER(vp)]
    lib.qt_multiply_tau.restype = ctypes.c_int
    lib.qt_multiply_tau.argtypes = [vp, vp, ctypes.c_double, ctypes.c_int, vp, ctypes.POINTER(vp)]
    lib.qt_norms.restype = ctypes.c_int
    lib.qt_norms.argtypes = [vp, vp, vp, ctypes.c_int, vp]
    lib.qt_add.restype = ctypes.c_int
    lib.qt_add.argtypes = [vp, vp, vp, ctypes.POINTER(vp)]
    lib.qt_truncate.restype = ctypes.c_int
    lib.qt_truncate.argtypes = [vp, ctypes.c_double, vp, ctypes.POINTER(vp), i64p, ctypes.POINTER(ctypes.c_double)]
    lib.qt_sysq.restype = ctypes.c_int
    lib.qt_sysq.argtypes = [vp, ctypes.c_int, vp, ctypes.POINTER(vp)]
    lib.qt_info.restype = ctypes.c_int
    lib.qt_info.argtypes = [vp, i64p, i64p, i32p, i32p, ctypes.POINTER(ctypes.c_int)]
    lib.qt_nblocks.restype = ctypes.c_int
    lib.qt_nblocks.argtypes = [vp, i64p]
    lib.qt_to_blocks.restype = ctypes.c_int
    lib.qt_to_blocks.argtypes = [vp, vp, vp, vp, ctypes.c_int, ctypes.c_int, vp]
    lib.qt_to_blocks_noalloc.restype = ctypes.c_int
    lib.qt_to_blocks_noalloc.argtypes = [vp, vp, vp, vp, ctypes.c_int, vp]
    lib.qt_get_blocks.restype = ctypes.c_int
    lib.qt_get_blocks.argtypes = [vp, i64, vp, vp, vp, vp, ctypes.c_int, ctypes.c_int, vp]
    lib.qt_stats.restype = ctypes.c_int
    lib.qt_stats.argtypes = [vp, i64p, i32, i64p]
    lib.qt_levels.restype = ctypes.c_int
    lib.qt_levels.argtypes = [vp, i64p, i32, i32p]
    lib.qt_prepare.restype = ctypes.c_int
    lib.qt_prepare.argtypes = [vp, ctypes.c_int, vp]
    lib.qt_free.restype = None
    lib.qt_free.argtypes = [vp]
    lib.qt_profile.restype = ctypes.c_int
    lib.qt_profile.argtypes = [ctypes.c_int]
    lib.qt_profile_read.restype = ctypes.c_int
    lib.qt_profile_read.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                    i64p, i64p, i64p]
    lib.qt_plan_create.restype = ctypes.c_int
    lib.qt_plan_create.argtypes = [i32, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_int, vp, ctypes.POINTER(vp)]
    lib.qt_plan_execute.restype = ctypes.c_int
    lib.qt_plan_execute.argtypes = [vp, vp]
    lib.qt_plan_replay.restype = ctypes.c_int
    lib.qt_plan_replay.argtypes = [vp, vp]
    lib.qt_plan_tune.restype = ctypes.c_int
    lib.qt_plan_tune.argtypes = [vp, vp, ctypes.c_int, i32p, ctypes.POINTER(ctypes.c_float)]
    lib.qt_plan_set_schedule.restype = ctypes.c_int
    lib.qt_plan_set_schedule.argtypes = [vp, i32]
    lib.qt_plan_result.restype = ctypes.c_int
    lib.qt_plan_result.argtypes = [vp, i32, ctypes.POINTER(vp)]
    lib.qt_plan_info.restype = ctypes.c_int
    lib.qt_plan_info.argtypes = [vp, i64p, i64p, i32p]
    lib.qt_plan_destroy.restype = None
    lib.qt_plan_destroy.argtypes = [vp]
    lib.qt_tune_leaf.restype = ctypes.c_int
    lib.qt_tune_leaf.argtypes = [vp, vp, ctypes.c_int, vp, ctypes.c_int, i32p, i32p, ctypes.POINTER(ctypes.c_float),
                                 i32, i32p]
    lib.qt_tune_cache.restype = ctypes.c_int
    lib.qt_tune_cache.argtypes = [ctypes.c_char_p]
    lib.qt_tune_leaf_cached.restype = ctypes.c_int
    lib.qt_tune_leaf_cached.argtypes = [vp, vp, ctypes.c_int, vp, ctypes.c_int, ctypes.c_char_p, i32p, i32p]
    lib.qt_plan_tune_cached.restype = ctypes.c_int
    lib.qt_plan_tune_cached.argtypes = [vp, vp, ctypes.c_int, ctypes.c_char_p, i32p, i32p]
    lib.qt_last_error.restype = ctypes.c_char_p
    lib.qt_last_error.argtypes = []
    lib.qt_probe_batched.restype = ctypes.c_int
    lib.qt_probe_batched.argtypes = [ctypes.c_int, i32, i64, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]
    lib.qt_probe_mfma.restype = ctypes.c_int
    lib.qt_probe_mfma.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]
    lib.qt_version.restype = ctypes.c_char_p
    lib.qt_version.argtypes = []
    lib.qt_set_allocator.restype = ctypes.c_int
    lib.qt_set_allocator.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    return lib


lib = _load()

# Device allocator callbacks (qt_set_allocator): alloc(bytes, stream, ctx) -> ptr, free_(ptr, stream, ctx).
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)
_installed = None     # the callbacks installed now
_kept = []            # every callback pair ever installed: buffers made under one are returned through it


def set_allocator(alloc, free_):
    """qt_set_allocator with Python callables alloc(nbytes, stream) -> int and
    free_(ptr, stream); (None, None) restores HIP's stream-ordered pool."""
    global _installed
    if alloc is None and free_ is None:
        _check(lib.qt_set_allocator(None, None, None))
        _installed = None
        return
    a = ALLOC_FN(lambda n, st, ctx: alloc(n, st))
    f = FREE_FN(lambda p, st, ctx: free_(p, st))
    _kept.append((a, f, alloc, free_))
    _check(lib.qt_set_allocator(ctypes.cast(a, ctypes.c_void_p), ctypes.cast(f, ctypes.c_void_p), None))
    _installed = (a, f, alloc, free_)


class TorchAllocator:
    """Device memory from torch's caching allocator.

    A buffer is a raw block of torch's caching allocator, allocated on the
    stream the library names, so torch ties it to that stream. A buffer freed
    on the stream it was made on goes back to torch at once: torch hands it
    out again only to later work on that stream. A buffer freed on another
    stream (its last use was queued there) goes back once an event recorded
    on that stream has completed, checked at every later alloc or free: that
    is the ordering qt_set_allocator asks for. ``outstanding()`` counts the
    buffers the library holds; ``pending()`` those freed but waiting for
    their event.
    """

    def __init__(self):
        import collections
        import threading
        import torch
        self._torch = torch
        self._raw_alloc = torch._C._cuda_cudaCachingAllocator_raw_alloc
        self._raw_delete = torch._C._cuda_cudaCachingAllocator_raw_delete
        self._live = {}                            # pointer -> stream it was made on
        self._waiting = collections.deque()        # (event, pointer), in the order freed
        self._events = []                          # completed events, for reuse
        self._streams = {}
        self._lock = threading.Lock()

    def _stream(self, ptr):
        st = self._streams.get(ptr)
        if st is None:
            torch = self._torch
            st = torch.cuda.ExternalStream(ptr) if ptr else torch.cuda.default_stream()
            self._streams[ptr] = st
        return st

    def _drain(self):
        # under the lock: give back the buffers whose last use has finished
        while self._waiting and self._waiting[0][0].query():
            ev, p = self._waiting.popleft()
            self._raw_delete(p)
            self._events.append(ev)

    def alloc(self, nbytes, stream):
        st = stream or 0
        with self._lock:
            self._drain()
            try:
                p = self._raw_alloc(max(int(nbytes), 1), st)
            except Exception:
                return None
            self._live[p] = st
        return p

    def free(self, p, stream):
        st = stream or 0
        with self._lock:
            made_on = self._live.pop(p, None)
            if made_on is None:
                return
            if st == made_on:
                self._raw_delete(p)
            else:
                ev = self._events.pop() if self._events else self._torch.cuda.Event()
                ev.record(self._stream(st))
                self._waiting.append((ev, p))
            self._drain()

    def outstanding(self) -> int:
        with self._lock:
            return len(self._live)

    def pending(self) -> int:
        with self._lock:
            self._drain()
            return len(self._waiting)


def use_torch_allocator() -> TorchAllocator:
    """Route the library's device memory through torch's caching allocator."""
    ta = TorchAllocator()
    set_allocator(ta.alloc, ta.free)
    return ta


def use_hip_pool():
    """Back to HIP's stream-ordered pool (the library's own default)."""
    set_allocator(None, None)


def _default_allocator():
    """On a GPU, torch's caching allocator serves the library's device memory
    (QT_ALLOCATOR=hip keeps HIP's stream-ordered pool instead)."""
    if os.environ.get("QT_ALLOCATOR", "torch") != "torch":
        return None
    try:
        import torch
    except ImportError:
        return None
    if not torch.cuda.is_available():
        return None
    return use_torch_allocator()


EXPORTS = ("qt_build", "qt_multiply", "qt_multiply_ex", "qt_multiply_tau", "qt_norms", "qt_add", "qt_truncate", "qt_sysq", "qt_info", "qt_nblocks", "qt_to_blocks", "qt_to_blocks_noalloc", "qt_get_blocks", "qt_stats", "qt_levels", "qt_prepare", "qt_free",
           "qt_plan_create", "qt_plan_execute", "qt_plan_replay", "qt_plan_tune", "qt_plan_set_schedule", "qt_plan_result", "qt_plan_info",
           "qt_plan_destroy", "qt_tune_leaf", "qt_tune_cache", "qt_tune_leaf_cached", "qt_plan_tune_cached", "qt_profile", "qt_profile_read", "qt_probe_mfma", "qt_probe_batched", "qt_last_error", "qt_version",
           "qt_set_allocator")
NOALLOC_MAX_BLOCKS = 1 << 20   # QT_NOALLOC_MAX_BLOCKS
PLAN_SCHEDULES = ("flat", "balanced", "xcd-dynamic", "dynamic-16")   # QT_PLAN_SCHEDULES
PLAN_ORDER_MORTON, PLAN_TILE_WAVE, PLAN_CONFIGS = 4, 8, 16


def plan_config_name(c: int) -> str:
    """Name of plan configuration c: the schedule, then '+morton' (every
    problem in Morton order) and '+wave-tiles' (b = 64: a wave per 32 x 32
    tile instead of a workgroup per C block sharing operands through LDS)."""
    return PLAN_SCHEDULES[c & 3] + ("+morton" if c & PLAN_ORDER_MORTON else "") + \
        ("+wave-tiles" if c & PLAN_TILE_WAVE else "")


def plan_config(name) -> int:
    """Inverse of plan_config_name (an int is returned as it is)."""
    if isinstance(name, int):
        return name
    parts = name.split("+")
    c = PLAN_SCHEDULES.index(parts[0])
    for p in parts[1:]:
        c |= {"morton": PLAN_ORDER_MORTON, "wave-tiles": PLAN_TILE_WAVE}[p]
    return c


def _check(status: int):
    if status != QT_OK:
        raise QtError(status, lib.qt_last_error().decode(errors="replace"))


def _stream_ptr(stream):
    if stream is None:
        import torch
        if not torch.cuda.is_available():
            return None
        stream = torch.cuda.current_stream()
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


class Matrix:
    """Owning wrapper of a qt_matrix handle (freed with qt_free)."""

    def __init__(self, handle: int):
        self._h = ctypes.c_void_p(handle)

    @property
    def handle(self):
        return self._h

    def free(self):
        if self._h is not None and self._h.value:
            lib.qt_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def info(self) -> dict:
        r, c, n = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        b, leaf, vt = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int()
        _check(lib.qt_info(self._h, ctypes.byref(r), ctypes.byref(c), ctypes.byref(b), ctypes.byref(leaf),
                           ctypes.byref(vt)))
        _check(lib.qt_nblocks(self._h, ctypes.byref(n)))
        return {"n_rows": r.value, "n_cols": c.value, "b": b.value, "leaf": leaf.value, "nblocks": n.value,
                "value_type": PREC_NAME[vt.value]}

    @property
    def nblocks(self) -> int:
        return self.info()["nblocks"]

    def stats(self) -> dict:
        pairs = (ctypes.c_int64 * 64)()
        prods = ctypes.c_int64()
        _check(lib.qt_stats(self._h, pairs, 64, ctypes.byref(prods)))
        nl = ctypes.c_int32()
        _check(lib.qt_levels(self._h, None, 0, ctypes.byref(nl)))   # the depth + 1
        return {"pairs": np.array(pairs[:nl.value], np.int64), "products": prods.value}

    def levels(self) -> np.ndarray:
        """Non-NIL quadtree nodes per level, root first (qt_levels)."""
        nodes = (ctypes.c_int64 * 64)()
        nl = ctypes.c_int32()
        _check(lib.qt_levels(self._h, nodes, 64, ctypes.byref(nl)))
        return np.array(nodes[:nl.value], np.int64)

    def to_blocks(self, dtype: str = "f64", stream=None):
        """Copy out as (I, J, V) numpy arrays sorted by (I, J)."""
        inf = self.info()
        n, b = inf["nblocks"], inf["b"]
        I = np.empty(n, np.int32)
        J = np.empty(n, np.int32)
        V = np.empty((n, b, b), np.float64 if dtype == "f64" else np.float32)
        _check(lib.qt_to_blocks(self._h, I.ctypes.data, J.ctypes.data, V.ctypes.data, PREC[dtype], MEM_HOST,
                                _stream_ptr(stream)))
        return I, J, V

    def pattern(self, stream=None):
        """Block positions (I, J) sorted row-major, without the values."""
        n = self.info()["nblocks"]
        I = np.empty(n, np.int32)
        J = np.empty(n, np.int32)
        _check(lib.qt_to_blocks(self._h, I.ctypes.data, J.ctypes.data, None, PREC["f64"], MEM_HOST,
                                _stream_ptr(stream)))
        return I, J

    def norms(self, stream=None):
        """qt_norms: (squared Frobenius norm of every block in (I, J) order, of the matrix)."""
        n = self.info()["nblocks"]
        bn = np.empty(max(n, 1), np.float64)
        tot = ctypes.c_double()
        _check(lib.qt_norms(self._h, bn.ctypes.data, ctypes.byref(tot), MEM_HOST, _stream_ptr(stream)))
        return bn[:n], tot.value

    def get_blocks(self, I, J, dtype: str = "f64", stream=None):
        """Chosen blocks (I[t], J[t]) as (values, found) numpy arrays (qt_get_blocks)."""
        I = np.ascontiguousarray(I, np.int32)
        J = np.ascontiguousarray(J, np.int32)
        b = self.info()["b"]
        V = np.empty((len(I), b, b), np.float64 if dtype == "f64" else np.float32)
        F = np.empty(len(I), np.int32)
        _check(lib.qt_get_blocks(self._h, len(I), I.ctypes.data, J.ctypes.data, V.ctypes.data, F.ctypes.data,
                                 PREC[dtype], MEM_HOST, _stream_ptr(stream)))
        return V, F.astype(bool)

    def to_blocks_device(self, I, J, V, dtype: str = "f64", stream=None):
        """Copy out into caller-provided torch device tensors (no host sync)."""
        _check(lib.qt_to_blocks(self._h, I.data_ptr(), J.data_ptr(), V.data_ptr(), PREC[dtype], MEM_DEVICE,
                                _stream_ptr(stream)))

    def to_blocks_noalloc(self, I, J, V, dtype: str = "f64", stream=None):
        """qt_to_blocks_noalloc: the same copy-out into caller-provided torch
        device tensors, using the library's fixed scratch instead of any
        allocation (V may be None for the pattern only)."""
        _check(lib.qt_to_blocks_noalloc(self._h, I.data_ptr(), J.data_ptr(), None if V is None else V.data_ptr(),
                                        PREC[dtype], _stream_ptr(stream)))


def build(n_rows: int, n_cols: int, b: int, leaf: int, I, J, V, stream=None) -> Matrix:
    """qt_build from a block list (numpy arrays: host; torch GPU tensors: device)."""
    out = ctypes.c_void_p()
    n = int(I.shape[0])
    if _is_torch(I):
        assert I.dtype.__str__() == "torch.int32" and J.dtype.__str__() == "torch.int32"
        assert str(V.dtype) == "torch.float64" and V.is_contiguous()
        where = MEM_DEVICE if I.is_cuda else MEM_HOST
        pI, pJ, pV = I.data_ptr(), J.data_ptr(), V.data_ptr()
        keep = (I, J, V)
    else:
        I = np.ascontiguousarray(I, np.int32)
        J = np.ascontiguousarray(J, np.int32)
        V = np.ascontiguousarray(V, np.float64)
        where = MEM_HOST
        pI, pJ, pV = I.ctypes.data, J.ctypes.data, V.ctypes.data
        keep = (I, J, V)
    _check(lib.qt_build(n_rows, n_cols, b, leaf, n, pI if n else None, pJ if n else None, pV if n else None,
                        where, _stream_ptr(stream), ctypes.byref(out)))
    del keep
    return Matrix(out.value)


def from_blockmatrix(M, leaf: int, stream=None) -> Matrix:
    """qt_build from a ``workloads.BlockMatrix`` (host arrays)."""
    return build(M.n_rows, M.n_cols, M.b, leaf, M.I, M.J, M.V, stream=stream)


def multiply(A: Matrix, B: Matrix, prec: str = "f64", stream=None) -> Matrix:
    """qt_multiply: C = A*B at precision "f64", "f32" or "bf16x3"."""
    out = ctypes.c_void_p()
    _check(lib.qt_multiply(A.handle, B.handle, PREC[prec], _stream_ptr(stream), ctypes.byref(out)))
    return Matrix(out.value)


class _Borrowed(Matrix):
    """A result handle owned by a Plan (never freed through this wrapper)."""

    def __init__(self, handle: int, plan):
        super().__init__(handle)
        self._plan = plan          # keeps the plan alive while the handle is used

    def free(self):
        self._h = None


class Plan:
    """qt_plan_*: many independent C_i = A_i * B_i, numeric phase in one launch."""

    def __init__(self, As, Bs, prec: str = "f64", stream=None):
        n = len(As)
        arrA = (ctypes.c_void_p * n)(*[a.handle.value for a in As])
        arrB = (ctypes.c_void_p * n)(*[b.handle.value for b in Bs])
        out = ctypes.c_void_p()
        _check(lib.qt_plan_create(n, arrA, arrB, PREC[prec], _stream_ptr(stream), ctypes.byref(out)))
        self._h = out
        self.count = n
        self._keep = (list(As), list(Bs))

    def execute(self, stream=None, graph: bool = True):
        """qt_plan_replay (graph=True: the plan's captured graph replayed) or
        qt_plan_execute (graph=False: the kernels launched on `stream`)."""
        fn = lib.qt_plan_replay if graph else lib.qt_plan_execute
        _check(fn(self._h, _stream_ptr(stream)))

    def tune(self, reps: int = 3, stream=None):
        """qt_plan_tune: the fastest configuration's name and the mean time
        (ms) of every configuration it tried."""
        cfg = ctypes.c_int32()
        ms = (ctypes.c_float * PLAN_CONFIGS)()
        _check(lib.qt_plan_tune(self._h, _stream_ptr(stream), reps, ctypes.byref(cfg), ms))
        return plan_config_name(cfg.value), {plan_config_name(i): ms[i] for i in range(PLAN_CONFIGS) if ms[i] >= 0}

    def tune_cached(self, batch_class: str, reps: int = 3, stream=None):
        """qt_plan_tune_cached: the configuration the tuning cache holds for
        this batch class, else the tuner's (then stored); (name, cached)."""
        cfg, cached = ctypes.c_int32(), ctypes.c_int32()
        _check(lib.qt_plan_tune_cached(self._h, _stream_ptr(stream), reps, batch_class.encode(), ctypes.byref(cfg),
                                       ctypes.byref(cached)))
        return plan_config_name(cfg.value), bool(cached.value)

    def set_schedule(self, name):
        """qt_plan_set_schedule with a configuration name (or number)."""
        _check(lib.qt_plan_set_schedule(self._h, plan_config(name)))

    def result(self, i: int) -> Matrix:
        out = ctypes.c_void_p()
        _check(lib.qt_plan_result(self._h, i, ctypes.byref(out)))
        return _Borrowed(out.value, self)

    def info(self) -> dict:
        items, prods, sched = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
        _check(lib.qt_plan_info(self._h, ctypes.byref(items), ctypes.byref(prods), ctypes.byref(sched)))
        return {"work_items": items.value, "products": prods.value, "schedule": plan_config_name(sched.value),
                "config": sched.value}

    def destroy(self):
        if self._h is not None and self._h.value:
            lib.qt_plan_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def tune_leaf(A: Matrix, B: Matrix, prec: str = "f64", reps: int = 3, stream=None):
    """qt_tune_leaf: fastest leaf size for C = A*B, with the tried sizes' times (ms)."""
    best = ctypes.c_int32()
    leaves = (ctypes.c_int32 * 8)()
    ms = (ctypes.c_float * 8)()
    n = ctypes.c_int32()
    _check(lib.qt_tune_leaf(A.handle, B.handle, PREC[prec], _stream_ptr(stream), reps, ctypes.byref(best), leaves,
                            ms, 8, ctypes.byref(n)))
    return best.value, {leaves[i]: ms[i] for i in range(n.value)}


def tune_cache(path):
    """qt_tune_cache: keep the tuners' choices in the text file `path` (None: no file)."""
    _check(lib.qt_tune_cache(None if path is None else os.fsencode(path)))


def tune_leaf_cached(A: Matrix, B: Matrix, pattern_class: str, prec: str = "f64", reps: int = 3, stream=None):
    """qt_tune_leaf_cached: the leaf size the tuning cache holds for this
    pattern class, else the tuner's (then stored); (leaf, cached)."""
    best, cached = ctypes.c_int32(), ctypes.c_int32()
    _check(lib.qt_tune_leaf_cached(A.handle, B.handle, PREC[prec], _stream_ptr(stream), reps, pattern_class.encode(),
                                   ctypes.byref(best), ctypes.byref(cached)))
    return best.value, bool(cached.value)


OP_TRANS_A, OP_TRANS_B, OP_UPPER = 1, 2, 4


def multiply_ex(A: Matrix, B: Matrix, trans_a: bool = False, trans_b: bool = False, upper: bool = False,
                prec: str = "f64", stream=None) -> Matrix:
    """qt_multiply_ex: C = op(A) op(B), optionally only the upper block triangle."""
    flags = (OP_TRANS_A if trans_a else 0) | (OP_TRANS_B if trans_b else 0) | (OP_UPPER if upper else 0)
    out = ctypes.c_void_p()
    _check(lib.qt_multiply_ex(A.handle, B.handle, flags, PREC[prec], _stream_ptr(stream), ctypes.byref(out)))
    return Matrix(out.value)


def multiply_tau(A: Matrix, B: Matrix, tau: float, prec: str = "f64", stream=None) -> Matrix:
    """qt_multiply_tau: C = A*B without the products whose operands' Frobenius
    norms multiply to less than tau (at every quadtree level)."""
    out = ctypes.c_void_p()
    _check(lib.qt_multiply_tau(A.handle, B.handle, float(tau), PREC[prec], _stream_ptr(stream), ctypes.byref(out)))
    return Matrix(out.value)


def add(A: Matrix, B: Matrix, stream=None) -> Matrix:
    """qt_add: C = A + B (union of the block patterns)."""
    out = ctypes.c_void_p()
    _check(lib.qt_add(A.handle, B.handle, _stream_ptr(stream), ctypes.byref(out)))
    return Matrix(out.value)


def truncate(M: Matrix, eps: float, stream=None):
    """qt_truncate: drop the smallest blocks while ||removed||_F < eps; returns (T, removed, ||E||_F^2)."""
    out = ctypes.c_void_p()
    k = ctypes.c_int64()
    e2 = ctypes.c_double()
    _check(lib.qt_truncate(M.handle, eps, _stream_ptr(stream), ctypes.byref(out), ctypes.byref(k), ctypes.byref(e2)))
    return Matrix(out.value), k.value, e2.value


def sysq(A: Matrix, prec: str = "f64", stream=None) -> Matrix:
    """qt_sysq: upper block triangle of S*S, S symmetric given by its upper block triangle A."""
    out = ctypes.c_void_p()
    _check(lib.qt_sysq(A.handle, PREC[prec], _stream_ptr(stream), ctypes.byref(out)))
    return Matrix(out.value)


def prepare(M: Matrix, prec: str, stream=None):
    """qt_prepare: build the operand forms a multiply at ``prec`` reads."""
    _check(lib.qt_prepare(M.handle, PREC[prec], _stream_ptr(stream)))


def profile(enable: bool):
    _check(lib.qt_profile(1 if enable else 0))


def profile_read() -> dict:
    a, b = ctypes.c_double(), ctypes.c_double()
    calls, prods, cb = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(lib.qt_profile_read(ctypes.byref(a), ctypes.byref(b), ctypes.byref(calls), ctypes.byref(prods),
                               ctypes.byref(cb)))
    return {"symbolic_ms": a.value, "numeric_ms": b.value, "calls": calls.value, "products": prods.value,
            "c_blocks": cb.value}


def probe_mfma(prec: str = "f64", stream=None) -> float:
    """qt_probe_mfma: TFLOP/s of a register-only loop of the path's MFMA instruction."""
    out = ctypes.c_double()
    _check(lib.qt_probe_mfma(PREC[prec], _stream_ptr(stream), ctypes.byref(out)))
    return out.value


def probe_batched(prec: str = "f64", b: int = 32, count: int = 64000, stream=None) -> float:
    """qt_probe_batched: TFLOP/s of `count` b x b block products C_i = A B
    (one operand pair for all) through the numeric kernels."""
    out = ctypes.c_double()
    _check(lib.qt_probe_batched(PREC[prec], b, count, _stream_ptr(stream), ctypes.byref(out)))
    return out.value


def version() -> str:
    return lib.qt_version().decode()


# installed last: it calls into the library through the helpers above
ALLOCATOR = _default_allocator()
