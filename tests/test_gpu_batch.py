"""GPU: batched multiplies (qt_plan_*) and the leaf-size tuner, through the C ABI.

Every plan result must equal the single-multiply result bit for bit (the
same per-wave block GEMM, the same product order) and match the CPU oracle
(pattern exact, fp64 within 1e-12 relative to |A||B|). Graph replays are
checked against direct launches several times, with other GPU work between
replays.
"""
import numpy as np
import pytest

import oracle
import workloads as wl
from tests._util import compare, positions, random_pattern

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


def _problems(b=32, seed=0):
    rng = np.random.default_rng(seed)
    probs = []
    probs.append((wl.banded(40, 2, b, seed=1), wl.banded(40, 3, b, seed=2)))
    probs.append((random_pattern(rng, 70, 70, 0.03, b), random_pattern(rng, 70, 70, 0.03, b)))
    probs.append((wl.decay3d(256, 14.0, 16, b, seed=3), wl.decay3d(256, 14.0, 16, b, seed=4)))
    probs.append((random_pattern(rng, 23, 57, 0.1, b), random_pattern(rng, 57, 31, 0.1, b)))   # rectangular
    probs.append((random_pattern(rng, 5, 5, 0.0, b), random_pattern(rng, 5, 5, 0.5, b)))      # empty A
    probs.append((random_pattern(rng, 1, 1, 1.0, b), random_pattern(rng, 1, 1, 1.0, b)))      # one block
    probs.append((random_pattern(rng, 120, 120, 0.01, b), random_pattern(rng, 120, 120, 0.02, b)))
    return probs


def _blocks(h, A, B):
    I, J, V = h.to_blocks("f64")
    return wl.BlockMatrix(A.n_rows, B.n_cols, A.b, I, J, V)


def _check_against_oracle(C, A, B, leaf, tol):
    ref, _ = oracle.multiply(A, B, leaf)
    absAB, _ = oracle.multiply(A, B, leaf, use_abs=True)
    same, _, e_f, e_cw = compare(ref, C, absAB)
    assert same, (ref.nnz, C.nnz)
    assert e_cw <= tol, e_cw


@pytest.mark.parametrize("schedule", ["flat", "balanced", "xcd-dynamic", "dynamic-16", "balanced+morton",
                                      "flat+morton"])
def test_plan_matches_single_multiplies(qt, schedule):
    probs = _problems()
    leaf = 128
    hs = [(qt.from_blockmatrix(A, leaf), qt.from_blockmatrix(B, leaf)) for A, B in probs]
    singles = [_blocks(qt.multiply(a, b), A, B) for (a, b), (A, B) in zip(hs, probs)]
    _say("plan", schedule, len(probs), "problems")
    plan = qt.Plan([a for a, _ in hs], [b for _, b in hs], "f64")
    plan.set_schedule(schedule)
    plan.execute(graph=False)
    for i, (A, B) in enumerate(probs):
        C = _blocks(plan.result(i), A, B)
        assert np.array_equal(positions(C), positions(singles[i]))
        assert np.array_equal(C.V, singles[i].V)          # bitwise: same kernel body, same order
        _check_against_oracle(C, A, B, leaf, 1e-12)
    inf = plan.info()
    assert inf["schedule"] == schedule
    assert inf["products"] == sum(oracle.product_count(A, B) for A, B in probs)
    plan.destroy()


def test_plan_graph_replays(qt):
    import torch
    probs = _problems(seed=1)
    hs = [(qt.from_blockmatrix(A, 64), qt.from_blockmatrix(B, 64)) for A, B in probs]
    plan = qt.Plan([a for a, _ in hs], [b for _, b in hs], "f64")
    plan.set_schedule("balanced")
    plan.execute(graph=False)
    eager = [_blocks(plan.result(i), A, B) for i, (A, B) in enumerate(probs)]
    other = qt.from_blockmatrix(probs[1][0], 64)
    for rep in range(4):
        _say("graph replay", rep)
        junk = qt.multiply(other, other)                  # unrelated GPU work between replays
        x = torch.ones(1 << 20, device="cuda")
        x.mul_(2.0)
        plan.execute(graph=True)
        torch.cuda.synchronize()
        for i, (A, B) in enumerate(probs):
            C = _blocks(plan.result(i), A, B)
            assert np.array_equal(C.V, eager[i].V), (rep, i)
        junk.free()
    # switching the schedule re-captures the graph
    plan.set_schedule("flat")
    plan.execute(graph=True)
    for i, (A, B) in enumerate(probs):
        assert np.array_equal(_blocks(plan.result(i), A, B).V, eager[i].V)
    plan.destroy()


def test_plan_execute_captured_by_the_caller(qt):
    """qt_plan_execute launches without allocating or synchronizing, so a
    caller can capture it into a graph of its own: the C_i are computed by
    the first replay (they were never computed before it), and every later
    replay, with other GPU work between, gives them bit for bit again; with
    a dynamic schedule the replays also re-run the counter reset (a replay
    that skipped the work would take no time)."""
    import torch
    probs = _problems(seed=2)
    hs = [(qt.from_blockmatrix(A, 64), qt.from_blockmatrix(B, 64)) for A, B in probs]
    plan = qt.Plan([a for a, _ in hs], [b for _, b in hs], "f64")
    plan.set_schedule("flat")
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        plan.execute(stream=s, graph=False)
    # computed only now, while the plan's C_i exist, so no C_i can hold them
    singles = [qt.multiply(a, b) for a, b in hs]
    ref = [_blocks(h, A, B) for h, (A, B) in zip(singles, probs)]
    other = qt.from_blockmatrix(probs[2][0], 64)
    for rep in range(4):
        _say("caller graph replay", rep)
        junk = qt.multiply(other, other)
        x = torch.ones(1 << 20, device="cuda")
        x.mul_(2.0)
        g.replay()
        torch.cuda.synchronize()
        for i, (A, B) in enumerate(probs):
            assert np.array_equal(_blocks(plan.result(i), A, B).V, ref[i].V), (rep, i)
        junk.free()
    del g
    # a dynamic schedule: warmed eagerly (its grid size is looked up once), then captured
    plan.set_schedule("xcd-dynamic")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(s):
        e0.record()
        plan.execute(stream=s, graph=False)
        e1.record()
    torch.cuda.synchronize()
    eager_ms = e0.elapsed_time(e1)
    g2 = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g2, stream=s):
        plan.execute(stream=s, graph=False)
    for rep in range(3):
        with torch.cuda.stream(s):
            e0.record()
            g2.replay()
            e1.record()
        torch.cuda.synchronize()
        _say("dynamic replay", rep, "ms", e0.elapsed_time(e1), "eager", eager_ms)
        assert e0.elapsed_time(e1) > 0.3 * eager_ms
        for i, (A, B) in enumerate(probs):
            assert np.array_equal(_blocks(plan.result(i), A, B).V, ref[i].V), (rep, i)
    del g2
    for h in singles:
        h.free()
    plan.destroy()


@pytest.mark.parametrize("prec,b", [("f32", 32), ("bf16x3", 32), ("f64", 64), ("bf16x3", 64), ("f64", 16)])
def test_plan_precisions_and_block_sizes(qt, prec, b):
    rng = np.random.default_rng(7)
    probs = [(random_pattern(rng, 20, 20, 0.15, b), random_pattern(rng, 20, 20, 0.15, b)),
             (random_pattern(rng, 9, 14, 0.3, b), random_pattern(rng, 14, 6, 0.3, b))]
    leaf = 2 * b
    hs = [(qt.from_blockmatrix(A, leaf), qt.from_blockmatrix(B, leaf)) for A, B in probs]
    singles = [_blocks(qt.multiply(a, bb, prec), A, B) for (a, bb), (A, B) in zip(hs, probs)]
    _say("plan", prec, "b", b)
    plan = qt.Plan([a for a, _ in hs], [bb for _, bb in hs], prec)
    sched, times = plan.tune(reps=2)
    assert sched in times and qt.plan_config(sched) == plan.info()["config"]
    assert len(times) >= 4 and all(t > 0 for t in times.values())
    if b == 64:   # the tile shape is among the choices
        assert "flat+wave-tiles" in times and "balanced+wave-tiles" in times
    plan.execute(graph=True)
    for i, (A, B) in enumerate(probs):
        C = _blocks(plan.result(i), A, B)
        assert np.array_equal(C.V, singles[i].V)
    plan.destroy()


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3"])
def test_plan_every_config_bitwise_at_b64(qt, prec):
    """At b = 64 every configuration (schedules, launch orders, LDS-shared or
    per-wave tiles) gives bitwise the single multiply's result, on problems
    with and without a launch order of their own."""
    rng = np.random.default_rng(8)
    b = 64
    probs = [(random_pattern(rng, 24, 24, 0.04, b), random_pattern(rng, 24, 24, 0.04, b)),   # ~1 product per C block
             (wl.decay3d(192, 12.0, 16, b, seed=11), wl.decay3d(192, 12.0, 16, b, seed=12)),
             (random_pattern(rng, 7, 11, 0.4, b), random_pattern(rng, 11, 5, 0.4, b))]
    hs = [(qt.from_blockmatrix(A, 2 * b), qt.from_blockmatrix(B, 2 * b)) for A, B in probs]
    singles = [_blocks(qt.multiply(a, bb, prec), A, B) for (a, bb), (A, B) in zip(hs, probs)]
    plan = qt.Plan([a for a, _ in hs], [bb for _, bb in hs], prec)
    for c in range(qt.PLAN_CONFIGS):
        name = qt.plan_config_name(c)
        _say("plan b=64", prec, name)
        plan.set_schedule(name)
        plan.execute(graph=(c % 2 == 0))
        for i, (A, B) in enumerate(probs):
            C = _blocks(plan.result(i), A, B)
            assert np.array_equal(positions(C), positions(singles[i])), (name, i)
            assert np.array_equal(C.V, singles[i].V), (name, i)
    plan.destroy()


def test_plan_results_outlive_handles_and_free_is_ignored(qt):
    probs = _problems(seed=2)[:2]
    hs = [(qt.from_blockmatrix(A, 64), qt.from_blockmatrix(B, 64)) for A, B in probs]
    plan = qt.Plan([a for a, _ in hs], [b for _, b in hs], "f64")
    plan.execute()
    r = plan.result(0)
    qt.lib.qt_free(r.handle)                              # owned by the plan: ignored
    C = _blocks(plan.result(0), *probs[0])
    _check_against_oracle(C, probs[0][0], probs[0][1], 64, 1e-12)
    with pytest.raises(qt.QtError):
        plan.result(5)
    plan.destroy()


def test_tune_leaf(qt):
    A = wl.decay3d(512, 16.0, 16, 32, seed=9)
    h = qt.from_blockmatrix(A, 32)
    best, times = qt.tune_leaf(h, h, "f64", reps=2)
    assert best in (32, 64, 128, 256) and set(times) == {32, 64, 128, 256}
    hb = qt.from_blockmatrix(A, best)
    C = _blocks(qt.multiply(hb, hb), A, A)
    _check_against_oracle(C, A, A, best, 1e-12)


def test_tuning_cache_file(qt, tmp_path):
    """The tuners' choices go to the cache file and come back from it: the
    first call times and stores, a repeat (also after re-reading the file)
    returns the stored choice without timing, and a plan is set to it."""
    path = str(tmp_path / "tune.txt")
    A = wl.decay3d(512, 16.0, 16, 32, seed=13)
    h = qt.from_blockmatrix(A, 64)
    qt.tune_cache(path)
    try:
        leaf, cached = qt.tune_leaf_cached(h, h, "decay n2^9 test", "f64", reps=1)
        assert not cached and leaf in (32, 64, 128, 256)
        text = open(path).read()
        assert "leaf decay n2^9 test" in text and ("\t%d\n" % leaf) in text
        assert qt.tune_leaf_cached(h, h, "decay n2^9 test", "f64", reps=1) == (leaf, True)
        qt.tune_cache(path)                                   # read the file again
        assert qt.tune_leaf_cached(h, h, "decay n2^9 test", "f64", reps=1) == (leaf, True)
        assert qt.tune_leaf_cached(h, h, "decay n2^9 test", "f32", reps=1)[1] is False   # another precision
        probs = _problems(seed=3)[:3]
        hs = [(qt.from_blockmatrix(a, 64), qt.from_blockmatrix(b, 64)) for a, b in probs]
        plan = qt.Plan([a for a, _ in hs], [b for _, b in hs], "f64")
        name, cached = plan.tune_cached("three problems", reps=1)
        assert not cached and plan.info()["schedule"] == name
        plan.set_schedule("dynamic-16" if name != "dynamic-16" else "flat")
        assert plan.tune_cached("three problems", reps=1) == (name, True)
        assert plan.info()["schedule"] == name                # set to the stored configuration
        plan.execute()
        for i, (a, b) in enumerate(probs):
            _check_against_oracle(_blocks(plan.result(i), a, b), a, b, 64, 1e-12)
        plan.destroy()
    finally:
        qt.tune_cache(None)
