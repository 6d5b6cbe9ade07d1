"""GPU parity at the benchmark workloads' full sizes, in the benchmark's launch
configuration (same leaf sizes, same entry points).

The CPU oracle cannot run the full quadtree multiply here in seconds, so:
  * the C block pattern is compared exactly with the boolean product of the
    block patterns (computed by sparse 0/1 products);
  * sampled C blocks are compared with C(I,J) = sum_K A(I,K) B(K,J) computed
    straight from the definition, relative to (|A||B|)(I,J) from the same
    definition on absolute values;
  * sampled absent positions must come back as absent.
For the 131072-dimension decay workload (C is 24 GB) the pattern is checked
through its exact block count and sampled present/absent positions.
"""
import numpy as np
import pytest

import oracle
import workloads as wl

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


def _ref_blocks(A, I, J):
    idx = oracle.make_index(A, A)
    absA = wl.BlockMatrix(A.n_rows, A.n_cols, A.b, A.I, A.J, np.abs(A.V))
    refs, absrefs, ks = [], [], []
    for i, j in zip(I, J):
        refs.append(oracle.block_by_definition(A, A, i, j, idx))
        absrefs.append(oracle.block_by_definition(absA, absA, i, j, idx))
        ks.append(len(set(idx[0].get(int(i), {})) & set(idx[1].get(int(j), {}))))
    return refs, absrefs, ks


def _sample_present_absent(pos_ref, nbc, nb_total, rng, n):
    pres = pos_ref[rng.choice(pos_ref.size, size=min(n, pos_ref.size), replace=False)]
    cand = rng.choice(nb_total, size=4 * n, replace=False)
    absent = np.setdiff1d(cand, pos_ref)[:n]
    return pres // nbc, pres % nbc, absent // nbc, absent % nbc


def _check_samples(C, dtype, I, J, refs, absrefs, ks, rel, abs_slack_per_term=0.0, b=32):
    V, F = C.get_blocks(I, J, dtype)
    assert F.all()
    worst = 0.0
    for t in range(len(I)):
        err = np.abs(V[t].astype(np.float64) - refs[t])
        bound = rel(ks[t]) * absrefs[t] + abs_slack_per_term * ks[t] * b
        assert np.all(err <= bound), (t, float((err - bound).max()))
        with np.errstate(divide="ignore", invalid="ignore"):
            r = np.where(absrefs[t] > 0, err / absrefs[t], 0.0)
        worst = max(worst, float(r.max()))
    return worst


def _full_case(qt, name, precs, n_samples=120):
    A = wl.config(name)
    leaf = wl.CONFIGS[name]["leaf"]
    _say(name, "nnz", A.nnz, "leaf", leaf)
    h = qt.from_blockmatrix(A, leaf)
    pos_ref = oracle.pattern_by_definition(A, A)
    rng = np.random.default_rng(123)
    Ip, Jp, Ia, Ja = _sample_present_absent(pos_ref, A.nb_cols, A.nb_rows * A.nb_cols, rng, n_samples)
    refs, absrefs, ks = _ref_blocks(A, Ip, Jp)
    out = {}
    for prec in precs:
        _say(name, prec)
        C = qt.multiply(h, h, prec)
        I, J = C.pattern()
        pos = I.astype(np.int64) * A.nb_cols + J
        assert np.array_equal(pos, pos_ref), "C block pattern differs from the boolean product"
        _, F = C.get_blocks(Ia, Ja)
        assert not F.any()
        b = A.b
        if prec == "f64":
            out[prec] = _check_samples(C, "f64", Ip, Jp, refs, absrefs, ks, lambda k: 1e-12, b=b)
        elif prec == "f32":
            out[prec] = _check_samples(C, "f32", Ip, Jp, refs, absrefs, ks,
                                       lambda k: (k * b + 2) * 2.0 ** -24, 4 * 2.0 ** -126, b)
        else:
            out[prec] = _check_samples(C, "f64", Ip, Jp, refs, absrefs, ks,
                                       lambda k: 3 * 2.0 ** -16 + (3 * b + 4) * 2.0 ** -24, 4 * 2.0 ** -126, b)
        C.free()
    _say(name, "worst componentwise errors", out)
    return out


def test_decay32768_full(qt):
    e = _full_case(qt, "decay32768", ["f64", "f32", "bf16x3"])
    assert e["f64"] <= 1e-12


def test_decay32768_every_block(qt):
    """The headline workload with every C block against the oracle's
    quadtree multiply (not a sample): FP64 componentwise within 1e-12 of
    (|A||B|)_ij; FP32 and BF16X3 within their a-priori bounds with k the
    largest number of block products of any C block."""
    import scipy.sparse as sp
    from tests._util import compare
    A = wl.config("decay32768")
    leaf = wl.CONFIGS["decay32768"]["leaf"]
    ref, _ = oracle.multiply(A, A, leaf)
    absAB, _ = oracle.multiply(A, A, leaf, use_abs=True)
    # block products of every C block: the 0/1 pattern product, in C's (I, J) order
    S = sp.csr_matrix((np.ones(A.nnz), (A.I, A.J)), shape=(A.nb_rows, A.nb_cols))
    k = np.asarray((S @ S)[ref.I, ref.J]).ravel()[:, None, None]
    h = qt.from_blockmatrix(A, leaf)
    b = A.b
    for prec in ("f64", "f32", "bf16x3"):
        _say("decay32768 every block", prec)
        C = qt.multiply(h, h, prec)
        I, J, V = C.to_blocks("f32" if prec == "f32" else "f64")
        got = wl.BlockMatrix(A.n_rows, A.n_cols, b, I, J, V.astype(np.float64))
        same, _, e_f, e_cw = compare(ref, got, absAB)
        assert same
        if prec == "f64":
            assert e_cw <= 1e-12 and e_f <= 1e-12, (e_cw, e_f)
        else:
            rel = (k * b + 2) * 2.0 ** -24 if prec == "f32" else 3 * 2.0 ** -16 + (3 * b + 4) * 2.0 ** -24
            err = np.abs(got.V - ref.V)
            assert np.all(err <= rel * absAB.V + 4 * 2.0 ** -126 * k * b), prec
        C.free()


def test_random65536_full(qt):
    e = _full_case(qt, "random65536", ["f64", "f32"])
    assert e["f64"] <= 1e-12


def test_banded1024_bench_config(qt):
    e = _full_case(qt, "banded1024", ["f64", "f32", "bf16x3"], n_samples=60)
    assert e["f64"] <= 1e-12


@pytest.mark.slow
def test_decay131072_sampled(qt):
    """b = 64, leaf 512: fp64, fp32 and split-bf16 paths; exact C block count."""
    name = "decay131072"
    A = wl.config(name)
    leaf = wl.CONFIGS[name]["leaf"]
    _say(name, "nnz", A.nnz)
    h = qt.from_blockmatrix(A, leaf)
    pos_ref = oracle.pattern_by_definition(A, A)
    rng = np.random.default_rng(321)
    Ip, Jp, Ia, Ja = _sample_present_absent(pos_ref, A.nb_cols, A.nb_rows * A.nb_cols, rng, 40)
    refs, absrefs, ks = _ref_blocks(A, Ip, Jp)
    b = A.b
    for prec in ("f64", "f32", "bf16x3"):
        _say(name, prec)
        C = qt.multiply(h, h, prec)
        assert C.nblocks == pos_ref.size
        _, F = C.get_blocks(Ia, Ja)
        assert not F.any()
        if prec == "f64":
            w = _check_samples(C, "f64", Ip, Jp, refs, absrefs, ks, lambda k: 1e-12, b=b)
            assert w <= 1e-12
        elif prec == "f32":
            _check_samples(C, "f32", Ip, Jp, refs, absrefs, ks, lambda k: (k * b + 2) * 2.0 ** -24,
                           4 * 2.0 ** -126, b)
        else:
            _check_samples(C, "f64", Ip, Jp, refs, absrefs, ks,
                           lambda k: 3 * 2.0 ** -16 + (3 * b + 4) * 2.0 ** -24, 4 * 2.0 ** -126, b)
        assert C.stats()["products"] == oracle.product_count(A, A)
        C.free()


def test_random65536_split_full(qt):
    e = _full_case(qt, "random65536", ["bf16x3"])
    assert e["bf16x3"] <= 3 * 2.0 ** -16 + (3 * 32 + 4) * 2.0 ** -24


@pytest.mark.slow
def test_batch64_full(qt):
    """The 64-problem batch at its full size in the benchmark's launch
    configuration (leaf size per pattern class from the tuner, the tuned
    schedule, graph replay, fp32): every plan result equals the single
    multiply bit for bit, its pattern equals the boolean product, and sampled
    blocks of every problem agree with the definition within the fp32 bound."""
    import math
    probs = wl.batch_mix(64, 5)
    b = probs[0][0].b
    cache, hs = {}, []
    for A, B in probs:
        fill = max(A.nnz, 1) / float(A.nb_rows * A.nb_cols)
        cls = (A.meta.get("pattern"), int(round(math.log2(A.nb_rows))), int(round(math.log2(fill * 1000))))
        if cls not in cache:
            cache[cls], _ = qt.tune_leaf(qt.from_blockmatrix(A, 8 * b), qt.from_blockmatrix(B, 8 * b), "f32", reps=1)
        hs.append((qt.from_blockmatrix(A, cache[cls]), qt.from_blockmatrix(B, cache[cls])))
    _say("batch64: leaves", sorted(set(cache.values())))
    plan = qt.Plan([a for a, _ in hs], [h for _, h in hs], "f32")
    sched, _ = plan.tune(reps=1)
    _say("batch64: schedule", sched)
    for _ in range(2):
        plan.execute(graph=True)
    rng = np.random.default_rng(55)
    for i, ((A, B), (ha, hb)) in enumerate(zip(probs, hs)):
        Cp = plan.result(i)
        Cs = qt.multiply(ha, hb, "f32")
        Ip, Jp, Vp = Cp.to_blocks("f32")
        Is, Js, Vs = Cs.to_blocks("f32")
        assert np.array_equal(Ip, Is) and np.array_equal(Jp, Js) and np.array_equal(Vp, Vs), i
        pos_ref = oracle.pattern_by_definition(A, B)
        assert np.array_equal(Ip.astype(np.int64) * B.nb_cols + Jp, pos_ref), i
        if len(Ip) == 0:
            continue
        idx = oracle.make_index(A, B)
        absA = wl.BlockMatrix(A.n_rows, A.n_cols, b, A.I, A.J, np.abs(A.V))
        absB = wl.BlockMatrix(B.n_rows, B.n_cols, b, B.I, B.J, np.abs(B.V))
        for t in rng.choice(len(Ip), size=min(3, len(Ip)), replace=False):
            ref = oracle.block_by_definition(A, B, Ip[t], Jp[t], idx)
            absref = oracle.block_by_definition(absA, absB, Ip[t], Jp[t], idx)
            k = len(set(idx[0].get(int(Ip[t]), {})) & set(idx[1].get(int(Jp[t]), {})))
            err = np.abs(Vp[t].astype(np.float64) - ref)
            assert np.all(err <= (k * b + 2) * 2.0 ** -24 * absref + 4 * 2.0 ** -126 * k * b), (i, t)
        Cs.free()
