#!/usr/bin/env python3
"""Benchmark of the quadtree block-sparse multiply C = A*A on one MI355X.

Workload (default): the 3D-decay matrix with 2048 atoms in a cube of side
40, 16 basis functions per atom (n = 32768), block size 32, blocks below
1e-10 dropped, leaf 256; inputs resident in HBM before timing. One step is
one full qt_multiply (symbolic traversal + numeric MFMA kernel + C
assembly), called back to back on one stream as an application would; the
library runs each traversal on its own stream, beside the previous step's
numeric kernel. The metric counts 2*b^3 flops per nonzero block product.
The latency of a lone call on an idle GPU is reported beside it.

Prints one JSON line with the fp64 path as the headline value, the
roofline of the numeric kernel (HIP events on the multiply's stream), the
fp32 and split-bf16 paths with their speedup and error against the CPU
oracle, and the oracle itself timed on the host cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "block-product TFLOP/s and MFMA-peak fraction, split vs FP64 path at stated error"
PEAK = {"f64": 78.6, "f32": 157.3, "bf16x3": 2516.6}   # dense MFMA TFLOP/s, MI355X
HBM_PEAK_GBS = 8000.0                                   # HBM3E, MI355X

# Error bounds each path must meet against the fp64 oracle, normwise (e_F =
# ||C - C_ref||_F / ||C_ref||_F) and by the largest entry error over max |C_ref|:
# fp64 is held to 1e-12; fp32 and the split-bf16 path to their a-priori bounds
# per block product (inputs rounded to fp32, products summed in fp32: about
# (k b + 2) 2^-24 for fp32 with k products per C block; 3 2^-16 + (b + 2) 2^-24
# for split bf16) with room for the longest product lists of the workloads.
TOLERANCE = {"f64": {"e_F": 1e-12, "e_max_rel": 1e-12},
             "f32": {"e_F": 1e-5, "e_max_rel": 1e-4},
             "bf16x3": {"e_F": 1e-4, "e_max_rel": 1e-3}}


def check_path(entry: dict, prec: str) -> list:
    """Failed checks of one path's result (pattern, then the error bounds)."""
    if entry.get("pattern_matches_oracle") is False:
        return [f"{prec}: C block pattern differs from the oracle"]
    bad = []
    for key, lim in TOLERANCE[prec].items():
        if key in entry and not entry[key] <= lim:
            bad.append(f"{prec}: {key} = {entry[key]:.3g} above {lim:g}")
    return bad


def cpu_model() -> str:
    """The host CPU's model name (first 'model name' line of /proc/cpuinfo)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def code_digest(*paths: str) -> str:
    """SHA-256 of C++/HIP sources with their comments and whitespace removed:
    it changes when the code changes, not when only a comment does."""
    import hashlib
    import re
    h = hashlib.sha256()
    for path in paths:
        text = open(path, encoding="utf-8").read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update("".join(text.split()).encode() + b"\0")
    return h.hexdigest()


# what a numeric kernel's HBM traffic depends on: the kernels, and the order
# in which the multiply launches C's blocks
TRAFFIC_SOURCES = tuple(os.path.join(ROOT, "paper_1501_07800_amd", "csrc", f)
                        for f in ("qt_numeric.hip", "qt_multiply.hip"))


def measured_traffic(workload: str, prec: str):
    """HBM bytes per launch of the numeric kernel from the committed rocprofv3
    counter summary (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy's
    reading), or None when there is none for this workload or the kernels'
    code or launch order has changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{prec}_{workload}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("code_sha256") != code_digest(*TRAFFIC_SOURCES):
        return None
    return rec.get("traffic_bytes")


COPY_BYTES = 1 << 31   # plain device copy used to calibrate the traffic counters
CPU_SAMPLE_FLOPS = 1.0e11   # block-product work the CPU oracle is given at most (a few s per run)
CPU_SAMPLE_FLOPS_1T = 8.0e9  # the same for the one-thread runs


def row_sample(wl, A, P, max_flops, name):
    """The C block rows 0 .. R-1 of C = A*A as the oracle's sample: A's first
    R block rows (times A), R the smallest that holds max_flops of block
    products, or all of A when the whole product is within max_flops.
    Returns (A's rows, their block products, R or None, description)."""
    import numpy as np
    b = A.b
    if 2.0 * b ** 3 * P <= max_flops:
        return A, P, None, f"the full {name} workload, C = A*A"
    rowcnt = np.bincount(A.I, minlength=A.nb_rows).astype(np.float64)
    p_row = np.bincount(A.I, weights=rowcnt[A.J], minlength=A.nb_rows)
    R = int(np.searchsorted(np.cumsum(p_row), max_flops / (2.0 * b ** 3))) + 1
    R = min(R, A.nb_rows)
    keep = A.I < R
    Ao = wl.BlockMatrix(A.n_rows, A.n_cols, b, A.I[keep], A.J[keep], A.V[keep])
    P_o = int(p_row[:R].sum())
    return Ao, P_o, R, (f"C block rows 0..{R - 1} of {A.nb_rows} of {name} (A's first {R} block rows "
                        f"times A: {P_o} of {P} block products)")


def calibrate_copy():
    """A plain device-to-device copy of COPY_BYTES, three times: the reading
    of FETCH_SIZE / WRITE_SIZE for it gives the counters' scale."""
    import torch
    x = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": COPY_BYTES, "copies": 3}), flush=True)


def roofline_bound(flops: float, alg_bytes: float, numeric_ms: float, peak_tflops: float) -> dict:
    """The numeric kernel's roofline: MFMA-bound when its arithmetic intensity
    over the algorithmic bytes is at least the ridge point (peak / HBM
    bandwidth), reported in TFLOP/s; else HBM-bound, reported in GB/s of
    algorithmic bytes against the HBM peak."""
    intensity = flops / alg_bytes
    ridge = peak_tflops * 1e12 / (HBM_PEAK_GBS * 1e9)
    tflops = flops / (numeric_ms * 1e-3) / 1e12
    if intensity >= ridge:
        roof = {"bound": "mfma", "achieved": tflops, "peak": peak_tflops, "unit": "TFLOP/s",
                "frac": tflops / peak_tflops}
    else:
        gbs = alg_bytes / (numeric_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                "achieved_tflops": tflops}
    roof.update({"algorithmic_bytes": alg_bytes, "arithmetic_intensity": intensity, "ridge": ridge})
    return roof


def _pmc_mean_kib(csv_path, counter, name_part):
    import csv
    vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(csv_path))
            if r["Counter_Name"] == counter and name_part in r["Kernel_Name"]]
    if not vals:
        raise SystemExit(f"no {counter} rows for kernels matching {name_part!r} in {csv_path}")
    return sum(vals) / len(vals), len(vals)


def _has_rows(csv_path, counter, name_part):
    import csv
    return any(r["Counter_Name"] == counter and name_part in r["Kernel_Name"] for r in csv.DictReader(open(csv_path)))


def traffic_from_counters(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, workload, prec, b, out_dir=None):
    """Writes profiles/traffic_<prec>_<workload>.json: HBM-side bytes per
    launch of the numeric kernel from rocprofv3 --pmc FETCH_SIZE and
    WRITE_SIZE (KiB per dispatch), each scaled so that the plain copy of
    COPY_BYTES reads as COPY_BYTES."""
    if b == 64:   # the LDS-shared kernels of the 64-wide blocks
        kname = {"f64": "k_numeric_f64_b64", "f32": "k_numeric_f32_b64", "bf16x3": "k_numeric_bf16x3_b64"}[prec]
    else:
        kname = {"f64": f"k_numeric<double, {b}>", "f32": f"k_numeric<float, {b}>",
                 "bf16x3": f"k_numeric_bf16x3<{b}>"}[prec]
        # C blocks launched grouped by inner index run in the by-k kernel
        byk = kname.replace("k_numeric<", "k_numeric_byk<")
        if byk != kname and _has_rows(fetch_csv, "FETCH_SIZE", byk):
            kname = byk
    cf, _ = _pmc_mean_kib(copy_fetch_csv, "FETCH_SIZE", "copyBuffer")
    cw, _ = _pmc_mean_kib(copy_write_csv, "WRITE_SIZE", "copyBuffer")
    f_scale = COPY_BYTES / (cf * 1024.0)
    w_scale = COPY_BYTES / (cw * 1024.0)
    kf, nf = _pmc_mean_kib(fetch_csv, "FETCH_SIZE", kname)
    kw, nw = _pmc_mean_kib(write_csv, "WRITE_SIZE", kname)
    fetch = kf * 1024.0 * f_scale
    write = kw * 1024.0 * w_scale
    rec = {"kernel": kname, "workload": workload, "prec": prec,
           "fetch_kib_per_dispatch": kf, "write_kib_per_dispatch": kw, "dispatches": [nf, nw],
           "copy_fetch_kib": cf, "copy_write_kib": cw, "fetch_scale": f_scale, "write_scale": w_scale,
           "fetch_bytes": fetch, "write_bytes": write, "traffic_bytes": fetch + write,
           "code_sha256": code_digest(*TRAFFIC_SOURCES)}
    out = os.path.join(out_dir or os.path.join(ROOT, "profiles"), f"traffic_{prec}_{workload}.json")
    json.dump(rec, open(out, "w"), indent=1)
    print(json.dumps(rec), flush=True)
    return rec


def timed_steps(qt, torch, hA, prec, steps, warmup):
    for _ in range(warmup):
        qt.multiply(hA, hA, prec).free()
    torch.cuda.synchronize()
    qt.profile(True)
    t0 = time.perf_counter()
    last = None
    for i in range(steps):
        if last is not None:
            last.free()
        last = qt.multiply(hA, hA, prec)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = qt.profile_read()
    qt.profile(False)
    return (t1 - t0), prof, last


def _time_call(torch, fn, reps):
    """Mean wall time (ms) of fn() over reps back-to-back calls, device-
    synchronized; each result is freed just before the next call (as in the
    headline loop)."""
    r = fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        if hasattr(r, "free"):
            r.free()
        r = fn()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps * 1e3
    if hasattr(r, "free"):
        r.free()
    return dt


def bench_ops(args, qt, torch, wl):
    """The operations beside C = A*B on the decay workload, one JSON line:
    transposed products (op(A) op(B)), the symmetric square with upper-
    triangular storage against the full square of the same symmetric matrix,
    C = A + B, and value-aware truncation. TFLOP/s count 2b^3 per block
    product as everywhere; add and truncate are reported in GB/s of block
    data read and written once."""
    import numpy as np
    cfg = wl.CONFIGS[args.workload]
    leaf = args.leaf or cfg["leaf"]
    A = wl.config(args.workload)
    b = A.b
    reps = max(3, args.steps // 2)
    hA = qt.from_blockmatrix(A, leaf)
    qt.prepare(hA, "f64")
    out = {}

    def prod_tf(C, ms):
        P = C.stats()["products"]
        return P, 2.0 * b ** 3 * P / (ms * 1e-3) / 1e12

    for name, ta, tb in (("A*A", False, False), ("A^T*A", True, False), ("A*A^T", False, True),
                         ("A^T*A^T", True, True)):
        ms = _time_call(torch, lambda: qt.multiply_ex(hA, hA, ta, tb, prec="f64"), reps)
        C = qt.multiply_ex(hA, hA, ta, tb, prec="f64")
        P, tf = prod_tf(C, ms)
        out[name] = {"ms": ms, "products": P, "tflops": tf, "nnz_C": C.nblocks}
        C.free()
        log(f"bench: {name}: {ms:.3f} ms, {tf:.2f} TFLOP/s")

    # symmetric S from A's upper block triangle (strictly upper blocks mirrored, transposed)
    up = A.I <= A.J
    st = A.I < A.J
    UI, UJ, UV = A.I[up], A.J[up], A.V[up]
    U = wl.BlockMatrix(A.n_rows, A.n_cols, b, UI, UJ, np.ascontiguousarray(UV))
    SI = np.concatenate([A.I[up], A.J[st]])
    SJ = np.concatenate([A.J[up], A.I[st]])
    SV = np.concatenate([A.V[up], A.V[st].transpose(0, 2, 1)])
    S = wl.BlockMatrix(A.n_rows, A.n_cols, b, SI, SJ, np.ascontiguousarray(SV))
    hU = qt.from_blockmatrix(U, leaf)
    hS = qt.from_blockmatrix(S, leaf)
    qt.prepare(hS, "f64")
    ms_full = _time_call(torch, lambda: qt.multiply(hS, hS, "f64"), reps)
    C = qt.multiply(hS, hS, "f64")
    P_full, tf_full = prod_tf(C, ms_full)
    C.free()
    ms_sq = _time_call(torch, lambda: qt.sysq(hU, "f64"), reps)
    C = qt.sysq(hU, "f64")
    P_sq, tf_sq = prod_tf(C, ms_sq)
    out["sysq"] = {"ms": ms_sq, "products": P_sq, "tflops": tf_sq, "nnz_C": C.nblocks,
                   "full_square_ms": ms_full, "full_square_products": P_full,
                   "products_ratio": P_sq / P_full, "speedup_vs_full": ms_full / ms_sq}
    log(f"bench: sysq: {ms_sq:.3f} ms ({P_sq} products) vs full S*S {ms_full:.3f} ms ({P_full})")

    # C = A + S (union of two different patterns)
    ms_add = _time_call(torch, lambda: qt.add(hA, hS), reps)
    C = qt.add(hA, hS)
    moved = (A.nnz + S.nnz + C.nblocks) * b * b * 8
    out["add"] = {"ms": ms_add, "nnz_A": A.nnz, "nnz_B": S.nnz, "nnz_C": C.nblocks,
                  "bytes": moved, "GB_per_s": moved / (ms_add * 1e-3) / 1e9}
    log(f"bench: add: {ms_add:.3f} ms, {out['add']['GB_per_s']:.0f} GB/s")

    # truncation of C = A*A at eps = 1e-6 ||C||_F
    C = qt.multiply(hA, hA, "f64")
    I, J, V = C.to_blocks("f64")
    eps = 1e-6 * float(np.linalg.norm(V))
    del I, J, V
    ms_tr = _time_call(torch, lambda: qt.truncate(C, eps)[0], reps)
    T, removed, e2 = qt.truncate(C, eps)
    moved = (C.nblocks + T.nblocks) * b * b * 8
    out["truncate"] = {"ms": ms_tr, "eps": eps, "nnz_in": C.nblocks, "nnz_out": T.nblocks, "removed": removed,
                       "removed_norm": float(np.sqrt(e2)), "bytes": moved,
                       "GB_per_s": moved / (ms_tr * 1e-3) / 1e9}
    log(f"bench: truncate: {ms_tr:.3f} ms, removed {removed} of {C.nblocks} blocks")
    T.free()
    C.free()
    print(json.dumps({"metric": METRIC, "workload": args.workload, "n": A.n_rows, "b": b, "leaf": leaf,
                      "dtype": "f64", "data": "synthetic", "reps": reps, "ops": out}), flush=True)


def bench_rmat(args, qt, torch, wl):
    """R-MAT locality sweep (Sec. 5.1, Fig. 4): C = A*A on an 8192 x 8192 block
    grid with 5 blocks per row, quadrant weight a from 0.25 (uniformly random)
    to 0.9; the multiply pairs per quadtree level (the task counts C_l) and
    the end-to-end rate at each a."""
    b, leaf = 16, 128
    rows = []
    for a in (0.25, 0.4, 0.55, 0.7, 0.8, 0.9):
        A = wl.rmat(13, 5, a, b, seed=7)
        h = qt.from_blockmatrix(A, leaf)
        qt.prepare(h, "f64")
        ms = _time_call(torch, lambda: qt.multiply(h, h, "f64"), max(3, args.steps // 4))
        C = qt.multiply(h, h, "f64")
        stt = C.stats()
        rows.append({"a": a, "nnz_A": A.nnz, "nnz_C": C.nblocks, "products": stt["products"],
                     "pairs_per_level": [int(x) for x in stt["pairs"]], "ms": ms,
                     "tflops": 2.0 * b ** 3 * stt["products"] / (ms * 1e-3) / 1e12})
        log(f"bench: rmat a={a}: {ms:.3f} ms, pairs {[int(x) for x in stt['pairs']]}")
        C.free()
        h.free()
    print(json.dumps({"metric": METRIC, "workload": "rmat8192x5", "b": b, "leaf": leaf, "dtype": "f64",
                      "data": "synthetic", "sweep": rows}), flush=True)


def bench_batch(args, qt, torch, wl):
    """The batch64 workload as the line's main result."""
    print(json.dumps(batch_result(args, qt, torch, wl)), flush=True)


def batch_result(args, qt, torch, wl):
    """64 independent C = A*B (uneven size, fill and pattern) in one launch.

    Leaf size per pattern class from the leaf tuner; the plan's schedule from
    the plan tuner; the timed step is one graph replay of the whole batch's
    numeric phase. Baseline: the same 64 products as 64 qt_multiply calls.
    """
    import math
    prec = args.prec if args.prec != "f64" or args.batch_prec_explicit else "f32"
    log("bench: generating the 64-problem batch (seed 5)")
    probs = wl.batch_mix(64, 5)
    b = probs[0][0].b
    # the leaf tuner's choices per pattern class go through the tuning cache file
    cache_path = os.environ.get("QT_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "qt", "tune.txt"))
    os.makedirs(os.path.dirname(cache_path), exist_ok=True)
    qt.tune_cache(cache_path)
    cache = {}
    hits = 0
    hs = []
    t_tune = time.perf_counter()
    for A, B in probs:
        fill = max(A.nnz, 1) / float(A.nb_rows * A.nb_cols)
        cls = (A.meta.get("pattern"), int(round(math.log2(A.nb_rows))), int(round(math.log2(fill * 1000))))
        if cls not in cache:
            ha, hb = qt.from_blockmatrix(A, 8 * b), qt.from_blockmatrix(B, 8 * b)
            cache[cls], cached = qt.tune_leaf_cached(ha, hb, f"{cls[0]} nb2^{cls[1]} fill2^{cls[2]}/1000", prec,
                                                     reps=2)
            hits += int(cached)
            del ha, hb
        leaf = cache[cls]
        ha, hb = qt.from_blockmatrix(A, leaf), qt.from_blockmatrix(B, leaf)
        qt.prepare(ha, prec)
        qt.prepare(hb, prec)
        hs.append((ha, hb))
    torch.cuda.synchronize()
    t_tune = time.perf_counter() - t_tune
    log(f"bench: {len(cache)} pattern classes tuned; leaves {sorted(set(cache.values()))}")

    # baseline: 64 sequential multiplies, timed as a caller runs them (no
    # per-phase events); their numeric kernels' time from a second, profiled pass
    for ha, hb in hs:
        qt.multiply(ha, hb, prec).free()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for ha, hb in hs:
            qt.multiply(ha, hb, prec).free()
    torch.cuda.synchronize()
    t_seq = (time.perf_counter() - t0) / args.steps
    qt.profile(True)
    for ha, hb in hs:
        qt.multiply(ha, hb, prec).free()
    torch.cuda.synchronize()
    prof = qt.profile_read()
    qt.profile(False)
    seq_numeric_ms = prof["numeric_ms"]
    P = prof["products"]
    flops = 2.0 * b ** 3 * P

    t0 = time.perf_counter()
    plan = qt.Plan([a for a, _ in hs], [bb for _, bb in hs], prec)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    sched, sched_ms = plan.tune(reps=3)   # every configuration, for the record
    log("bench: plan configurations (ms): " + ", ".join(f"{k} {v:.3f}" for k, v in sched_ms.items()))
    for _ in range(args.warmup):
        plan.execute(graph=True)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        plan.execute(graph=True)
    e1.record()
    torch.cuda.synchronize()
    t_exec = (time.perf_counter() - t0) / args.steps
    exec_ms = e0.elapsed_time(e1) / args.steps
    assert plan.info()["products"] == P
    value = flops / (exec_ms * 1e-3) / 1e12
    peak = PEAK["f32"] if prec in ("f32", "bf16x3") else PEAK["f64"]
    log(f"bench: batch {prec}: plan {value:.2f} TFLOP/s ({exec_ms:.3f} ms, schedule {sched}); "
        f"64 sequential multiplies {flops / t_seq / 1e12:.2f} TFLOP/s end to end ({t_seq * 1e3:.3f} ms), "
        f"numeric only {flops / (seq_numeric_ms * 1e-3) / 1e12:.2f} TFLOP/s")
    out = {
        "metric": METRIC, "value": value, "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": exec_ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": prec, "data": "synthetic",
        "config": {"workload": "batch64", "problems": len(probs), "b": b, "block_products": P, "prec": prec,
                   "op": "C_i = A_i*B_i, i = 1..64", "leaf_by_class": {str(k): v for k, v in cache.items()}},
        "mfma_peak_frac": value / peak,
        "plan": {"schedule": sched, "schedule_ms": sched_ms, "create_s": t_plan, "tune_s": t_tune,
                 "host_ms_per_step": t_exec * 1e3, "flat_ms": sched_ms.get("flat"),
                 "best_persistent": min(((k, v) for k, v in sched_ms.items() if not k.startswith("flat")),
                                        key=lambda kv: kv[1], default=None),
                 "tuning_cache": {"path": cache_path, "leaf_classes": len(cache), "hits": hits}},
        "sequential": {"tflops_end_to_end": flops / t_seq / 1e12, "ms_per_step": t_seq * 1e3,
                       "numeric_ms_sum": seq_numeric_ms,
                       "numeric_tflops": flops / (seq_numeric_ms * 1e-3) / 1e12},
        "speedup_vs_sequential": t_seq * 1e3 / exec_ms,
    }
    plan.destroy()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="decay32768")
    ap.add_argument("--leaf", type=int, default=0, help="leaf size (0: the workload's default)")
    ap.add_argument("--prec", default="f64", choices=["f64", "f32", "bf16x3"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-paths", action="store_true", help="time only --prec")
    ap.add_argument("--no-hbm-config", action="store_true",
                    help="leave out the random65536 fp64/fp32 entry of the default run")
    ap.add_argument("--no-large-configs", action="store_true",
                    help="leave out the decay131072 and batch64 entries of the default run")
    ap.add_argument("--ops", action="store_true",
                    help="time the other operations (transposes, symmetric square, add, truncate) on --workload")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run the plain copy that calibrates the traffic counters")
    ap.add_argument("--traffic-from", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV"),
                    help="write the numeric kernel's measured traffic for --workload/--prec from rocprofv3 "
                         "counter_collection.csv files (no GPU needed)")
    args = ap.parse_args()
    if args.traffic_from:
        import workloads as wl
        return traffic_from_counters(*args.traffic_from, args.workload, args.prec, wl.CONFIGS[args.workload]["b"])
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the multiply has no multi-GPU path; --gpus takes 1.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import workloads as wl

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        return calibrate_copy()
    import paper_1501_07800_amd as qt

    if args.workload == "rmat":
        return bench_rmat(args, qt, torch, wl)
    if args.ops:
        return bench_ops(args, qt, torch, wl)
    if args.workload == "batch64":
        args.batch_prec_explicit = "--prec" in sys.argv
        return bench_batch(args, qt, torch, wl)
    cfg = wl.CONFIGS[args.workload]
    leaf = args.leaf or cfg["leaf"]
    log(f"bench: generating {args.workload}")
    A = wl.config(args.workload)
    b = A.b
    log(f"bench: n={A.n_rows} b={b} nnz(A)={A.nnz}; building on the GPU (leaf {leaf})")
    hA = qt.from_blockmatrix(A, leaf)
    # the one-time operand forms of each path (fp32 copy, bf16 hi/lo split, and
    # the block-transposed bf16 B), timed on the handle: the "cold" cost a first
    # multiply at that precision pays on top of the warm step
    prepare_ms = {}
    for p in ("f64", "f32", "bf16x3"):
        if p == "bf16x3" and b == 16:
            continue
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        qt.prepare(hA, p)
        torch.cuda.synchronize()
        prepare_ms[p] = (time.perf_counter() - t0) * 1e3
    torch.cuda.synchronize()

    # the rate a register-only loop of the same MFMA instruction reaches on this GPU; run first, it also
    # brings the clocks up after the idle time of input generation
    probe = qt.probe_mfma(args.prec)
    log(f"bench: MFMA probe ({args.prec} instruction, no memory traffic): {probe:.1f} TFLOP/s")

    precs = [args.prec] if args.no_paths else [args.prec] + [p for p in ("f64", "f32", "bf16x3") if p != args.prec]
    results = {}
    for prec in precs:
        if prec == "bf16x3" and b == 16:
            continue
        log(f"bench: {prec}: {args.warmup} warmup + {args.steps} timed steps")
        dt, prof, C = timed_steps(qt, torch, hA, prec, args.steps, args.warmup)
        P = C.stats()["products"]
        flops = 2.0 * b ** 3 * P
        tflops = flops * args.steps / dt / 1e12
        num_ms = prof["numeric_ms"] / max(prof["calls"], 1)
        span_ms = prof["symbolic_ms"] / max(prof["calls"], 1)
        # one multiply on an idle GPU: the traversal's own time, and the latency of a lone call
        single = []
        sym_alone = []
        for _ in range(5):
            torch.cuda.synchronize()
            qt.profile(True)
            t0 = time.perf_counter()
            qt.multiply(hA, hA, prec).free()
            torch.cuda.synchronize()
            single.append((time.perf_counter() - t0) * 1e3)
            pr = qt.profile_read()
            qt.profile(False)
            sym_alone.append(pr["symbolic_ms"])
        single_ms, sym_ms = float(np.median(single)), float(np.median(sym_alone))
        results[prec] = {"C": C, "P": P, "tflops": tflops, "ms_per_step": dt / args.steps * 1e3,
                         "numeric_ms": num_ms, "symbolic_ms": sym_ms, "symbolic_span_in_loop_ms": span_ms,
                         "single_call_ms": single_ms,
                         "numeric_tflops": flops / (num_ms * 1e-3) / 1e12, "nnz_C": C.nblocks}
        log(f"bench: {prec}: {tflops:.2f} TFLOP/s end to end, numeric {num_ms:.3f} ms, symbolic {sym_ms:.3f} ms "
            f"alone ({span_ms:.3f} ms span beside the previous numeric kernel), lone call {single_ms:.3f} ms")

    # the same multiply with the boundary's host buffers included: build from
    # host block lists (PCIe in), multiply, copy C back to host (PCIe out)
    pcie_ms = None
    if not args.no_paths:
        reps_h = 3
        t0 = time.perf_counter()
        for _ in range(reps_h):
            h = qt.from_blockmatrix(A, leaf)
            Ch = qt.multiply(h, h, args.prec)
            Ch.to_blocks("f32" if args.prec == "f32" else "f64")
            Ch.free()
            h.free()
        torch.cuda.synchronize()
        pcie_ms = (time.perf_counter() - t0) / reps_h * 1e3
        log(f"bench: {args.prec} host to host (build from host arrays + multiply + C to host): {pcie_ms:.1f} ms")

    main_r = results[args.prec]
    P = main_r["P"]
    flops = 2.0 * b ** 3 * P
    esz = 4 if args.prec == "f32" else 8
    # algorithmic HBM bytes of one numeric launch: A's values read once (C = A*A)
    # and C written once
    alg_bytes = A.nnz * b * b * esz + main_r["nnz_C"] * b * b * (4 if args.prec == "f32" else 8)

    cpu = None
    ref = None
    sample_rows = None
    if not args.no_cpu_baseline:
        import oracle
        # the whole workload when the oracle finishes it in seconds, else the
        # C block rows 0 .. R-1 (A's first R block rows times A)
        Ao, P_o, sample_rows, what = row_sample(wl, A, P, CPU_SAMPLE_FLOPS, args.workload)
        log(f"bench: CPU oracle (fp64, OpenMP) on {what}, 3 runs")
        secs = []
        for _ in range(3):
            t0 = time.perf_counter()
            ref, st = oracle.multiply(Ao, A, leaf)
            secs.append(time.perf_counter() - t0)
            assert st.block_products == P_o
        med = float(np.median(secs))
        cpu = {"value": 2.0 * b ** 3 * P_o / med / 1e12, "unit": "TFLOP/s", "cores": oracle.threads(),
               "kind": "oracle", "seconds": med, "runs_s": secs, "statistic": "median of 3 runs",
               "sample": what, "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}
        log(f"bench: oracle {med:.2f} s (median of 3) on {cpu['cores']} threads")
        # one thread, on a smaller row sample (the same rows from the top)
        A1, P_1, _, what1 = row_sample(wl, A, P, CPU_SAMPLE_FLOPS_1T, args.workload)
        secs1 = []
        for _ in range(3):
            t0 = time.perf_counter()
            _, st1 = oracle.multiply(A1, A, leaf, threads=1)
            secs1.append(time.perf_counter() - t0)
            assert st1.block_products == P_1
        oracle.multiply(A1, A1, leaf, threads=cpu["cores"])   # back to the full thread count
        med1 = float(np.median(secs1))
        cpu["one_thread"] = {"value": 2.0 * b ** 3 * P_1 / med1 / 1e12, "unit": "TFLOP/s", "cores": 1,
                             "seconds": med1, "runs_s": secs1, "statistic": "median of 3 runs", "sample": what1}
        log(f"bench: oracle on one thread: {med1:.2f} s (median of 3) for {P_1} block products")

    paths = {}
    for prec, r in results.items():
        entry = {"tflops": r["tflops"], "ms_per_step": r["ms_per_step"], "numeric_ms": r["numeric_ms"],
                 "symbolic_ms": r["symbolic_ms"], "symbolic_span_in_loop_ms": r["symbolic_span_in_loop_ms"],
                 "single_call_ms": r["single_call_ms"], "numeric_tflops": r["numeric_tflops"],
                 "prepare_ms": prepare_ms.get(prec),
                 "mfma_peak_frac": r["numeric_tflops"] / (PEAK["f32"] if prec == "bf16x3" else PEAK[prec]),
                 "speedup_vs_f64": (r["tflops"] / results["f64"]["tflops"]) if "f64" in results else None}
        if ref is not None:
            if sample_rows is None:
                I, J, V = r["C"].to_blocks("f64")
            else:
                # C's pattern in the sampled rows, then those blocks' values
                I, J = r["C"].pattern()
                sel = I < sample_rows
                I, J = I[sel], J[sel]
                V, F = r["C"].get_blocks(I, J, "f64")
                assert F.all()
            if not (np.array_equal(I, ref.I) and np.array_equal(J, ref.J)):
                entry["pattern_matches_oracle"] = False
            else:
                d = V - ref.V
                entry["pattern_matches_oracle"] = True
                entry["e_max"] = float(np.abs(d).max())
                entry["e_max_rel"] = float(np.abs(d).max() / np.abs(ref.V).max())
                entry["e_F"] = float(np.linalg.norm(d) / np.linalg.norm(ref.V))
                if sample_rows is not None:
                    entry["error_sample"] = f"C block rows 0..{sample_rows - 1}"
        if prec == "bf16x3":
            entry["mfma_utilisation"] = 3 * r["numeric_tflops"] / PEAK["bf16x3"]
        # operand bytes the kernel loads per launch (every block product's two
        # operand blocks; hi and lo parts for the split path), over its time:
        # the feed from L2 into the CUs
        op_bytes = r["P"] * 2 * b * b * {"f64": 8, "f32": 4, "bf16x3": 4}[prec]
        entry["operand_feed_gbs"] = op_bytes / (r["numeric_ms"] * 1e-3) / 1e9
        entry["traffic_bytes"] = measured_traffic(args.workload, prec)
        paths[prec] = entry

    failed = [msg for prec, e in paths.items() for msg in check_path(e, prec)]

    # the HBM-bound configuration (uniformly random blocks, 1 % fill) beside
    # the headline: fp64 and fp32, each against the HBM roofline
    hbm = None
    if not args.no_paths and not args.no_hbm_config and args.workload != "random65536":
        hbm = hbm_config_entry(qt, torch, wl, "random65536", args.steps, args.warmup)
        failed += [msg for prec, e in hbm["paths"].items() for msg in check_path(e, prec)]

    # the b = 64 decay workload (LDS-shared kernels) and the 64-problem batch,
    # so that their figures come from the same run
    large = batch = None
    if not args.no_paths and not args.no_large_configs and args.workload == "decay32768":
        large = large_config_entry(qt, torch, wl, "decay131072", max(5, args.steps // 2), max(3, args.warmup // 4))
        failed += [msg for prec, e in large["paths"].items() for msg in check_path(e, prec)]
        bargs = argparse.Namespace(**vars(args))
        bargs.prec, bargs.batch_prec_explicit = "f32", True
        bargs.steps, bargs.warmup = max(5, args.steps // 2), 3
        batch = batch_result(bargs, qt, torch, wl)

    # the batched block GEMM's practical peak, shaped like the paper's Table 2
    # (64000 uniform b x b products, one operand pair reused)
    practical = None
    if not args.no_paths:
        practical = {"count": 64000, "what": "64000 products C_i = A B of b x b blocks through the numeric "
                                              "kernels, A and B the same for all (TFLOP/s)"}
        for prec in ("f64", "f32", "bf16x3"):
            practical[prec] = {str(bs): qt.probe_batched(prec, bs, 64000) for bs in (16, 32, 64)
                               if not (prec == "bf16x3" and bs == 16)}
        log(f"bench: practical peak (TFLOP/s): {practical}")

    peak = PEAK[args.prec] if args.prec != "bf16x3" else PEAK["f32"]
    roof = roofline_bound(flops, alg_bytes, main_r["numeric_ms"], peak)
    roof.update({"traffic": measured_traffic(args.workload, args.prec),
                 "kernel": "k_numeric (block GEMM per C block)",
                 "probe_tflops": probe,
                 "frac_of_probe": main_r["numeric_tflops"] / (probe if args.prec != "bf16x3" else probe / 3.0)})
    out = {
        "metric": METRIC,
        "value": main_r["tflops"],
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": args.workload, "n": A.n_rows, "b": b, "leaf": leaf, "nnz_A": A.nnz,
                   "block_products": P, "nnz_C": main_r["nnz_C"], "prec": args.prec, "op": "C = A*A"},
        "mfma_peak_frac": main_r["tflops"] / peak,
        "roofline": roof,
        "cpu_baseline": cpu,
        "host_to_host": None if pcie_ms is None else {
            "ms": pcie_ms, "tflops": flops / (pcie_ms * 1e-3) / 1e12,
            "what": "qt_build from host block lists + qt_multiply + qt_to_blocks to host (PCIe both ways)"},
        "paths": paths,
        "hbm_config": hbm,
        "large_config": large,
        "batch": batch,
        "practical_peak": practical,
        "checks": {"tolerance": TOLERANCE, "failed": failed,
                   "what": "C block pattern equal to the oracle's; errors against the fp64 oracle within "
                           "the tolerance of each path"},
    }
    if failed:
        # a result that fails its check is no measurement: no value, non-zero exit
        out["value"] = None
        print(json.dumps(out), flush=True)
        log("bench: CHECK FAILED: " + "; ".join(failed))
        sys.exit(1)
    print(json.dumps(out), flush=True)


def hbm_config_entry(qt, torch, wl, name, steps, warmup, samples=64):
    """Timed fp64 and fp32 multiplies of workload `name` (C = A*A), each with
    its numeric kernel against the HBM roofline (A read once, C written once),
    its C pattern checked against the boolean product of A's block pattern and
    `samples` C blocks against the definition C(I,J) = sum_K A(I,K) A(K,J)."""
    import numpy as np
    import oracle
    cfg = wl.CONFIGS[name]
    log(f"bench: generating {name}")
    A = wl.config(name)
    b, leaf = A.b, cfg["leaf"]
    hA = qt.from_blockmatrix(A, leaf)
    ref_pos = oracle.pattern_by_definition(A, A)
    rng = np.random.default_rng(11)
    pick = np.sort(rng.choice(len(ref_pos), size=min(samples, len(ref_pos)), replace=False))
    sI = (ref_pos[pick] // A.nb_cols).astype(np.int32)
    sJ = (ref_pos[pick] % A.nb_cols).astype(np.int32)
    index = oracle.make_index(A, A)
    sref = np.stack([oracle.block_by_definition(A, A, i, j, index) for i, j in zip(sI, sJ)])
    paths = {}
    for prec in ("f64", "f32"):
        qt.prepare(hA, prec)
        log(f"bench: {name} {prec}: {warmup} warmup + {steps} timed steps")
        dt, prof, C = timed_steps(qt, torch, hA, prec, steps, warmup)
        P = C.stats()["products"]
        flops = 2.0 * b ** 3 * P
        num_ms = prof["numeric_ms"] / max(prof["calls"], 1)
        esz = 4 if prec == "f32" else 8
        alg = (A.nnz + C.nblocks) * b * b * esz
        I, J = C.pattern()
        pos = I.astype(np.int64) * A.nb_cols + J
        entry = {"tflops": flops * steps / dt / 1e12, "ms_per_step": dt / steps * 1e3, "numeric_ms": num_ms,
                 "numeric_tflops": flops / (num_ms * 1e-3) / 1e12, "block_products": P, "nnz_C": C.nblocks,
                 "roofline": roofline_bound(flops, alg, num_ms, PEAK[prec]),
                 "pattern_matches_oracle": bool(np.array_equal(pos, ref_pos))}
        if entry["pattern_matches_oracle"]:
            V, F = C.get_blocks(sI, sJ, "f64")
            d = V - sref
            entry["e_max"] = float(np.abs(d).max())
            entry["e_max_rel"] = float(np.abs(d).max() / np.abs(sref).max())
            entry["e_F"] = float(np.linalg.norm(d) / np.linalg.norm(sref))
            entry["error_sample"] = f"{len(sI)} C blocks drawn uniformly, against the definition"
        entry["roofline"]["traffic"] = measured_traffic(name, prec)
        C.free()
        log(f"bench: {name} {prec}: {entry['tflops']:.2f} TFLOP/s end to end, numeric {num_ms:.3f} ms = "
            f"{entry['roofline']['achieved']:.0f} {entry['roofline']['unit']} ({entry['roofline']['frac']:.2f} "
            f"of the {entry['roofline']['bound']} roof)")
        paths[prec] = entry
    paths["f32"]["speedup_vs_f64"] = paths["f32"]["tflops"] / paths["f64"]["tflops"]
    hA.free()
    return {"workload": name, "n": A.n_rows, "b": b, "leaf": leaf, "nnz_A": A.nnz, "op": "C = A*A",
            "paths": paths}


def large_config_entry(qt, torch, wl, name, steps, warmup, samples=64):
    """Timed FP64, FP32 and BF16X3 multiplies of workload `name` (C = A*A),
    each numeric kernel against its MFMA roofline; the C pattern compared
    whole with the boolean product of A's block pattern, `samples` C blocks
    with the definition C(I,J) = sum_K A(I,K) A(K,J)."""
    import numpy as np
    import oracle
    cfg = wl.CONFIGS[name]
    log(f"bench: generating {name}")
    A = wl.config(name)
    b, leaf = A.b, cfg["leaf"]
    hA = qt.from_blockmatrix(A, leaf)
    ref_pos = oracle.pattern_by_definition(A, A)
    rng = np.random.default_rng(12)
    pick = np.sort(rng.choice(len(ref_pos), size=min(samples, len(ref_pos)), replace=False))
    sI = (ref_pos[pick] // A.nb_cols).astype(np.int32)
    sJ = (ref_pos[pick] % A.nb_cols).astype(np.int32)
    index = oracle.make_index(A, A)
    sref = np.stack([oracle.block_by_definition(A, A, i, j, index) for i, j in zip(sI, sJ)])
    paths = {}
    for prec in ("f64", "f32", "bf16x3"):
        qt.prepare(hA, prec)
        log(f"bench: {name} {prec}: {warmup} warmup + {steps} timed steps")
        dt, prof, C = timed_steps(qt, torch, hA, prec, steps, warmup)
        P = C.stats()["products"]
        flops = 2.0 * b ** 3 * P
        num_ms = prof["numeric_ms"] / max(prof["calls"], 1)
        # operand bytes per element: fp64 A; fp32 A; bf16 hi and lo of A and of its transposed
        # copy; C in fp32 for the FP32 path, else fp64
        alg = (A.nnz * {"f64": 8, "f32": 4, "bf16x3": 8}[prec] + C.nblocks * (4 if prec == "f32" else 8)) * b * b
        I, J = C.pattern()
        pos = I.astype(np.int64) * A.nb_cols + J
        if prec == "bf16x3":
            # the split path's MFMAs are bf16: three per block product, against the bf16 rate
            roof = roofline_bound(3 * flops, alg, num_ms, PEAK["bf16x3"])
        else:
            roof = roofline_bound(flops, alg, num_ms, PEAK[prec])
        entry = {"tflops": flops * steps / dt / 1e12, "ms_per_step": dt / steps * 1e3, "numeric_ms": num_ms,
                 "numeric_tflops": flops / (num_ms * 1e-3) / 1e12, "block_products": P, "nnz_C": C.nblocks,
                 "roofline": roof, "pattern_matches_oracle": bool(np.array_equal(pos, ref_pos))}
        if entry["pattern_matches_oracle"]:
            V, F = C.get_blocks(sI, sJ, "f64")
            d = V - sref
            entry["e_max"] = float(np.abs(d).max())
            entry["e_max_rel"] = float(np.abs(d).max() / np.abs(sref).max())
            entry["e_F"] = float(np.linalg.norm(d) / np.linalg.norm(sref))
            entry["error_sample"] = f"{len(sI)} C blocks drawn uniformly, against the definition"
        entry["roofline"]["traffic"] = measured_traffic(name, prec)
        C.free()
        log(f"bench: {name} {prec}: {entry['tflops']:.2f} TFLOP/s end to end, numeric {num_ms:.3f} ms "
            f"({entry['roofline']['frac']:.2f} of the {'bf16 ' if prec == 'bf16x3' else ''}"
            f"{entry['roofline']['bound']} roof)")
        paths[prec] = entry
    for prec in ("f32", "bf16x3"):
        paths[prec]["speedup_vs_f64"] = paths[prec]["tflops"] / paths["f64"]["tflops"]
    hA.free()
    return {"workload": name, "n": A.n_rows, "b": b, "leaf": leaf, "nnz_A": A.nnz, "op": "C = A*A",
            "paths": paths}


if __name__ == "__main__":
    main()
