#!/usr/bin/env python3
"""Benchmark of the quadtree block-sparse multiply C = A*A on one MI355X.

Workload (default): the 3D-decay matrix with 2048 atoms in a cube of side
40, 16 basis functions per atom (n = 32768), block size 32, blocks below
1e-10 dropped, leaf 256; inputs resident in HBM before timing. One step is
one full qt_multiply (symbolic traversal + numeric MFMA kernel + C
assembly). The metric counts 2*b^3 flops per nonzero block product.

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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


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


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="decay32768")
    ap.add_argument("--leaf", type=int, default=0, help="leaf size (0: the workload's default)")
    ap.add_argument("--prec", default="f64", choices=["f64", "f32", "bf16x3"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-paths", action="store_true", help="time only --prec")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the multiply has no multi-GPU path in this build "
              "(see the sharding paragraph of the design notes).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import workloads as wl

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    import paper_1501_07800_amd as qt

    cfg = wl.CONFIGS[args.workload]
    leaf = args.leaf or cfg["leaf"]
    log(f"bench: generating {args.workload}")
    A = wl.config(args.workload)
    b = A.b
    log(f"bench: n={A.n_rows} b={b} nnz(A)={A.nnz}; building on the GPU (leaf {leaf})")
    hA = qt.from_blockmatrix(A, leaf)
    for p in ("f64", "f32", "bf16x3"):
        if p == "bf16x3" and b == 16:
            continue
        qt.prepare(hA, p)
    torch.cuda.synchronize()

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
        sym_ms = prof["symbolic_ms"] / max(prof["calls"], 1)
        results[prec] = {"C": C, "P": P, "tflops": tflops, "ms_per_step": dt / args.steps * 1e3,
                         "numeric_ms": num_ms, "symbolic_ms": sym_ms,
                         "numeric_tflops": flops / (num_ms * 1e-3) / 1e12, "nnz_C": C.nblocks}
        log(f"bench: {prec}: {tflops:.2f} TFLOP/s end to end, numeric {num_ms:.3f} ms, symbolic {sym_ms:.3f} ms")

    main_r = results[args.prec]
    P = main_r["P"]
    flops = 2.0 * b ** 3 * P

    cpu = None
    ref = None
    if not args.no_cpu_baseline:
        import oracle
        log("bench: CPU oracle on the full workload (C = A*A, fp64, OpenMP)")
        t0 = time.perf_counter()
        ref, st = oracle.multiply(A, A, leaf)
        t1 = time.perf_counter()
        assert st.block_products == P
        cpu = {"value": flops / (t1 - t0) / 1e12, "unit": "TFLOP/s", "cores": oracle.threads(),
               "kind": "oracle", "seconds": t1 - t0,
               "sample": f"the full {args.workload} workload, C = A*A, one run"}
        log(f"bench: oracle {t1 - t0:.1f} s on {cpu['cores']} threads")

    paths = {}
    for prec, r in results.items():
        entry = {"tflops": r["tflops"], "ms_per_step": r["ms_per_step"], "numeric_ms": r["numeric_ms"],
                 "symbolic_ms": r["symbolic_ms"], "numeric_tflops": r["numeric_tflops"],
                 "mfma_peak_frac": r["numeric_tflops"] / (PEAK["f32"] if prec == "bf16x3" else PEAK[prec]),
                 "speedup_vs_f64": (r["tflops"] / results["f64"]["tflops"]) if "f64" in results else None}
        if ref is not None:
            I, J, V = r["C"].to_blocks("f64")
            if not (np.array_equal(I, ref.I) and np.array_equal(J, ref.J)):
                entry["pattern_matches_oracle"] = False
            else:
                d = V - ref.V
                entry["pattern_matches_oracle"] = True
                entry["e_max"] = float(np.abs(d).max())
                entry["e_max_rel"] = float(np.abs(d).max() / np.abs(ref.V).max())
                entry["e_F"] = float(np.linalg.norm(d) / np.linalg.norm(ref.V))
        if prec == "bf16x3":
            entry["mfma_utilisation"] = 3 * r["numeric_tflops"] / PEAK["bf16x3"]
        paths[prec] = entry

    peak = PEAK[args.prec] if args.prec != "bf16x3" else PEAK["f32"]
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
        "roofline": {"bound": "mfma", "achieved": main_r["numeric_tflops"], "peak": peak, "unit": "TFLOP/s",
                     "frac": main_r["numeric_tflops"] / peak, "traffic": None,
                     "kernel": "k_numeric (block GEMM per C block)"},
        "cpu_baseline": cpu,
        "paths": paths,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
