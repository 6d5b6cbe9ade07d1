"""CPU: the host-side logic of bench.py (no GPU): the roofline's choice of
bound, the digest that keys measured traffic to the kernels' code, and the
refusal to run on more than one GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_roofline_bound_mfma_and_hbm():
    # decay32768: 58.25 GFLOP over 1.355 GB (43 flop/B) -> MFMA-bound at fp64
    r = bench.roofline_bound(58.25e9, 1.355e9, 1.2, bench.PEAK["f64"])
    assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s"
    assert r["achieved"] == pytest.approx(58.25e9 / 1.2e-3 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / 78.6)
    # random65536: 56.24 GFLOP over 6.70 GB (8.4 flop/B) is below the fp64 ridge (9.8) -> HBM-bound
    r = bench.roofline_bound(56.24e9, 6.70e9, 2.6, bench.PEAK["f64"])
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["achieved"] == pytest.approx(6.70e9 / 2.6e-3 / 1e9)
    assert r["ridge"] == pytest.approx(78.6e12 / 8e12)
    # the same bytes at fp32 (half the C bytes) against the fp32 ridge (19.7)
    assert bench.roofline_bound(56.24e9, 3.35e9, 1.3, bench.PEAK["f32"])["bound"] == "hbm"


def test_code_digest_ignores_comments_only(tmp_path):
    a = tmp_path / "a.hip"
    b = tmp_path / "b.hip"
    c = tmp_path / "c.hip"
    a.write_text("int f(int x) { return x + 1; }  // add one\n/* block */\n")
    b.write_text("// a comment first\nint f(int x)\n{\n    return x + 1;\n}\n")
    c.write_text("int f(int x) { return x + 2; }\n")
    assert bench.code_digest(str(a)) == bench.code_digest(str(b))
    assert bench.code_digest(str(a)) != bench.code_digest(str(c))
    # several sources: each one's code counts, and where one ends
    assert bench.code_digest(str(a), str(c)) != bench.code_digest(str(a), str(a))
    assert bench.code_digest(str(a), str(c)) == bench.code_digest(str(b), str(c))


def test_measured_traffic_keyed_to_code():
    # a workload with no counter record has no traffic; a committed record is
    # used only while the numeric kernels and the launch order are the code
    # it was taken with
    assert bench.measured_traffic("no-such-workload", "f64") is None
    assert [os.path.basename(p) for p in bench.TRAFFIC_SOURCES] == ["qt_numeric.hip", "qt_multiply.hip"]
    rec = os.path.join(ROOT, "profiles", "traffic_f64_decay32768.json")
    if os.path.exists(rec):
        import json
        d = json.load(open(rec))
        expect = d["traffic_bytes"] if d.get("code_sha256") == bench.code_digest(*bench.TRAFFIC_SOURCES) else None
        assert bench.measured_traffic("decay32768", "f64") == expect


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_check_path_fails_on_pattern_and_bounds():
    ok = {"pattern_matches_oracle": True, "e_F": 1e-15, "e_max_rel": 4e-15}
    assert bench.check_path(ok, "f64") == []
    assert bench.check_path({"pattern_matches_oracle": False}, "f64")
    assert bench.check_path(dict(ok, e_F=2e-12), "f64")
    assert bench.check_path(dict(ok, e_max_rel=float("nan")), "f64")     # NaN never passes
    # the fp32 path is held to its own, looser bound
    assert bench.check_path(dict(ok, e_F=4e-7, e_max_rel=2e-6), "f32") == []
    assert bench.check_path(dict(ok, e_F=4e-5), "f32")
    assert bench.check_path(dict(ok, e_F=8e-7, e_max_rel=2e-6), "bf16x3") == []


def test_row_sample_takes_leading_block_rows():
    import numpy as np
    import workloads as wl
    rng = np.random.default_rng(3)
    n = 16
    pos = np.sort(rng.choice(n * n, size=60, replace=False))
    I, J = (pos // n).astype(np.int32), (pos % n).astype(np.int32)
    A = wl.BlockMatrix(n * 4, n * 4, 4, I, J, rng.standard_normal((60, 4, 4)))
    rowcnt = np.bincount(I, minlength=n)
    P = int(sum(rowcnt[j] for j in J))
    full = bench.row_sample(wl, A, P, 1e18, "t")
    assert full[0] is A and full[1] == P and full[2] is None
    flops_half = 2.0 * 4 ** 3 * P / 2
    Ao, P_o, R, _ = bench.row_sample(wl, A, P, flops_half, "t")
    assert (Ao.I < R).all() and Ao.nnz == int((I < R).sum())
    # block products of the sampled rows: sum over their blocks (i, k) of the blocks in row k
    assert P_o == int(sum(rowcnt[k] for i, k in zip(I, J) if i < R))
    assert 2.0 * 4 ** 3 * P_o >= flops_half


def _pmc_csv(path, counter, rows):
    import csv
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, v in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": v})
    return str(path)


def test_traffic_from_counters_scales_and_picks_the_kernel(tmp_path):
    """The copy calibration scales each counter so that the 2 GiB copy reads
    as 2 GiB; the numeric kernel's rows are averaged over its dispatches; a
    workload launched by inner index is read from the by-k kernel's rows (not
    from another kernel of the same block size in the run)."""
    gib2 = bench.COPY_BYTES / 1024.0            # the copy's bytes in KiB
    cf = _pmc_csv(tmp_path / "cf.csv", "FETCH_SIZE", [("__amd_rocclr_copyBuffer", gib2 / 2)] * 3)
    cw = _pmc_csv(tmp_path / "cw.csv", "WRITE_SIZE", [("__amd_rocclr_copyBuffer", gib2)] * 3)
    plain, byk = "void qt::k_numeric<double, 32>(double const*)", "void qt::k_numeric_byk<double, 32>(double const*)"
    f = _pmc_csv(tmp_path / "f.csv", "FETCH_SIZE", [(plain, 999.0), (byk, 100.0), (byk, 300.0)])
    w = _pmc_csv(tmp_path / "w.csv", "WRITE_SIZE", [(plain, 999.0), (byk, 50.0), (byk, 50.0)])
    rec = bench.traffic_from_counters(f, w, cf, cw, "random65536", "f64", 32, out_dir=str(tmp_path))
    assert rec["kernel"] == "k_numeric_byk<double, 32>" and rec["dispatches"] == [2, 2]
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    assert rec["fetch_bytes"] == pytest.approx(200.0 * 1024 * 2.0)
    assert rec["write_bytes"] == pytest.approx(50.0 * 1024)
    assert os.path.exists(tmp_path / "traffic_f64_random65536.json")
    # without by-k rows: the plain kernel
    f2 = _pmc_csv(tmp_path / "f2.csv", "FETCH_SIZE", [(plain, 400.0)])
    w2 = _pmc_csv(tmp_path / "w2.csv", "WRITE_SIZE", [(plain, 100.0)])
    rec = bench.traffic_from_counters(f2, w2, cf, cw, "decay32768", "f64", 32, out_dir=str(tmp_path))
    assert rec["kernel"] == "k_numeric<double, 32>" and rec["traffic_bytes"] == pytest.approx((800.0 + 100.0) * 1024)
    # the LDS-shared kernels of 64-wide blocks
    f3 = _pmc_csv(tmp_path / "f3.csv", "FETCH_SIZE", [("qt::k_numeric_f32_b64(float const*)", 10.0)])
    w3 = _pmc_csv(tmp_path / "w3.csv", "WRITE_SIZE", [("qt::k_numeric_f32_b64(float const*)", 10.0)])
    assert bench.traffic_from_counters(f3, w3, cf, cw, "decay131072", "f32", 64,
                                       out_dir=str(tmp_path))["kernel"] == "k_numeric_f32_b64"
