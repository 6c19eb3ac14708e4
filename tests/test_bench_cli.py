"""bench.py's command line on the CPU: one GPU only (--gpus N > 1 exits with
a message and status 2 before any GPU work), and --help lists the flags the
benchmark's sections use."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_help_lists_the_sections():
    r = _run("--help")
    assert r.returncode == 0
    for flag in ("--steps", "--warmup", "--frac-bits", "--no-fits", "--fits-only", "--no-batch", "--no-serve",
                 "--no-lookups", "--no-queries", "--no-cpu-baseline"):
        assert flag in r.stdout, flag


def _bench_module():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _full_record(mod):
    """A full record shaped like a real run's, every section present, with
    long strings where the real one has them."""
    long = "x" * 600
    per_eps = {str(e): {"ratio": 0.15, "bits_per_key": 9.6, "blob_bytes": 120_000_000, "nseg_total": 4_000_000,
                        "paper_size_formula_bits_per_key": 10.0, "decode_ms_cold": 0.2, "decode_GBps_cold": 4000.0,
                        "decode_ms_warm": 0.16, "decode_GBps_warm": 5000.0, "compress_ms": 0.8,
                        "compress_GBps": 1000.0} for e in (15, 63, 255)}
    return {
        "metric": mod.METRIC, "value": 4000.0, "unit": "GB/s", "n_gpus": 1, "steps": 20, "warmup": 5,
        "ms_per_step": 4.2, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "w" * 260, "n": 100_000_000, "key_bytes": 8, "log2_block": 10, "eps": [15, 63, 255],
                   "frac_bits": 0},
        "roofline": {"bound": "hbm", "achieved": 5000.0, "peak": 8000.0, "unit": "GB/s", "frac": 0.625,
                     "traffic": 1.05e9, "cache": "cold", "kernel": "decode_full_kernel<8, false> (lc_decompress)",
                     "bytes_per_launch": 920_000_000, "avg_launch_ms": 0.184},
        "roofline_warm": {"bound": "hbm", "achieved": 5700.0, "peak": 8000.0, "unit": "GB/s", "frac": 0.71,
                          "traffic": 1.05e9, "cache": "warm", "avg_launch_ms": 0.16, "decoded_GBps": 5000.0},
        "roofline_encode": {"bound": "alu", "kernel": long, "achieved": 14.4, "peak": 39.32, "unit": "T", "frac": 0.37,
                            "traffic": None, "hbm": {"achieved": 1100.0, "peak": 8000.0, "frac": 0.14, "bytes": long},
                            "avg_call_ms": 0.8, "valu_source": long},
        "per_eps": per_eps, "decompress_range_GBps": 3000.0, "access_lookups_per_s": 1.2e10,
        "lower_bound_lookups_per_s": 6e9, "paper_cpu_context": {"lc-simd": long},
        "lookups": {"workload": long, "x": [long] * 5}, "queries": {"workload": long, "y": [long] * 5},
        "fits": {"z": [long] * 10},
        "batching": {"workload": long, "decoded_GBps": {"batched": 2800.0, "per_list": 30.0}, "bits_per_key": 16.9,
                     "step_ms": {"batched_eager": 6.0, "batched_graph": 6.0, "per_list_eager": 724.0,
                                 "per_list_graph": 700.0}, "block_size_autotune": [long] * 5},
        "serving": {"workload": long, "points": [{"qps_offered": "saturation", "requests": 100000, "p50_us": 900.0,
                                                  "p99_us": 2000.0, "qps_achieved": 300000.0, "note": long}],
                    "saturation_speedup_vs_unbatched": 40.0},
        "cpu_baseline": {"value": 2.5, "unit": "GB/s", "cores": 16, "kind": "oracle", "sample": "s" * 120,
                         "single_core_GBps": 0.28, "compress_GBps": {"single_core": 0.2, "all_cores": 2.0},
                         "host": {"cpu": "Some CPU @ 2.70GHz", "cores_available": 16, "nproc": 128}},
    }


def test_headline_is_last_short_and_carries_the_roofline_and_cpu_baseline(capsys, tmp_path):
    import json
    mod = _bench_module()
    full = _full_record(mod)
    path = tmp_path / "full.json"
    mod.emit(full, str(path))
    out = capsys.readouterr()
    last = out.out.strip().splitlines()[-1]
    assert len(last.encode()) <= 2048 < 4096
    assert "batching" in last and "serving" in last
    h = json.loads(last)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "dtype"):
        assert h[k] == full[k], k
    assert h["config"]["workload"] == full["config"]["workload"]
    assert h["roofline"]["frac"] == 0.625 and h["roofline"]["cache"] == "cold"
    assert h["roofline_warm"]["cache"] == "warm"
    assert h["cpu_baseline"]["cores"] == 16 and h["cpu_baseline"]["kind"] == "oracle"
    assert h["cpu_baseline"]["value"] == 2.5
    # the full record goes to stderr and to the file, unchanged
    assert json.loads(path.read_text()) == full
    assert json.dumps(full) in out.err


def test_cpu_baseline_reports_host_cores_and_medians():
    import numpy as np
    mod = _bench_module()
    rng = np.random.default_rng(5)
    keys = np.cumsum(rng.integers(1, 1000, 300_000)).astype(np.uint64)
    r = mod.cpu_baseline(keys, [15, 63], budget_s=0.5, max_threads=4, reps=3)
    assert r["kind"] == "oracle" and r["unit"] == "GB/s"
    assert 1 <= r["cores"] <= 4 and r["value"] > 0 and r["single_core_GBps"] > 0
    assert r["host"]["cpu"] and r["host"]["cores_available"] >= 1
    assert "median of 3" in r["sample"]
    for op in ("access_lookups_per_s", "lower_bound_lookups_per_s"):
        assert r[op]["single_core"] > 0 and r[op]["all_cores"] > 0
    assert "eps 63" in r["queries"]
