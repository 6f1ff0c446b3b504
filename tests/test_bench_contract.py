"""The benchmark's one-GPU contract: asked for more than one GPU, by flag or by
a launcher's WORLD_SIZE, it exits with status 2 and says why, before touching
any device.  CPU only."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("args,env", [(["--gpus", "2"], {}), ([], {"WORLD_SIZE": "2"})])
def test_more_than_one_gpu_is_refused(args, env):
    e = dict(os.environ)
    e.update(env)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + args, cwd=ROOT, env=e,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2, (r.returncode, r.stderr)
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def _bench_module():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_roofline_objects_from_a_kernel_table():
    """The roofline of the dominant kernel and the path-level roofline, from a
    hand-made profile table: achieved = algorithmic bytes per launch over the
    average launch time, as a fraction of 8 TB/s; the path fraction is
    queries/s times the profiled bytes per query over 8 TB/s."""
    b = _bench_module()
    tab = [{"name": "spmm_separator_rows", "launches": 10, "total_ms": 2.0, "alg_bytes": 8.0e9},
           {"name": "m11_block_apply", "launches": 10, "total_ms": 0.5, "alg_bytes": 1.0e9}]
    for r in tab:
        r["avg_us"] = 1e3 * r["total_ms"] / r["launches"]
        r["alg_bytes_per_launch"] = r["alg_bytes"] / r["launches"]
        r["achieved_GBs"] = r["alg_bytes"] / (r["total_ms"] * 1e-3) / 1e9
    rf = b.roofline_of(tab, "no_such_workload", 5000.0)
    assert rf["kernel"] == "spmm_separator_rows" and rf["bound"] == "hbm" and rf["unit"] == "GB/s"
    assert rf["avg_launch_us"] == 200.0 and rf["alg_bytes_per_launch"] == 8.0e8
    assert abs(rf["achieved"] - 4000.0) < 1e-9 and abs(rf["frac"] - 0.5) < 1e-12
    assert rf["traffic"] is None  # no profile summary for this workload
    assert abs(rf["frac_of_measured_copy"] - 0.8) < 1e-12
    pr = b.path_roofline(tab, 10, 100.0)
    assert pr["alg_bytes_per_query"] == 9.0e8
    assert pr["frac"] == round(100.0 * 9.0e8 / 8.0e12, 4)  # reported to 4 digits
    assert abs(pr["roof_qps"] - 8.0e12 / 9.0e8) < 1e-6


def test_committed_traffic_summaries_match_the_kernel_source():
    """Every committed per-launch traffic summary names the SpMM source it was
    taken on; the bench reports its bytes only while that source is current,
    so a stale summary reads as no traffic."""
    import glob
    import json
    b = _bench_module()
    h = b.kernel_source_hash()
    files = glob.glob(os.path.join(ROOT, "profiles", "pmc_spmm_separator_rows_*.json"))
    assert files
    for f in files:
        d = json.load(open(f))
        wl = os.path.basename(f)[len("pmc_spmm_separator_rows_"):-len(".json")]
        got = b.load_traffic("spmm_separator_rows", wl, d["algorithmic_bytes_per_launch"])
        if d["kernel_source_sha256_16"] == h:
            assert got == d["hbm_bytes_per_launch"]
        else:
            assert got is None
