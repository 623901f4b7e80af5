"""CPU checks of the benchmark script's contract: one GPU only, counter tables that
apply only to the kernel source and factors they were measured on, and the parsing
of the device calibration."""
import hashlib
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _kernels_sha():
    with open(os.path.join(ROOT, "paper_2105_02995_amd", "csrc", "kernels.hip"), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def test_counter_tables_apply_only_to_the_profiled_source_and_factors():
    sha = _kernels_sha()
    table = {"k_demo<float, 2, 2>": {"bytes": 3.0e9, "kernels_sha256": sha, "bf_nnz": 7}}
    assert bench.counted(table, "k_demo<float, 2, 2> (rocprof name)", 7)["bytes"] == 3.0e9
    assert bench.counted(table, "k_demo<float, 2, 2>", 8) is None        # other factors
    assert bench.counted(table, "k_other<float>", 7) is None             # other kernel
    stale = {"k_demo<float, 2, 2>": {"bytes": 3.0e9, "kernels_sha256": "0" * 64, "bf_nnz": 7}}
    assert bench.counted(stale, "k_demo<float, 2, 2>", 7) is None        # other source


def test_committed_counter_tables_are_well_formed():
    for table, key in ((bench.TRAFFIC, "bytes"), (bench.MFMA_COUNTERS, "executed_flop"),
                       (bench.PLAIN_TRAFFIC, "bytes")):
        assert table
        for name, e in table.items():
            assert len(e["kernels_sha256"]) == 64
            assert e["bf_nnz"] > 0
            assert e[key] > 0
    for e in bench.MFMA_COUNTERS.values():
        assert 0.0 < e["busy"] <= 1.0


def test_calibration_output_parsing():
    out = bench.parse_calibration([
        "read: 4 GiB per dispatch, 4096 workgroups, 5.59 TB/s",
        "read: 4 GiB per dispatch, 65536 workgroups, 6.02 TB/s",
        "read: 4 GiB per dispatch, 16384 workgroups, 5.96 TB/s",
        "mfma f32 16x16x4: 144.6 TFLOP/s",
        "mfma f64 16x16x4: 46.4 TFLOP/s",
        "unrelated line",
    ])
    assert out == {"read_tbs": 6.02, "mfma_loop_f32_tflops": 144.6, "mfma_loop_f64_tflops": 46.4}
