"""Host-side checks of bench.py's contract (no GPU needed).

* More than one GPU is refused with a message and a non-zero status, before anything
  touches a device.
* Measured HBM traffic is reported only for the workload and precision the committed
  rocprofv3 counters were taken on (Ly=8 chi=3200, BF16x3); any other request gets none.
"""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_measured_traffic_only_for_its_own_workload():
    assert bench.measured_traffic("ly6_chi800", "bf16x3") == {}
    assert bench.measured_traffic("ly8_chi3200", "fp32") == {}
    rec = bench.measured_traffic("ly8_chi3200", "bf16x3")
    # the committed counters either match the current kernel sources (then every matvec
    # kernel the bench names has an entry) or do not (then nothing is reported)
    if rec:
        for k in ("mrd::gemm_bf3_kernel<0, 128, 64, 2, 2, false, false>",
                  "mrd::gemm_bf3_kernel<148, 128, 32, 4, 1, true, false>",
                  "mrd::mix_slab_kernel<float, float, false>",
                  "mrd::gemm_split_reduce_kernel<float, 148, mrd::GemmProb, false>"):
            assert rec[k]["read_bytes"] > 0 and rec[k]["write_bytes"] > 0
