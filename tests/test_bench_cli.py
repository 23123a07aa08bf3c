"""The bench's command line on the CPU: more than one GPU is refused with a
message (this build measures one GPU), before any GPU work; the measured
record's byte model is the one the roofline uses."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_algorithmic_bytes_per_node():
    sys.path.insert(0, ROOT)
    import bench
    # D3Q19: populations read + write, two concentrations (FP32 + FP16
    # remainder) read + write, the flux (3 floats) or the moments (float4)
    # read + write
    assert bench.BYTES_FUSED == {"fp32": 200, "fp16": 124, "fp16_dev": 132, "moments": 56}
    assert bench.BYTES_LBM["fp32"] == 152 and bench.BYTES_NP == 36
