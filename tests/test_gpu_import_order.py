"""The binding works whatever the caller imported first: a fresh process that
calls a host-only entry point before anything has imported torch still steps
a solver on the GPU (the library must bind the HIP runtime torch uses, not
the system one: loaded first, it bound the system runtime, which shared no
device state with torch's and found no device)."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = """
import paper_2110_13055_amd as P
ok, est, msg = P.flow_check(*P.preset("channel2d_128x64")[:2])   # host only, before torch
assert ok and est > 0
s = P.Solver(*P.preset("channel2d_128x64")[:2])
s.flow_steps(10)
s.np_step(4, fused=True)
u = s.velocity()
assert abs(u).max() > 0
print("import order ok", s.n_fluid, flush=True)
"""


def test_host_call_before_torch_then_gpu_steps():
    env = dict(os.environ, PYTHONPATH=ROOT + os.pathsep + os.environ.get("PYTHONPATH", ""))
    r = subprocess.run([sys.executable, "-c", SCRIPT], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "import order ok" in r.stdout
