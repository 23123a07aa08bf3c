"""The 3D plain method's whole protocol on the GPU (Sec. 2: the flow is run
to a steady state first, then the ions are transported on it): the seeded
64^3 sub-case of the 128^3 sphere electrode (porosity 0.5, radii 3-6, inlet
velocity 5e-4, 20 thermal voltages) is run to a steady flow (residual 1e-8,
or the FP32 stagnation point), then 20000 Nernst-Planck steps on the frozen
flow. The FP64 oracle's result of the same protocol is stored in
tests/golden/cfg1_sub64.npz (written by make_cfg1_sub64.py beside it, which
calls only the oracle): every 4th fluid node of the steady velocity and of the
final concentrations, the adsorbed totals. Bars: velocity rel L2 1e-5 over the
stored nodes, |C - C_oracle| <= 1e-4, adsorbed totals 1e-4 relative."""
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("streaming", ["pull", "aa"])
def test_cfg1_protocol_on_the_64_cube(streaming):
    import paper_2110_13055_amd as P
    from make_cfg1_sub64 import FLOW_TOL, NP_STEPS, case
    ref = np.load(os.path.join(HERE, "golden", "cfg1_sub64.npz"))
    g, p = case()
    p.streaming = P.STREAM_PULL if streaming == "pull" else P.STREAM_AA
    print(f"cfg1 sub-case {g.nx}^3 streaming={streaming}", flush=True)
    s = P.Solver(g, p)
    assert s.n_fluid == int(ref["n_fluid"])
    rc, steps, r = s.flow_to_steady(tol=FLOW_TOL, max_steps=400000, check_every=100)
    idx = np.arange(0, s.n_fluid, int(ref["stride"]))
    u = s.velocity()[:, idx].astype(np.float64)
    uo = ref["u"].astype(np.float64)
    err = float(np.linalg.norm(u - uo) / np.linalg.norm(uo))
    print(f"flow rc={rc} steps={steps} r={r:.3e} (oracle {int(ref['flow_steps'])} steps); u relL2={err:.3e}",
          flush=True)
    assert rc in (P._lib.OK, P._lib.STAGNATED)
    assert err <= 1e-5
    s.np_step(int(ref["np_steps"]))
    c = s.concentration()[:, idx]
    dc = float(np.abs(c - ref["c"]).max())
    a, ao = s.adsorbed_total(), ref["adsorbed"]
    print(f"ions: max |dC| {dc:.2e}, adsorbed {a} vs {ao}", flush=True)
    assert np.abs(ref["c"] - 1.0).max() > 0.05
    assert dc <= 1e-4
    assert np.all(np.abs(a - ao) <= 1e-4 * np.abs(ao))
