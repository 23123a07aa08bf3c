"""Writes cfg1_sub64.npz: the FP64 oracle's result of the 3D plain-method
protocol (flow to a steady state, then 20000 Nernst-Planck steps on the frozen
flow; Sec. 2) on the seeded 64^3 sub-case of the 128^3 sphere electrode
(porosity 0.5, radii 3-6, inlet velocity 5e-4, 20 thermal voltages).

Calls only oracle/ (and the seeded primitive generator through it). Stored:
the steps and residual of the flow stop; every 4th fluid node (lexicographic
fluid order) of the steady velocity and of both concentrations after the ion
steps (float32: their rounding, 6e-8 relative, is far below the parity bars);
the adsorbed totals and the balance in float64.

    python tests/golden/make_cfg1_sub64.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

EDGE, FLOW_TOL, NP_STEPS, STRIDE = 64, 1e-8, 20000, 4


def case():
    import paper_2110_13055_amd as P
    g, p, _ = P.preset("spheres3d_128")
    g.nx = g.ny = g.nz = EDGE
    return g, p


def main():
    from helpers import oracle_solver
    g, p = case()
    o = oracle_solver(g, p)
    t0 = time.time()
    rc, steps, r = o.flow_to_steady(tol=FLOW_TOL, max_steps=400000, check_every=100)
    assert rc == 0, rc
    u = o.velocity()
    print(f"flow: {steps} steps, r = {r:.3e}, {time.time() - t0:.0f} s", flush=True)
    o.freeze_velocity()
    assert o.np_steps(NP_STEPS) == 0
    c = o.conc()
    print(f"ions: {NP_STEPS} steps, {time.time() - t0:.0f} s", flush=True)
    idx = np.arange(0, o.nf, STRIDE)
    np.savez_compressed(os.path.join(HERE, "cfg1_sub64.npz"), n_fluid=o.nf, flow_steps=steps, flow_residual=r,
                        np_steps=NP_STEPS, stride=STRIDE, u=u[:, idx].astype(np.float32),
                        c=c[:, idx].astype(np.float32), adsorbed=o.adsorbed_total(), balance=o.balance())


if __name__ == "__main__":
    main()
