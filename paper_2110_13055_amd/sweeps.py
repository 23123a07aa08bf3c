"""Parameter sweeps of the paper's Sec. 5 on the GPU.

    python -m paper_2110_13055_amd.sweeps fibres [--n 150] [--out FILE]

The fibrous-electrode sweep: 12 electrodes of straight overlapping fibres
(diameters 4, 6, 8 voxels = 400, 600, 800 nm; porosity 0.5-0.8; 150^3
voxels), the physical values of Sec. 5 in lattice units (``presets.py``).
Each electrode's flow is stepped to its steady state; then all 12 advance
their ions together as one batch on the frozen flow, in chunks, until the
salt removal of every electrode changes by less than ``--tol`` between
chunks. Reports per electrode: achieved porosity, specific surface, l_c,
U, Pe, Da and the salt removal percentage P_rm (Sec. 4.1).

Potential: the fibre surface carries -1.2 V (Sec. 5). With the charge of
Eq. (5) neglected and no other Dirichlet boundary, the Laplace solution of
Eq. (4) is that value in the whole pore space (``cdi_solve_potential`` with
field-free x ends returns it), so there is no migration; the removal is set
by advection, diffusion and adsorption, as the paper's reading of its
Fig. 16 through the specific surface suggests. The sweep solves that
potential anyway, so the run exercises the path the paper describes.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import _lib as L
from .presets import FIBRE_PSI_SURFACE, fibre_sweep
from .solver import Batch, Potential, Solver


def _finish(rows, solvers, prm, done):
    for r, s, v in zip(rows, solvers, prm):
        r.update(ion_steps=done, P_rm_na=float(v[0]), P_rm_cl=float(v[1]), P_rm=float(v[2]),
                 removed_amount_per_window=float(v[3]), adsorbed=s.adsorbed_total().tolist())


def run_fibres(n: int = 150, chunk: int = 20000, max_steps: int = 1_000_000, tol: float = 2e-3,
               flow_tol: float = 1e-6, flow_max: int = 60000, log=print, checkpoint=None):
    """checkpoint(rows), if given, receives the rows after every chunk."""
    import torch
    cases = fibre_sweep(n=n)
    stream = torch.cuda.Stream()
    solvers, rows = [], []
    for (d, phi), g, p in cases:
        t0 = time.perf_counter()
        s = Solver(g, p, stream=stream)
        rc, steps, res = s.flow_to_steady(flow_tol, flow_max, 100)
        it, _ = s.solve_potential(Potential(psi_electrode=FIBRE_PSI_SURFACE, tol=1e-8))
        diag = s.diagnostics()
        info = s.info()
        rows.append(dict(diameter_vox=d, porosity_target=phi, porosity=info.porosity, n_fluid=s.n_fluid,
                         flow_steps=steps, flow_residual=res, flow_status=L.STATUS_NAMES.get(rc, rc),
                         potential_iterations=it, specific_surface=diag["specific_surface"], l_c=diag["l_c"],
                         U=diag["U"], Pe=diag["Pe"][0], Da=diag["Da"][0], n_inlet=diag["n_inlet"]))
        solvers.append(s)
        log(f"flow d={d} phi={phi}: {steps} steps, r={res:.2e}, U={diag['U']:.3e}, "
            f"{time.perf_counter() - t0:.1f} s", flush=True)
    b = Batch(solvers, stream=stream)
    modes = [L.MODE_IONS] * len(solvers)
    prev = None
    done = 0
    t0 = time.perf_counter()
    while done < max_steps:
        bal0 = [s.mass_balance() for s in solvers]
        b.advance(chunk, modes)
        done += chunk
        prm = np.array([s.salt_removal(b0, s.mass_balance(), chunk, r["n_inlet"], r["U"])
                        for s, b0, r in zip(solvers, bal0, rows)])
        change = np.inf if prev is None else float(np.abs(prm[:, 2] - prev[:, 2]).max())
        log(f"ions {done} steps ({time.perf_counter() - t0:.0f} s): P_rm "
            + " ".join(f"{v:.3f}" for v in prm[:, 2]) + f"  max change {change:.2e}", flush=True)
        prev = prm
        _finish(rows, solvers, prm, done)
        for r in rows:
            r["converged"] = bool(change < tol)
        if checkpoint:
            checkpoint(rows)
        if change < tol:
            break
    b.close()
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("sweep", choices=("fibres",))
    ap.add_argument("--n", type=int, default=150)
    ap.add_argument("--chunk", type=int, default=20000)
    ap.add_argument("--max-steps", type=int, default=1_000_000)
    ap.add_argument("--tol", type=float, default=2e-3)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)

    def dump(rows):
        if a.out:
            with open(a.out, "w") as fh:
                fh.write("\n".join(json.dumps(r) for r in rows) + "\n")

    rows = run_fibres(a.n, a.chunk, a.max_steps, a.tol, checkpoint=dump)
    dump(rows)
    print("\n".join(json.dumps(r) for r in rows), flush=True)


if __name__ == "__main__":
    sys.exit(main())
