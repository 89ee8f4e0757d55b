"""Write the fine-grid reference of the accuracy test (Example 5.1) used by the
convergence pins in tests/test_oracle_pins.py.

The paper measures the L1 errors of Tables 5.1/5.2 against a fine-grid run of
the same initial data (periodic [0,1], b = sin^2(pi x), h = 5 + exp(cos 2 pi x),
hu = sin(cos 2 pi x), t = 0.1, CFL 0.1).  This script runs the oracle (and only
the oracle) on 6400 cells of the moving mesh eq. (5.1), whose nodes are uniform
again at t_end, and stores the cell averages of h + b and hu block-averaged onto
800 cells (exact: an average over 8 fine cells is the average over the coarse
cell).  The run takes a few hours of one CPU core.

    python tests/golden/make_convergence_reference.py [n_fine]
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2208_06588_amd import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "table52_reference.txt")
N_COARSE = 800


def main(n_fine: int = 6400) -> None:
    wl = W.accuracy_1d(n_fine, mesh="paper")
    P = O.params(bc=O.BC_PERIODIC, mesh=O.MESH_PAPER, mesh_A=wl["mesh_A"], mesh_k=wl["mesh_k"],
                 mesh_omega=wl["mesh_omega"], cfl=0.1, weno_eps=wl["weno_eps"])
    t0 = time.time()
    r = O.run(P, wl["h"], wl["hu"], wl["b"], wl["x"], wl["xi"], t_end=wl["t_end"])
    if r["status"] != 0:
        raise SystemExit(f"oracle status {r['status']}")
    f = n_fine // N_COARSE
    eta = (r["h"] + r["b"]).reshape(-1, f).mean(axis=1)
    hu = r["hu"].reshape(-1, f).mean(axis=1)
    xdev = np.abs(r["x"] - wl["xi"]).max()
    with open(OUT, "w") as fh:
        fh.write("# Example 5.1 reference: oracle, special source-term scheme, moving mesh eq. (5.1),\n")
        fh.write(f"# {n_fine} cells, CFL 0.1, t = {r['t']:.17g}, {r['stats'].steps} steps "
                 f"({time.time() - t0:.0f} s); max |x(t_end) - xi| = {xdev:.3e}.\n")
        fh.write(f"# Cell averages of h+b and hu on {N_COARSE} uniform cells (means of {f} fine cells).\n")
        fh.write("# written by tests/golden/make_convergence_reference.py (calls only oracle/)\n")
        for a, c in zip(eta, hu):
            fh.write(f"{a:.17e} {c:.17e}\n")
    print(f"wrote {OUT}: {n_fine} cells, {r['stats'].steps} steps, {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 6400)
