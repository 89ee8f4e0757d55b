"""Write the fine-grid reference of the 2D accuracy test (Example 5.6) used by
the 2D pins in tests/test_oracle_pins_2d.py.

Tables 5.6-5.8 measure L1 errors of h + b, hu, hv at t = 0.05 against a fine
run of the same periodic data on [0,1]^2.  This script runs the 2D oracle (and
only the oracle) on 200 x 200 cells of the tensor-product moving mesh (nodes
back on the uniform grid at t_end, since sin(2 pi) = 0), CFL 0.4 (the paper's
for 200 x 200), and stores the cell averages of h + b, hu, hv block-averaged
onto 50 x 50 uniform cells (a mean of 4 x 4 fine cells of equal area is the
coarse cell's average).  The run takes a few minutes of one CPU core.

    python tests/golden/make_2d_reference.py [n_fine]
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

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "ex56_reference.txt")
N_COARSE = 50


def main(n_fine: int = 200) -> None:
    wl = W.accuracy_2d(n_fine)
    P = O.params2(cfl=0.4, Ax=wl["Ax"], kx=wl["kx"], omx=wl["omx"], Ay=wl["Ay"], ky=wl["ky"],
                  omy=wl["omy"])
    t0 = time.time()
    r = O.run2(P, wl["h"], wl["hu"], wl["hv"], wl["b"], wl["xi"], wl["yi"], wl["xi"], wl["yi"],
               t_end=wl["t_end"])
    if r["status"] != 0:
        raise SystemExit(f"oracle status {r['status']}")
    f = n_fine // N_COARSE

    def coarse(a):
        return a.reshape(N_COARSE, f, N_COARSE, f).mean(axis=(1, 3))

    eta, hu, hv = coarse(r["h"] + r["b"]), coarse(r["hu"]), coarse(r["hv"])
    xdev = max(np.abs(r["x"] - wl["xi"]).max(), np.abs(r["y"] - wl["yi"]).max())
    with open(OUT, "w") as fh:
        fh.write("# Example 5.6 reference: 2D oracle (special source-term scheme), tensor-product\n")
        fh.write(f"# moving mesh, {n_fine} x {n_fine} cells, CFL 0.4, t = {r['t']:.17g}, "
                 f"{r['steps']} steps ({time.time() - t0:.0f} s); max node offset at t_end "
                 f"{xdev:.3e}.\n")
        fh.write(f"# Cell averages of h+b, hu, hv on {N_COARSE} x {N_COARSE} uniform cells (means of "
                 f"{f} x {f} fine cells), row j = 0..{N_COARSE - 1} (y), column i (x); one line per "
                 "cell, i fastest.\n")
        fh.write("# written by tests/golden/make_2d_reference.py (calls only oracle/)\n")
        for a, b, c in zip(eta.ravel(), hu.ravel(), hv.ravel()):
            fh.write(f"{a:.17e} {b:.17e} {c:.17e}\n")
    print(f"wrote {OUT}: {n_fine}^2 cells, {r['steps']} steps, {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 200)
