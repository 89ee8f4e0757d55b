"""Fifth-order convergence of the oracle on Example 5.1 (Tables 5.1 and 5.2):
N = 50 .. 800 cells of the moving mesh eq. (5.1), CFL 0.1 as the paper runs
it, t = 0.1, against the committed 6400-cell oracle reference
(tests/golden/table52_reference.txt, written by make_convergence_reference.py;
the mesh is uniform again at t_end, so averages of fine cells are the coarse
cells' averages).  Every scheme converges to the same solution: the special
source-term treatment, the hydrostatic reconstruction, the scheme without
well-balancing, and the special source-term scheme with the bottom projected
(eq. (3.16)).  The runs go to a process pool (the 800-cell runs take a couple
of minutes each)."""
import concurrent.futures as cf
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_2208_06588_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")
NS = (50, 100, 200, 400, 800)
SCHEMES = {
    "special": (dict(), "table5.2"),
    "hydrostatic": (dict(flags=O.FLAG_HYDROSTATIC), "table5.2hr"),
    "nonwb": (dict(flags=O.FLAG_NONWB), "table5.1"),
    "projected": (dict(bottom=O.BOTTOM_SIN2, bottom_p=(1.0, 1.0, 0.0, 0.0)), "table5.2"),
}


def _gold(name):
    rows = []
    with open(os.path.join(GOLD, name)) as f:
        for ln in f:
            ln = ln.strip()
            if ln and not ln.startswith("#"):
                rows.append(ln.split())
    return rows


def _run(job):
    scheme, n = job
    kw, _ = SCHEMES[scheme]
    wl = W.accuracy_1d(n, mesh="paper")
    P = O.params(bc=O.BC_PERIODIC, mesh=O.MESH_PAPER, mesh_A=wl["mesh_A"], mesh_k=wl["mesh_k"],
                 mesh_omega=wl["mesh_omega"], cfl=0.1, weno_eps=wl["weno_eps"], **kw)
    r = O.run(P, wl["h"], wl["hu"], wl["b"], wl["x"], wl["xi"], t_end=0.1, max_steps=10 ** 6)
    return scheme, n, r["status"], r["h"] + r["b"], r["hu"]


@pytest.fixture(scope="module")
def errors():
    ref = np.array([[float(v) for v in row] for row in _gold("table52_reference.txt")])
    assert ref.shape == (800, 2)
    jobs = [(s, n) for n in sorted(NS, reverse=True) for s in SCHEMES]
    out = {}
    with cf.ProcessPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        for scheme, n, st, eta, hu in ex.map(_run, jobs):
            assert st == 0, (scheme, n, st)
            f = 800 // n
            ce = ref[:, 0].reshape(-1, f).mean(axis=1)
            cm = ref[:, 1].reshape(-1, f).mean(axis=1)
            out[scheme, n] = (float(np.abs(eta - ce).mean()), float(np.abs(hu - cm).mean()))
    return out


@pytest.mark.slow
@pytest.mark.parametrize("scheme", list(SCHEMES))
def test_errors_match_the_paper_tables(errors, scheme):
    """L1 errors of h + b and hu against Table 5.2 (special source term,
    hydrostatic reconstruction) or Table 5.1 (without well-balancing); the
    projected bottom against the special source-term column.  From N = 200 on
    the errors agree with the printed three digits to 2 % (measured: 1.720e-5,
    6.798e-7, 2.231e-8 for h + b against 1.72e-5, 6.80e-7, 2.23e-8), at 50 and
    100 cells to 12 % (the printed reference is another scheme's 12800-cell
    run, here the oracle's own 6400-cell run)."""
    table = SCHEMES[scheme][1]
    paper = {int(r[1]): (float(r[2]), float(r[3])) for r in _gold("paper_tables.txt")
             if r[0] == table}
    for n in NS:
        for k in range(2):
            e, p = errors[scheme, n][k], paper[n][k]
            assert abs(e / p - 1.0) < (0.02 if n >= 200 else 0.12), (scheme, n, k, e, p)


@pytest.mark.slow
@pytest.mark.parametrize("scheme", list(SCHEMES))
def test_fifth_order_from_400_to_800(errors, scheme):
    """The observed order reaches the scheme's fifth order: above 4.5 from 400
    to 800 cells and above 4.2 from 200 to 400, for h + b and hu, and within
    0.05 of the orders of the printed table (4.66 and 4.93)."""
    table = SCHEMES[scheme][1]
    paper = {int(r[1]): (float(r[2]), float(r[3])) for r in _gold("paper_tables.txt")
             if r[0] == table}
    for k in range(2):
        o1 = math.log2(errors[scheme, 200][k] / errors[scheme, 400][k])
        o2 = math.log2(errors[scheme, 400][k] / errors[scheme, 800][k])
        p1 = math.log2(paper[200][k] / paper[400][k])
        p2 = math.log2(paper[400][k] / paper[800][k])
        assert o1 > 4.2 and o2 > 4.5, (scheme, k, o1, o2)
        assert abs(o1 - p1) < 0.05 and abs(o2 - p2) < 0.05, (scheme, k, o1, o2, p1, p2)
