"""Pins of the 2D tensor-product oracle (the scheme of Sec. 2-4 in two
dimensions on a mesh whose nodes move along each logical direction) against
facts fixed by the paper and by mathematics: polynomial reproduction of one
sweep, the reduction to the pinned 1D scheme for data constant in y, the x/y
transposition symmetry, the constant state under mesh motion (GCL), discrete
conservation, the still-water state of Example 5.11 (Table 5.12) and the
errors of Example 5.6 (Table 5.8)."""
import math
import os

import numpy as np

import oracle as O
from paper_2208_06588_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")
S5 = math.sqrt(5.0)
GL_S = np.array([0.0, 0.5 - S5 / 10, 0.5 + S5 / 10, 1.0])


def _gold(name):
    rows = []
    with open(os.path.join(GOLD, name)) as f:
        for ln in f:
            ln = ln.strip()
            if ln and not ln.startswith("#"):
                rows.append(ln.split())
    return rows


def _poly_avg(coef, a, b):
    P = np.polynomial.polynomial.polyint(coef)
    return (np.polynomial.polynomial.polyval(b, P) - np.polynomial.polynomial.polyval(a, P)) / (b - a)


def _p2(**kw):
    return O.params2(**kw)


def _run2(P, wl, **kw):
    return O.run2(P, wl["h"], wl["hu"], wl["hv"], wl["b"], wl["xi"], wl["yi"], wl["xi"], wl["yi"],
                  **kw)


def test_sweep_reproduces_polynomials_on_nonuniform_widths():
    """One sweep of the dimension-by-dimension reconstruction (Sec. 2.2 along one
    direction) on smooth data: point values at the 4 Gauss-Lobatto points of the
    middle cell are exact for quartic averages on a non-uniform stencil, and the
    derivative of b (the hybrid combination of the candidate derivatives) is
    exact for a quadratic b."""
    wid = np.array([0.011, 0.009, 0.010, 0.012, 0.0085])
    e = np.concatenate([[0.0], np.cumsum(wid)]) - wid[0] - wid[1]
    rng = np.random.default_rng(3)
    quart = [rng.normal(size=5) * np.array([1, 10, 100, 1e3, 1e4]) for _ in range(5)]
    quad = rng.normal(size=3) * np.array([1, 10, 100])
    avg = [np.array([_poly_avg(c, e[k], e[k + 1]) for k in range(5)]) for c in quart]
    bav = np.array([_poly_avg(quad, e[k], e[k + 1]) for k in range(5)])
    h5, mx5, my5, ext5 = avg[0], avg[1], avg[2], avg[3]
    e5 = h5 + bav
    out, cls = O.sweep2(wid, e5, mx5, my5, h5, bav, wid.max(), eps=1e3, ext5=ext5)
    assert cls == 0
    pts = GL_S * wid[2]
    pv = np.polynomial.polynomial.polyval
    for v, c in ((0, quart[0]), (1, quart[1]), (2, quart[2]), (5, quart[3]), (3, quad)):
        exact = pv(pts, c)
        assert np.abs(out[v] - exact).max() < 1e-9 * max(1.0, np.abs(exact).max()), v
    dq = np.polynomial.polynomial.polyder(quad)
    assert np.abs(out[4] - pv(pts, dq)).max() < 1e-9 * np.abs(pv(pts, dq)).max()


def test_y_constant_data_reduce_to_the_1d_scheme():
    """Example 5.1 data extended constantly in y, the y nodes at rest: every row
    of the 2D run equals the pinned 1D oracle's run (same time steps, classes
    and state; hv stays at round-off).  Pins the x-sweep, the edge fluxes, the
    special source and the area recurrence against the 1D scheme."""
    n, ny = 64, 5
    wl = W.accuracy_1d(n)
    p1 = O.params(bc=O.BC_PERIODIC, mesh=O.MESH_SINE, mesh_A=0.05, mesh_k=1.0,
                  mesh_omega=math.pi, cfl=0.6, weno_eps=wl["weno_eps"])
    r1 = O.run(p1, wl["h"], wl["hu"], wl["b"], wl["x"], wl["xi"], t_end=0.1)
    assert r1["status"] == 0
    yi = W.uniform_nodes(ny, 0.0, 1.0)
    P = _p2(cfl=0.6, weno_eps=wl["weno_eps"], Ax=0.05, kx=1.0, omx=math.pi, Ay=0.0)
    tile = lambda a: np.tile(np.asarray(a), (ny, 1))
    r2 = O.run2(P, tile(wl["h"]), tile(wl["hu"]), np.zeros((ny, n)), tile(wl["b"]), wl["xi"], yi,
                wl["xi"], yi, t_end=0.1)
    assert r2["status"] == 0 and r2["steps"] == r1["stats"].steps
    assert tuple(r2["n_class"]) == tuple(ny * c for c in r1["stats"].n_class)
    for k in ("h", "hu", "b"):
        assert np.abs(r2[k] - r1[k][None, :]).max() < 1e-12 * max(1.0, np.abs(r1[k]).max()), k
    assert np.abs(r2["hv"]).max() < 1e-12
    assert np.abs(r2["x"] - r1["x"]).max() < 1e-15 and np.array_equal(r2["y"], yi)


def test_transposition_symmetry():
    """Exchanging the roles of x and y (state transposed, hu and hv swapped, mesh
    parameters swapped) transposes the result.  With a large epsilon in the
    weights every cell is smooth, both sweeps are linear and commute, and the
    symmetry holds to round-off; it pins the y-direction terms (fluxes, source,
    node motion) against the x-direction ones on a non-square grid."""
    nx, ny = 20, 24
    xi, yi = W.uniform_nodes(nx, 0.0, 1.0), W.uniform_nodes(ny, 0.0, 1.0)
    tp = 2 * math.pi
    f = lambda g: W.cell_averages_2d(g, xi, yi)
    b = f(lambda x, y: np.sin(tp * x) + 0.5 * np.cos(tp * y))
    h = f(lambda x, y: 10.0 + np.exp(np.sin(tp * x)) * np.cos(tp * y))
    hu = f(lambda x, y: np.sin(np.cos(tp * x)) * np.sin(tp * y))
    hv = f(lambda x, y: 0.7 * np.cos(tp * x) * np.cos(np.sin(tp * y)))
    mx = dict(A=0.03, k=1.0, om=2 * math.pi / 0.05)
    my = dict(A=0.02, k=2.0, om=4 * math.pi / 0.05)
    Pa = _p2(cfl=0.5, weno_eps=1e6, Ax=mx["A"], kx=mx["k"], omx=mx["om"], Ay=my["A"], ky=my["k"],
             omy=my["om"])
    Pb = _p2(cfl=0.5, weno_eps=1e6, Ax=my["A"], kx=my["k"], omx=my["om"], Ay=mx["A"], ky=mx["k"],
             omy=mx["om"])
    ra = O.run2(Pa, h, hu, hv, b, xi, yi, xi, yi, max_steps=12)
    rb = O.run2(Pb, h.T, hv.T, hu.T, b.T, yi, xi, yi, xi, max_steps=12)
    assert ra["status"] == 0 and rb["status"] == 0
    assert ra["n_class"][1] == ra["n_class"][2] == 0
    for ka, kb in (("h", "h"), ("hu", "hv"), ("hv", "hu"), ("b", "b")):
        d = np.abs(ra[ka] - rb[kb].T).max()
        assert d < 1e-12 * max(1.0, np.abs(ra[ka]).max()), (ka, d)
    assert np.abs(ra["x"] - rb["y"]).max() < 1e-15 and np.abs(ra["y"] - rb["x"]).max() < 1e-15


def test_constant_state_preserved_under_mesh_motion():
    """A constant state over a flat bottom stays constant while both directions
    of the mesh move (the discrete GCL of eq. (3.15) with the area recurrence),
    periodic and transmissive boundaries alike."""
    for bcy in (O.BC_PERIODIC, O.BC_TRANSMISSIVE):
        nx, ny = 16, 12
        xi, yi = W.uniform_nodes(nx, 0.0, 1.0), W.uniform_nodes(ny, 0.0, 1.0)
        z = np.zeros((ny, nx))
        P = _p2(cfl=0.5, Ax=0.03, kx=1.0, omx=40.0, Ay=0.02, ky=1.0, omy=80.0, bcy=bcy)
        r = O.run2(P, z + 2.0, z + 0.3, z - 0.2, z, xi, yi, xi, yi, max_steps=25)
        assert r["status"] == 0 and r["steps"] == 25
        assert np.abs(r["x"] - xi).max() > 1e-3 and np.abs(r["y"] - yi).max() > 1e-3
        assert np.abs(r["h"] - 2.0).max() < 1e-13
        assert np.abs(r["hu"] - 0.3).max() < 1e-13 and np.abs(r["hv"] + 0.2).max() < 1e-13
        assert np.abs(r["b"]).max() < 1e-15


def test_mass_and_bottom_are_conserved():
    """Periodic boundaries: sum over cells of area x eta and of area x b are
    constant (the flux form of eq. (3.14) telescopes)."""
    wl = W.accuracy_2d(25)
    P = _p2(cfl=0.6, Ax=wl["Ax"], kx=1.0, omx=wl["omx"], Ay=wl["Ay"], ky=1.0, omy=wl["omy"])
    r = _run2(P, wl, max_steps=30)
    assert r["status"] == 0
    m = r["mass"]
    assert abs(m[2] - m[0]) < 1e-14 * abs(m[0])
    assert abs(m[3] - m[1]) < 1e-13


def test_still_water_table_5_12():
    """Example 5.11 (b = 0.8 exp(-50 r^2), h + b = 1, at rest) on 100 x 100
    moving cells to t = 0.1: the still-water state is kept at round-off, as
    Table 5.12 prints for the special source-term scheme (errors near 1e-15)."""
    wl = W.still_water_2d(100)
    P = _p2(cfl=0.6, Ax=wl["Ax"], kx=1.0, omx=wl["omx"], Ay=wl["Ay"], ky=1.0, omy=wl["omy"])
    r = _run2(P, wl, t_end=wl["t_end"])
    assert r["status"] == 0 and abs(r["t"] - 0.1) < 1e-15
    paper = [float(v) for row in _gold("paper_tables.txt") if row[0] == "table5.12"
             for v in row[1:]]
    err = [np.abs(r["h"] + r["b"] - 1.0), np.abs(r["hu"]), np.abs(r["hv"])]
    got = [e.mean() for e in err] + [e.max() for e in err]
    for g, p in zip(got, paper):
        assert g < 10 * p, (got, paper)


def test_accuracy_example_5_6_against_table_5_8():
    """Example 5.6 at 25 x 25 and 50 x 50 (CFL 0.6, t = 0.05): the L1 errors
    of h + b, hu, hv against a 200 x 200 oracle run (averaged onto the coarse
    cells) are within 30 % of Table 5.8's, and so the orders at the coarse end
    (2.6, 3.4, 2.8 in the paper) are reproduced."""
    ref = np.array([[float(v) for v in row] for row in _gold("ex56_reference.txt")])
    ref = ref.T.reshape(3, 50, 50)
    paper = {int(r[1]): [float(v) for v in r[3:]] for r in _gold("paper_tables.txt")
             if r[0] == "table5.8"}
    errs = {}
    for n in (25, 50):
        wl = W.accuracy_2d(n)
        P = _p2(cfl=0.6, Ax=wl["Ax"], kx=1.0, omx=wl["omx"], Ay=wl["Ay"], ky=1.0, omy=wl["omy"])
        r = _run2(P, wl, t_end=wl["t_end"])
        assert r["status"] == 0
        f = 50 // n
        rc = ref.reshape(3, n, f, n, f).mean(axis=(2, 4))
        got = [r["h"] + r["b"], r["hu"], r["hv"]]
        errs[n] = [float(np.abs(g - c).mean()) for g, c in zip(got, rc)]
        for e, p in zip(errs[n], paper[n]):
            assert 0.7 < e / p < 1.3, (n, errs[n], paper[n])
    for a, b in zip(errs[25], errs[50]):
        assert math.log2(a / b) > 2.3
