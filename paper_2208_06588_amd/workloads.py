"""Seeded synthetic inputs shaped like the paper's 1D tests.

This module only builds initial data (nodes and cell averages of analytic
initial conditions).  It holds none of the scheme's arithmetic, imports
nothing else from the package, and serves both the GPU path and the oracle.

Cell averages use the 5-point Gauss-Legendre rule on each cell, with cells
split at the breakpoints of piecewise-defined data.
"""
from __future__ import annotations

import math

import numpy as np

G = 9.812  # gravitational constant used throughout Sec. 5

_GL5_X = np.array([-0.9061798459386640, -0.5384693101056831, 0.0,
                   0.5384693101056831, 0.9061798459386640])
_GL5_W = np.array([0.2369268850561891, 0.4786286704993665, 0.5688888888888889,
                   0.4786286704993665, 0.2369268850561891])


def uniform_nodes(n: int, x0: float, x1: float) -> np.ndarray:
    return x0 + (x1 - x0) * (np.arange(n + 1, dtype=np.float64) / n)


def cell_averages(f, nodes: np.ndarray, breaks=()) -> np.ndarray:
    """Average of f over each cell [nodes[j], nodes[j+1]] (5-point Gauss-Legendre,
    cells containing a breakpoint are split there)."""
    return interval_averages(lambda xs, idx: f(xs), nodes[:-1], nodes[1:], breaks)


def interval_averages(f, a: np.ndarray, b: np.ndarray, breaks=()) -> np.ndarray:
    """Average over [a_j, b_j] of f(x, j) (f gets an (m, 5) array of points and
    the (m,) cell indices), 5-point Gauss-Legendre, split at breakpoints."""

    def gl(lo, hi, idx):
        mid = 0.5 * (lo + hi)
        half = 0.5 * (hi - lo)
        xs = mid[:, None] + half[:, None] * _GL5_X[None, :]
        return (f(xs, idx) * _GL5_W[None, :]).sum(axis=1) * half

    integ = gl(a, b, np.arange(a.size))
    for c in breaks:
        idx = np.nonzero((a < c) & (c < b))[0]
        if idx.size:
            cc = np.full(idx.size, c)
            integ[idx] = gl(a[idx], cc, idx) + gl(cc, b[idx], idx)
    return integ / (b - a)


# --------------------------------------------------------------------------
# Example 5.1 (accuracy test) and the smooth periodic parity case
# --------------------------------------------------------------------------
def accuracy_1d(n: int = 200, mesh: str = "sine"):
    """[0,1] periodic; b = sin^2(pi x), h = 5 + exp(cos 2 pi x), hu = sin(cos 2 pi x)
    (eq. (5.3)).  mesh='sine': X = xi + 0.05 sin(2 pi xi) sin(pi t);
    mesh='paper': eq. (5.1) with t_end = 0.1."""
    xi = uniform_nodes(n, 0.0, 1.0)
    b = cell_averages(lambda x: np.sin(np.pi * x) ** 2, xi)
    h = cell_averages(lambda x: 5.0 + np.exp(np.cos(2 * np.pi * x)), xi)
    hu = cell_averages(lambda x: np.sin(np.cos(2 * np.pi * x)), xi)
    if mesh == "sine":
        m = dict(mesh="sine", mesh_A=0.05, mesh_k=1.0, mesh_omega=math.pi)
    else:
        m = dict(mesh="paper", mesh_A=1.0, mesh_k=0.0, mesh_omega=2 * math.pi / 0.1)
    return dict(xi=xi, x=xi.copy(), h=h, hu=hu, b=b, bc="periodic", t_end=0.1, cfl=0.6,
                weno_eps=1e-6, **m)


# --------------------------------------------------------------------------
# Example 5.3 (still water)
# --------------------------------------------------------------------------
def still_water_1d(n: int = 200, bottom: str = "smooth", t_end: float = 0.5):
    """[0,10]; b = 5 exp(-0.4 (x-5)^2) (eq. (5.6)) or 4 on [4,8] (eq. (5.7));
    h + b = 10, hu = 0; moving mesh eq. (5.1); transmissive boundaries."""
    xi = uniform_nodes(n, 0.0, 10.0)
    if bottom == "smooth":
        bf = lambda x: 5.0 * np.exp(-0.4 * (x - 5.0) ** 2)
        br = ()
    else:
        bf = lambda x: np.where((x >= 4.0) & (x <= 8.0), 4.0, 0.0)
        br = (4.0, 8.0)
    b = cell_averages(bf, xi, br)
    h = cell_averages(lambda x: 10.0 - bf(x), xi, br)
    hu = np.zeros(n)
    return dict(xi=xi, x=xi.copy(), h=h, hu=hu, b=b, bc="transmissive", t_end=t_end, cfl=0.6,
                weno_eps=1e-6, mesh="paper", mesh_A=1.0, mesh_k=0.0,
                mesh_omega=2 * math.pi / t_end)


# --------------------------------------------------------------------------
# Example 5.2, Moses's second problem (dry bed in the middle, flat bottom)
# --------------------------------------------------------------------------
def moses2_1d(n: int = 200, t_end: float = 1.0):
    xi = uniform_nodes(n, -300.0, 300.0)
    hf = lambda x: np.where(np.abs(x) < 70.0, 0.0, 10.0)
    h = cell_averages(hf, xi, (-70.0, 70.0))
    return dict(xi=xi, x=xi.copy(), h=h, hu=np.zeros(n), b=np.zeros(n), bc="transmissive",
                t_end=t_end, cfl=0.08, weno_eps=1e-6, mesh="paper", mesh_A=1.0, mesh_k=0.0,
                mesh_omega=2 * math.pi / t_end)


# --------------------------------------------------------------------------
# Example 5.5, dam break over a rectangular bump (projected bottom)
# --------------------------------------------------------------------------
def dam_break_bump_1d(n: int = 104, t_end: float = 15.0):
    """[0, 1500]; b = 8 on [562.5, 937.5], 0 elsewhere (eq. (5.12)); hu = 0,
    h + b = 20 for x <= 750 and 15 beyond (eq. (5.13)); transmissive.  The
    bottom is the projection of eq. (3.16) of that step onto the moving cells
    (bottom 'step', parameters (8, 562.5, 937.5)), and the nodes follow the
    quartic map of eq. (5.14) ('aligned': its roots include the two jump points).
    n must be a multiple of 8: then 562.5 = 3L/8, 750 and 937.5 = 5L/8 are nodes
    (the example's 100 cells would put the jump points inside cells)."""
    if n % 8:
        raise ValueError("n must be a multiple of 8 for the jump points to be nodes")
    xi = uniform_nodes(n, 0.0, 1500.0)
    bf = lambda x: np.where((x >= 562.5) & (x <= 937.5), 8.0, 0.0)
    ef = lambda x: np.where(x <= 750.0, 20.0, 15.0)
    br = (562.5, 750.0, 937.5)
    b = cell_averages(bf, xi, br)
    h = cell_averages(lambda x: ef(x) - bf(x), xi, br)
    return dict(xi=xi, x=xi.copy(), h=h, hu=np.zeros(n), b=b, bc="transmissive", t_end=t_end,
                cfl=0.6, weno_eps=1e-6, mesh="aligned", mesh_A=1.0, mesh_k=0.0,
                mesh_omega=2 * math.pi / t_end, bottom_p=(8.0, 562.5, 937.5, 0.0))


# --------------------------------------------------------------------------
# Example 5.4 (LeVeque perturbation), ragged batch
# --------------------------------------------------------------------------
def _lev_bottom(x):
    return np.where(np.abs(x - 1.5) < 0.1, 0.25 * (np.cos(10 * np.pi * (x - 1.5)) + 1.0), 0.0)


def _perturbation_cells(a, b, eps_cell):
    """Cell averages of the bump bottom and of h = 1 - b + eps 1_[1.1,1.2] over
    cells [a, b]; cells away from [1.1, 1.6] hold the exact values b = 0, h = 1."""
    br = (1.1, 1.2, 1.4, 1.6)
    bb = np.zeros(a.size)
    hh = np.ones(a.size)
    sel = np.nonzero((b > 1.1) & (a < 1.6))[0]
    if sel.size:
        aa, bs, es = a[sel], b[sel], eps_cell[sel]
        bb[sel] = interval_averages(lambda x, i: _lev_bottom(x), aa, bs, br)
        hh[sel] = interval_averages(
            lambda x, i: 1.0 - _lev_bottom(x) + np.where((x >= 1.1) & (x <= 1.2), es[i][:, None], 0.0),
            aa, bs, br)
    return hh, bb


def perturbation_instance(n: int, eps: float):
    """[0,2]; bump bottom; h = 1 - b + eps on [1.1,1.2], else 1 - b; hu = 0."""
    xi = uniform_nodes(n, 0.0, 2.0)
    h, b = _perturbation_cells(xi[:-1], xi[1:], np.full(n, eps))
    return xi, h, np.zeros(n), b


def perturbation_batch(ninst: int = 4096, nmin: int = 1000, nmax: int = 20000,
                       seed: int = 2208065881, subset: int | None = None):
    """Ragged batch: cell counts uniform in [nmin, nmax], eps uniform in
    [1e-5, 1e-2] (NumPy PCG64, drawn in that order).  Packed SoA with
    cell offsets; node arrays hold ncell+1 entries per instance.  subset=k
    keeps the first k instances of the same draw.  Same values as
    perturbation_instance, computed for all instances at once."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ns = rng.integers(nmin, nmax + 1, ninst)
    eps = rng.uniform(1e-5, 1e-2, ninst)
    if subset is not None:
        ns = ns[:subset]
        eps = eps[:subset]
    ns = ns.astype(np.int64)
    cell_off = np.zeros(len(ns) + 1, dtype=np.int64)
    cell_off[1:] = np.cumsum(ns)
    inst_of_cell = np.repeat(np.arange(len(ns)), ns)
    local = np.arange(cell_off[-1]) - np.repeat(cell_off[:-1], ns)
    nn = ns[inst_of_cell].astype(np.float64)
    a = 0.0 + (2.0 - 0.0) * (local / nn)
    bnd = 0.0 + (2.0 - 0.0) * ((local + 1) / nn)
    hh, bb = _perturbation_cells(a, bnd, eps[inst_of_cell])
    xi = np.concatenate([uniform_nodes(int(n), 0.0, 2.0) for n in ns])
    return dict(cell_off=cell_off, xi=xi, x=xi.copy(), h=hh, hu=np.zeros(cell_off[-1]), b=bb,
                bc="transmissive", t_end=0.2, cfl=0.6, weno_eps=1e-9, mesh="sine", mesh_A=0.05,
                mesh_k=1.0, mesh_omega=math.pi, eps=eps)


def pack(instances, **meta):
    ns = np.array([len(h) for (_, h, _, _) in instances], dtype=np.int64)
    cell_off = np.zeros(len(ns) + 1, dtype=np.int64)
    cell_off[1:] = np.cumsum(ns)
    xi = np.concatenate([i[0] for i in instances])
    h = np.concatenate([i[1] for i in instances])
    hu = np.concatenate([i[2] for i in instances])
    b = np.concatenate([i[3] for i in instances])
    return dict(cell_off=cell_off, xi=xi, x=xi.copy(), h=h, hu=hu, b=b, **meta)


# --------------------------------------------------------------------------
# 1D analogue of Example 5.10 (parabolic basin), wet/dry, fluid-following mesh
# --------------------------------------------------------------------------
def bowl_1d(n: int = 1 << 24, h0: float = 10.0, a: float = 3000.0, r0: float | None = None):
    """[-2a, 2a]; b = h0 (x/a)^2; h from eq. (5.22) at t = 0 restricted to a
    line (zero outside the wet region); hu = 0; transmissive boundaries."""
    if r0 is None:
        r0 = 0.8 * a
    A = (a ** 4 - r0 ** 4) / (a ** 4 + r0 ** 4)
    xi = uniform_nodes(n, -2 * a, 2 * a)
    bf = lambda x: h0 * (x / a) ** 2
    hf = lambda x: np.maximum(0.0, h0 * (math.sqrt(1 - A * A) / (1 - A)
                                         - (x / a) ** 2 * (1 - A * A) / (1 - A) ** 2))
    b = cell_averages(bf, xi)
    h = cell_averages(hf, xi)
    return dict(xi=xi, x=xi.copy(), h=h, hu=np.zeros(n), b=b, bc="transmissive", cfl=0.08,
                weno_eps=1e-6, mesh="fluid", mesh_A=0.0, mesh_k=0.0, mesh_omega=0.0)


# --------------------------------------------------------------------------
# Bathymetry-inversion batch (gauge misfit)
# --------------------------------------------------------------------------
def inversion_batch(ninst: int = 256, n: int = 65536, seed: int = 2208065883,
                    ngauge: int = 64):
    """ninst instances of n cells on [0,1]: b = sum of 8 Gaussian bumps
    (amplitudes U[0,0.3], widths U[0.01,0.05], centres U[0,1]); still water
    eta = 1 plus a Gaussian hump 0.05 (centre U[0.25,0.75]); hu = 0;
    ngauge gauges per instance uniform in [0.02, 0.98]; also an independent
    'true' bottom for synthetic observations.  Draw order per instance:
    bottom (A, s, c), hump centre, true bottom (A, s, c), gauges."""
    import torch  # multi-threaded exp on the host; values do not depend on the thread count

    rng = np.random.Generator(np.random.PCG64(seed))
    params = []
    for _ in range(ninst):
        bot = (rng.uniform(0.0, 0.3, 8), rng.uniform(0.01, 0.05, 8), rng.uniform(0.0, 1.0, 8))
        ch = rng.uniform(0.25, 0.75)
        tru = (rng.uniform(0.0, 0.3, 8), rng.uniform(0.01, 0.05, 8), rng.uniform(0.0, 1.0, 8))
        gx = np.sort(rng.uniform(0.02, 0.98, ngauge))
        params.append((bot, ch, tru, gx))
    xi = uniform_nodes(n, 0.0, 1.0)
    a, bnd = xi[:-1], xi[1:]
    mid = 0.5 * (a + bnd)
    half = 0.5 * (bnd - a)
    xs = torch.from_numpy(mid[:, None] + half[:, None] * _GL5_X[None, :])
    wts = torch.from_numpy(_GL5_W)
    hw = torch.from_numpy(half)
    wid = torch.from_numpy(bnd - a)

    def avg(vals):  # cell averages from values at the Gauss points, per instance row
        return ((vals * wts).sum(dim=-1) * hw / wid).numpy()

    def bumps(P):  # P: list of (A, s, c) per instance -> (m, n, 5) values
        A = torch.tensor(np.stack([p[0] for p in P]))[:, :, None, None]
        sw = torch.tensor(np.stack([p[1] for p in P]))[:, :, None, None]
        c = torch.tensor(np.stack([p[2] for p in P]))[:, :, None, None]
        v = torch.zeros((len(P),) + tuple(xs.shape), dtype=torch.float64)
        z = torch.empty_like(v)
        for k in range(8):
            torch.sub(xs[None], c[:, k], out=z)
            z.div_(sw[:, k])
            z.mul_(z).neg_().exp_().mul_(A[:, k])
            v.add_(z)
        return v

    hs, bs, bts, gxs = [], [], [], []
    for c0 in range(0, ninst, 16):
        chunk = params[c0:c0 + 16]
        bv = bumps([q[0] for q in chunk])
        ch = torch.tensor([q[1] for q in chunk])[:, None, None]
        eta = 1.0 + 0.05 * torch.exp(-((xs[None] - ch) / 0.05) ** 2)
        hs.extend(avg(torch.clamp(eta - bv, min=0.0)))
        bs.extend(avg(bv))
        bts.extend(avg(bumps([q[2] for q in chunk])))
        gxs.extend(q[3] for q in chunk)
    insts = [(xi, h, np.zeros(n), b) for h, b in zip(hs, bs)]
    out = pack(insts, bc="transmissive", cfl=0.6, weno_eps=1e-6, mesh="sine", mesh_A=0.05,
               mesh_k=1.0, mesh_omega=math.pi)
    out["b_true"] = np.concatenate(bts)
    out["gauge_x"] = np.concatenate(gxs)
    return out


# --------------------------------------------------------------------------
# Two dimensions (tensor-product cells): Examples 5.6 and 5.11, and the
# 2048 x 2048 smooth periodic configuration
# --------------------------------------------------------------------------
def cell_averages_2d(f, xn: np.ndarray, yn: np.ndarray) -> np.ndarray:
    """Averages of f(x, y) over the rectangles [xn_i, xn_i+1] x [yn_j, yn_j+1]
    (5 x 5 Gauss-Legendre points per cell); array [ny, nx]."""
    xm, xh = 0.5 * (xn[1:] + xn[:-1]), 0.5 * (xn[1:] - xn[:-1])
    ym, yh = 0.5 * (yn[1:] + yn[:-1]), 0.5 * (yn[1:] - yn[:-1])
    out = np.zeros((len(ym), len(xm)))
    for a, wa in zip(_GL5_X, _GL5_W):
        X = (xm + a * xh)[None, :]
        for c, wc in zip(_GL5_X, _GL5_W):
            Y = (ym + c * yh)[:, None]
            out += 0.25 * wa * wc * f(X, Y)
    return out


def accuracy_2d(n: int = 100, t_end: float = 0.05):
    """Example 5.6 on [0,1]^2, periodic: b = sin 2 pi x + cos 2 pi y,
    h = 10 + exp(sin 2 pi x) cos 2 pi y, hu = sin(cos 2 pi x) sin 2 pi y,
    hv = cos 2 pi x cos(sin 2 pi y); nodes moving per direction (the
    tensor-product form of eq. (5.2)): x = xi + 0.03 sin(2 pi xi) sin(2 pi t / t_end),
    y = eta + 0.02 sin(2 pi eta) sin(4 pi t / t_end)."""
    xi = uniform_nodes(n, 0.0, 1.0)
    tp = 2 * math.pi
    b = cell_averages_2d(lambda x, y: np.sin(tp * x) + np.cos(tp * y), xi, xi)
    h = cell_averages_2d(lambda x, y: 10.0 + np.exp(np.sin(tp * x)) * np.cos(tp * y), xi, xi)
    hu = cell_averages_2d(lambda x, y: np.sin(np.cos(tp * x)) * np.sin(tp * y), xi, xi)
    hv = cell_averages_2d(lambda x, y: np.cos(tp * x) * np.cos(np.sin(tp * y)), xi, xi)
    return dict(xi=xi, yi=xi.copy(), h=h, hu=hu, hv=hv, b=b, bc="periodic", t_end=t_end,
                Ax=0.03, kx=1.0, omx=2 * math.pi / t_end, Ay=0.02, ky=1.0, omy=4 * math.pi / t_end)


def still_water_2d(n: int = 100, t_end: float = 0.1):
    """Example 5.11 on [0,1]^2: b = 0.8 exp(-50 ((x-0.5)^2 + (y-0.5)^2)),
    h + b = 1, hu = hv = 0; nodes as in accuracy_2d with this t_end."""
    xi = uniform_nodes(n, 0.0, 1.0)
    bf = lambda x, y: 0.8 * np.exp(-50.0 * ((x - 0.5) ** 2 + (y - 0.5) ** 2))
    b = cell_averages_2d(bf, xi, xi)
    h = cell_averages_2d(lambda x, y: 1.0 - bf(x, y), xi, xi)
    z = np.zeros_like(h)
    return dict(xi=xi, yi=xi.copy(), h=h, hu=z, hv=z.copy(), b=b, bc="periodic", t_end=t_end,
                Ax=0.03, kx=1.0, omx=2 * math.pi / t_end, Ay=0.02, ky=1.0, omy=4 * math.pi / t_end)


def smooth_2d(n: int = 2048):
    """The 2048 x 2048 periodic configuration: b = sin 2 pi x + cos 2 pi y,
    h = 10 + exp(sin 2 pi x) cos 2 pi y, hu = sin(cos 2 pi x) sin 2 pi y,
    hv = cos 2 pi x cos(sin 2 pi y) on [0,1]^2; nodes x = xi + 0.02 sin(2 pi xi)
    sin(pi t) and y likewise (tensor-product form of its perturbation)."""
    wl = accuracy_2d(n)
    wl.update(Ax=0.02, omx=math.pi, Ay=0.02, omy=math.pi, t_end=0.0)
    return wl


def dam_break_2d(nx: int = 200, ny: int | None = None, t_end: float = 1.75, amp=(0.03, 0.02),
                 h_out: float = 0.0):
    """Example 5.9, the circular dam break on [-100, 100]^2: b = 0, h = 10 for
    r <= 60 and h_out outside (0: the example's dry bed), hu = hv = 0,
    transmissive; nodes moving per
    direction in the tensor-product form of eq. (5.2):
    x = xi + amp[0] sin(2 pi xi / 200) sin(2 pi t / t_end),
    y = eta + amp[1] sin(2 pi eta / 200) sin(4 pi t / t_end).  The cells
    cut by the dam hold the exact averages of the step."""
    ny = nx if ny is None else ny
    # nodes and averages mirror-symmetric to the bit about both axes
    xi, yi = uniform_nodes(nx, -100.0, 100.0), uniform_nodes(ny, -100.0, 100.0)
    xi, yi = 0.5 * (xi - xi[::-1]), 0.5 * (yi - yi[::-1])
    h = h_out + _disc_averages_2d(xi, yi, 60.0, 10.0 - h_out)
    h = ((h + h[:, ::-1]) + (h[::-1, :] + h[::-1, ::-1])) * 0.25
    z = np.zeros_like(h)
    return dict(xi=xi, yi=yi, h=h, hu=z, hv=z.copy(), b=z.copy(), bc="transmissive", t_end=t_end,
                Ax=amp[0], kx=1.0 / 200.0, omx=2 * math.pi / t_end, Ay=amp[1], ky=1.0 / 200.0,
                omy=4 * math.pi / t_end)


def vortex_2d(refine: int = 1, moving: bool = True, t_end: float = 2.0):
    """Example 5.7 (a quasi-stationary vortex carried at 1 m/s) on [0,4] x [0,2],
    periodic, b = 0: inside r_m = 0.45 of (1, 1) the tangential speed v_r(r) of
    the example and h = 1 - (vmax s)^2 / g exp(1 / (r^2 - r_m^2)) (in balance:
    g h' = v_r^2 / r), vmax = 0.5; u = 1 - v_r (y - 1) / r, v = v_r (x - 1) / r
    (a rotation about the centre: the example's (y - 2) and the sign of its v
    read as typos).  moving: the piecewise-uniform 110 x 70 mesh of eq. (5.17)-
    (5.18) (the last x segment 1.5 + 0.05 (i - 60), the example's (i - 1.5) read
    as a typo), translated at w = (1, 0) (eq. (5.19)); else uniform 110 x 70.
    refine = 2 halves every cell (220 x 140).  The exact solution is the initial
    vortex moved by t: on the moving mesh the initial cell averages themselves."""
    g, vmax, rm = 9.812, 0.5, 0.45
    rvm = 0.5 * math.sqrt(-2.0 + 2.0 * math.sqrt(1.0 + 4.0 * rm ** 4))
    s = abs(rvm ** 2 - rm ** 2) / (rvm * math.sqrt(2.0 * math.exp(1.0 / (rvm ** 2 - rm ** 2))))

    def fields(x, y, cx):
        dx, dy = x - cx, y - 1.0
        r2 = dx * dx + dy * dy
        inside = r2 < rm * rm
        e = np.where(inside, np.exp(1.0 / np.where(inside, r2 - rm * rm, -1.0)), 0.0)
        h = 1.0 - (vmax * s) ** 2 / g * e
        r = np.sqrt(r2)
        vr = np.where(inside, vmax * s * r / np.where(inside, rm * rm - r2, 1.0)
                      * np.sqrt(2.0 * e), 0.0)
        rr = np.where(r > 0.0, r, 1.0)
        u = 1.0 - vr * dy / rr
        v = vr * dx / rr
        return h, h * u, h * v

    if moving:
        xn = np.concatenate([0.05 * np.arange(0, 11), 0.5 + 0.02 * np.arange(1, 51),
                             1.5 + 0.05 * np.arange(1, 51)])
        yn = np.concatenate([0.05 * np.arange(0, 11), 0.5 + 0.02 * np.arange(1, 51),
                             1.5 + 0.05 * np.arange(1, 11)])
    else:
        xn, yn = uniform_nodes(110, 0.0, 4.0), uniform_nodes(70, 0.0, 2.0)
    if refine > 1:
        fine = lambda a: np.concatenate([a[:-1, None] + (a[1:] - a[:-1])[:, None]
                                         * (np.arange(refine) / refine)[None, :], ], axis=0).ravel()
        xn = np.append(fine(xn), xn[-1])
        yn = np.append(fine(yn), yn[-1])

    def averages(cx):
        out = [np.zeros((len(yn) - 1, len(xn) - 1)) for _ in range(3)]
        w = _GL5_W[:, None] * _GL5_W[None, :]
        for p in range(4):
            for q in range(4):
                xa = xn[:-1] + (xn[1:] - xn[:-1]) * (p / 4.0)
                xb = xn[:-1] + (xn[1:] - xn[:-1]) * ((p + 1) / 4.0)
                ya = yn[:-1] + (yn[1:] - yn[:-1]) * (q / 4.0)
                yb = yn[:-1] + (yn[1:] - yn[:-1]) * ((q + 1) / 4.0)
                px = 0.5 * (xa + xb)[:, None] + 0.5 * (xb - xa)[:, None] * _GL5_X[None, :]
                py = 0.5 * (ya + yb)[:, None] + 0.5 * (yb - ya)[:, None] * _GL5_X[None, :]
                for o, f in zip(out, fields(px[None, :, None, :], py[:, None, :, None], cx)):
                    o += (f * w[None, None]).sum(axis=(2, 3)) * 0.25 / 16.0
        return out

    h, hu, hv = averages(1.0)
    # exact water height at t_end on the final cells: moving mesh, the initial
    # averages; static mesh, the vortex centred at 1 + t_end (periodic in x)
    h_end = h.copy() if moving else averages(1.0 + (t_end % 4.0))[0]
    return dict(xi=xn, yi=yn, h=h, hu=hu, hv=hv, b=np.zeros_like(h), h_end=h_end,
                bc="periodic", t_end=t_end, Vx=1.0 if moving else 0.0, cfl=0.6)


def parabolic_basin_2d(n: int = 100, amp=(0.03, 0.02), periods: float = 1.0):
    """Example 5.10 (long wave in a parabolic basin) on [-4000, 4000]^2: b =
    h0 (x^2 + y^2) / a^2, h = max(0, h0 (sqrt(1 - A^2) / (1 - A) - r^2 / a^2
    (1 - A^2) / (1 - A)^2)), hu = hv = 0, h0 = 1, a = 2500, r0 = 2000, A =
    (a^4 - r0^4) / (a^4 + r0^4); the exact solution is periodic with T = 2 pi /
    kappa, kappa = sqrt(8 g h0) / a (g = 9.812), so the state at t = T is the
    initial one.  Transmissive (the water stays far inside), CFL 0.08; nodes
    moving per direction in the tensor-product form of eq. (5.2) with t_end =
    periods T.  b's cell averages are exact; h's by the 5 x 5 Gauss-Legendre
    rule on 4 x 4 sub-cells of each cell.  Trace depths at most dry_eps = 1e-3
    (a thousandth of h0) carry no discharge: with 1e-6 the thin shoreline
    layer's velocities hu / h grow without bound and the run loses positivity
    within a few steps."""
    h0, a, r0, g = 1.0, 2500.0, 2000.0, 9.812
    A = (a ** 4 - r0 ** 4) / (a ** 4 + r0 ** 4)
    kappa = math.sqrt(8.0 * g * h0) / a
    T = 2.0 * math.pi / kappa
    xi = uniform_nodes(n, -4000.0, 4000.0)
    xi = 0.5 * (xi - xi[::-1])
    x0, x1 = xi[:-1], xi[1:]
    mx = (x1 ** 3 - x0 ** 3) / (3.0 * (x1 - x0))  # cell average of x^2
    b = (h0 / a ** 2) * (mx[None, :] + mx[:, None])

    def hfun(x, y):
        r2 = x * x + y * y
        return np.maximum(0.0, h0 * (math.sqrt(1.0 - A * A) / (1.0 - A)
                                     - r2 / a ** 2 * (1.0 - A * A) / (1.0 - A) ** 2))

    sub = np.linspace(0.0, 1.0, 5)
    xs = (x0[:, None] + (x1 - x0)[:, None] * sub[None, :])  # [n, 5] sub-cell nodes
    h = np.zeros((n, n))
    for p in range(4):
        for q in range(4):
            xn = np.stack([xs[:, p], xs[:, p + 1]], axis=1)
            hx = 0.5 * (xn[:, 1] - xn[:, 0])
            cx = 0.5 * (xn[:, 1] + xn[:, 0])
            yn = np.stack([xs[:, q], xs[:, q + 1]], axis=1)
            hy = 0.5 * (yn[:, 1] - yn[:, 0])
            cy = 0.5 * (yn[:, 1] + yn[:, 0])
            px = cx[:, None] + hx[:, None] * _GL5_X[None, :]  # [n, 5]
            py = cy[:, None] + hy[:, None] * _GL5_X[None, :]
            f = hfun(px[None, :, None, :], py[:, None, :, None])  # [ny, nx, 5, 5]
            w = _GL5_W[:, None] * _GL5_W[None, :]
            h += (f * w[None, None]).sum(axis=(2, 3)) * 0.25 / 16.0
    h = ((h + h[:, ::-1]) + (h[::-1, :] + h[::-1, ::-1])) * 0.25
    z = np.zeros_like(h)
    t_end = periods * T
    return dict(xi=xi, yi=xi.copy(), h=h, hu=z, hv=z.copy(), b=b, bc="transmissive", t_end=t_end,
                T=T, Ax=amp[0], kx=1.0 / 8000.0, omx=2 * math.pi / t_end, Ay=amp[1],
                ky=1.0 / 8000.0, omy=4 * math.pi / t_end, cfl=0.08, dry_eps=1e-3)


def parabolic_basin_exact_2d(x: np.ndarray, y: np.ndarray, t: float) -> np.ndarray:
    """Cell averages of Example 5.10's exact depth at time t on the cells
    [x_i, x_i+1] x [y_j, y_j+1] ([ny, nx]): 5 x 5 Gauss-Legendre on 4 x 4
    sub-cells (the shoreline's kink is the only non-smooth part)."""
    h0, a, r0, g = 1.0, 2500.0, 2000.0, 9.812
    A = (a ** 4 - r0 ** 4) / (a ** 4 + r0 ** 4)
    kappa = math.sqrt(8.0 * g * h0) / a
    c = 1.0 - A * math.cos(kappa * t)
    hf = lambda X, Y: np.maximum(0.0, h0 * (math.sqrt(1.0 - A * A) / c
                                            - (X * X + Y * Y) / a ** 2 * (1.0 - A * A) / c ** 2))
    x, y = np.asarray(x), np.asarray(y)
    out = np.zeros((len(y) - 1, len(x) - 1))
    w = _GL5_W[:, None] * _GL5_W[None, :]
    for p in range(4):
        for q in range(4):
            xa = x[:-1] + (x[1:] - x[:-1]) * (p / 4.0)
            xb = x[:-1] + (x[1:] - x[:-1]) * ((p + 1) / 4.0)
            ya = y[:-1] + (y[1:] - y[:-1]) * (q / 4.0)
            yb = y[:-1] + (y[1:] - y[:-1]) * ((q + 1) / 4.0)
            px = 0.5 * (xa + xb)[:, None] + 0.5 * (xb - xa)[:, None] * _GL5_X[None, :]
            py = 0.5 * (ya + yb)[:, None] + 0.5 * (yb - ya)[:, None] * _GL5_X[None, :]
            f = hf(px[None, :, None, :], py[:, None, :, None])
            out += (f * w[None, None]).sum(axis=(2, 3)) * 0.25 / 16.0
    return out


def _disc_area(x0: float, x1: float, y0: float, y1: float, r: float) -> float:
    """Area of the rectangle [x0, x1] x [y0, y1] inside the disc of radius r
    about the origin: the integral over x of the chord of the disc clipped to
    [y0, y1], exact on each piece between the abscissae where the clipping
    changes (the antiderivative of sqrt(r^2 - x^2) is
    (x sqrt(r^2 - x^2) + r^2 asin(x / r)) / 2)."""
    F = lambda x: 0.5 * (x * math.sqrt(max(r * r - x * x, 0.0)) + r * r * math.asin(max(-1.0, min(1.0, x / r))))
    cuts = {x0, x1}
    for y in (y0, y1):
        if abs(y) < r:
            s = math.sqrt(r * r - y * y)
            cuts.update(c for c in (-s, s) if x0 < c < x1)
    cuts.update(c for c in (-r, r) if x0 < c < x1)
    pts = sorted(cuts)
    area = 0.0
    for a, b in zip(pts[:-1], pts[1:]):
        xm = 0.5 * (a + b)
        if abs(xm) >= r:
            continue
        s = math.sqrt(r * r - xm * xm)
        top_arc, bot_arc = s < y1, -s > y0
        if min(y1, s) <= max(y0, -s):
            continue
        arc = F(b) - F(a)
        area += (arc if top_arc else y1 * (b - a)) - (-arc if bot_arc else y0 * (b - a))
    return area


def _disc_averages_2d(xn: np.ndarray, yn: np.ndarray, r: float, value: float) -> np.ndarray:
    """Cell averages [ny, nx] of value inside the disc of radius r about the
    origin and 0 outside."""
    out = np.zeros((len(yn) - 1, len(xn) - 1))
    for j in range(len(yn) - 1):
        y0, y1 = float(yn[j]), float(yn[j + 1])
        for i in range(len(xn) - 1):
            x0, x1 = float(xn[i]), float(xn[i + 1])
            near = min(x0 * x0 if x0 > 0 else (x1 * x1 if x1 < 0 else 0.0), 1e300) + \
                (y0 * y0 if y0 > 0 else (y1 * y1 if y1 < 0 else 0.0))
            far = max(x0 * x0, x1 * x1) + max(y0 * y0, y1 * y1)
            if far <= r * r:
                out[j, i] = value
            elif near < r * r:
                out[j, i] = value * _disc_area(x0, x1, y0, y1, r) / ((x1 - x0) * (y1 - y0))
    return out
