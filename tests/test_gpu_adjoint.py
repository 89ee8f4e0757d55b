"""GPU discrete adjoint (through the C ABI) against the oracle's tape adjoint and
against central finite differences of the GPU forward run (frozen step sizes)."""
import math

import numpy as np
import pytest
import torch

import oracle as O
from paper_2208_06588_amd import alew, workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    torch.cuda.set_device(0)
    return torch.device("cuda", 0)


def _t(a, dev):
    return torch.tensor(np.asarray(a), dtype=torch.float64, device=dev)


def _case(kind, n):
    """Small instances that exercise different switches of the scheme."""
    xi = W.uniform_nodes(n, 0.0, 1.0)
    xc = 0.5 * (xi[1:] + xi[:-1])
    if kind == "smooth":  # bumps under still water with a hump
        b = 0.2 * np.exp(-((xc - 0.3) / 0.05) ** 2) + 0.1 * np.exp(-((xc - 0.7) / 0.03) ** 2)
        eta = 1.0 + 0.05 * np.exp(-((xc - 0.5) / 0.05) ** 2)
        h, hu = eta - b, 0.02 * np.sin(2 * np.pi * xc)
        bc = "transmissive"
    elif kind == "step":  # steps in bottom and surface: transition / non-smooth classes
        b = np.where((xc > 0.4) & (xc < 0.6), 0.3, 0.0)
        h = np.where(xc < 0.25, 1.3, 1.0) - b
        hu = np.zeros(n)
        bc = "periodic"
    else:  # shallow wet/dry: limiter and dry cut-offs
        b = np.zeros(n)
        h = np.where(np.abs(xc - 0.5) < 0.1, 0.0, 0.5) + 1e-3 * np.sin(7 * xc) ** 2
        h = np.where(np.abs(xc - 0.5) < 0.08, 0.0, h)
        hu = np.where(xc < 0.5, 0.05, -0.05) * (h > 0)
        bc = "transmissive"
    return xi, h, hu, b, bc


def _params(bc, cfl=0.6, hydro=False):
    g = alew.params(bc=bc, mesh="sine", mesh_A=0.05, mesh_k=1.0, mesh_omega=math.pi, cfl=cfl,
                    flags=alew.F_HYDROSTATIC if hydro else 0)
    o = O.params(bc=dict(periodic=O.BC_PERIODIC, transmissive=O.BC_TRANSMISSIVE)[bc],
                 mesh=O.MESH_SINE, mesh_A=0.05, mesh_k=1.0, mesh_omega=math.pi, cfl=cfl,
                 flags=O.FLAG_HYDROSTATIC if hydro else 0)
    return g, o


# Errors are measured cell by cell, |g - o| / max(1, |o|), so that cells with a
# gradient of order one are held to the bar however large the gradient is at a
# wet/dry front elsewhere.
# The 560-cell cases span three tiles of the reverse-stage kernel (250 owned
# cells each), with gauges dense enough that the adjoint is nonzero across the
# tile seams.
# (The wet/dry case on 560 cells runs at CFL 0.08, the positivity bound of the
# scheme; at 0.3 its forward run reaches negative depths.)
# Each case runs with the special source term and with the hydrostatic
# reconstruction (hydro=True).
@pytest.mark.parametrize("hydro", [False, True])
@pytest.mark.parametrize("kind,ckpt,tol,n,nsteps,ng,cfl", [
    ("smooth", 3, 1e-11, 64, 7, 6, 0.3), ("step", 2, 1e-11, 64, 7, 6, 0.3),
    ("wetdry", 16, 1e-11, 64, 7, 6, 0.3), ("smooth", 3, 1e-11, 560, 8, 40, 0.3),
    ("step", 4, 1e-11, 560, 8, 40, 0.3), ("wetdry", 5, 1e-11, 560, 8, 40, 0.08)])
def test_adjoint_matches_oracle(dev, kind, ckpt, tol, n, nsteps, ng, cfl, hydro):
    xi, h, hu, b, bc = _case(kind, n)
    gp, op = _params(bc, cfl=cfl, hydro=hydro)
    if hydro and kind == "wetdry" and n == 560:
        # the hydrostatic form also divides by the starred depths h* = max(0,
        # eta - max(b-, b+)), which at the wet/dry front are far below the trace
        # depths (bounded only by dry_eps = 1e-8): the momentum flux carries
        # hu^2 / h*, whose derivatives hu / h*^2 reach ~1e16 and cancel to
        # gradients of ~1e8 at the front, so the round-off of the two evaluation
        # orders is amplified by ~1e8 relative to the result there
        tol = 1e-8
    # step sizes: those the CFL rule picks in the oracle's own run
    r = O.run(op, h, hu, b, xi, xi, max_steps=1)
    dts = np.full(nsteps, r["stats"].dt_max)
    rng = np.random.default_rng(11)
    gx = np.sort(rng.uniform(0.03, 0.97, ng))
    gbar = rng.normal(size=ng)
    gh_o, dh_o, dhu_o, db_o, st = O.adjoint(op, h, hu, b, xi, xi, dts, gx, gbar)
    assert st == 0
    ctx = alew.Context(n, 1)
    T = {k: _t(v, dev) for k, v in dict(h=h, hu=hu, b=b, x=xi, xi=xi, dts=dts, gx=gx, gb=gbar).items()}
    gh = torch.zeros(ng, dtype=torch.float64, device=dev)
    dh, dhu, db = (torch.zeros(n, dtype=torch.float64, device=dev) for _ in range(3))
    ctx.adjoint(gp, [0, n], T["h"], T["hu"], T["b"], T["x"], T["xi"], nsteps, T["dts"], ng, T["gx"],
                gh, T["gb"], dh, dhu, db, ckpt_every=ckpt)
    torch.cuda.synchronize()
    np.testing.assert_allclose(gh.cpu().numpy(), gh_o, rtol=0, atol=1e-12)
    for name, g, o in (("h", dh, dh_o), ("hu", dhu, dhu_o), ("b", db, db_o)):
        g = g.cpu().numpy()
        scale = max(1.0, np.abs(o).max())
        err = np.abs(g - o).max() / scale
        cell = np.abs(g - o) / np.maximum(1.0, np.abs(o))
        big = cell > 1e-11
        print(f"adjoint {kind} n={n} hydro={hydro} d/d{name}: per-cell max {cell.max():.2e} "
              f"(cells above 1e-11: {int(big.sum())}, their |grad| "
              f"{np.sort(np.abs(o[big]))[:4]}..{np.abs(o[big]).max() if big.any() else 0:.2e}, "
              f"median |grad| {np.median(np.abs(o)):.2e}), global-scale {err:.2e}, "
              f"max |grad| {np.abs(o).max():.2e}", flush=True)
        assert err <= tol, err
        assert cell.max() <= tol, cell.max()


def test_adjoint_on_the_jump_aligned_mesh(dev):
    """The quartic map of eq. (5.14) with its interior roots at 0.375 and 0.625
    on [0, 1] (nodes 24 and 40 of 64; bottom_p[1], bottom_p[2]), the bottom
    evolved by eq. (3.17): the GPU adjoint against the oracle's tape adjoint,
    cell by cell at 1e-11."""
    n, nsteps, ng = 64, 7, 6
    xi, h, hu, b, bc = _case("step", n)
    bp = (0.0, 0.375, 0.625, 0.0)
    gp = alew.params(bc=bc, mesh="aligned", mesh_A=1.0, mesh_k=0.0, mesh_omega=math.pi,
                     cfl=0.3, bottom_p=bp)
    op = O.params(bc=O.BC_PERIODIC, mesh=O.MESH_ALIGNED, mesh_A=1.0, mesh_k=0.0,
                  mesh_omega=math.pi, cfl=0.3, bottom_p=bp)
    r = O.run(op, h, hu, b, xi, xi, max_steps=1)
    dts = np.full(nsteps, r["stats"].dt_max)
    rng = np.random.default_rng(12)
    gx = np.sort(rng.uniform(0.03, 0.97, ng))
    gbar = rng.normal(size=ng)
    gh_o, dh_o, dhu_o, db_o, st = O.adjoint(op, h, hu, b, xi, xi, dts, gx, gbar)
    assert st == 0
    ctx = alew.Context(n, 1)
    T = {k: _t(v, dev) for k, v in dict(h=h, hu=hu, b=b, x=xi, xi=xi, dts=dts, gx=gx, gb=gbar).items()}
    gh = torch.zeros(ng, dtype=torch.float64, device=dev)
    dh, dhu, db = (torch.zeros(n, dtype=torch.float64, device=dev) for _ in range(3))
    ctx.adjoint(gp, [0, n], T["h"], T["hu"], T["b"], T["x"], T["xi"], nsteps, T["dts"], ng, T["gx"],
                gh, T["gb"], dh, dhu, db, ckpt_every=3)
    torch.cuda.synchronize()
    np.testing.assert_allclose(gh.cpu().numpy(), gh_o, rtol=0, atol=1e-12)
    for g, o in ((dh, dh_o), (dhu, dhu_o), (db, db_o)):
        cell = np.abs(g.cpu().numpy() - o) / np.maximum(1.0, np.abs(o))
        assert cell.max() <= 1e-11, cell.max()


def _accuracy_case(n):
    # Example 5.1 data: strongly varying, so the hybrid weights stay in the
    # linear class and the map is smooth at the scale of the FD step (with
    # nearly flat water the WENO-Z weights vary on the scale of weno_eps = 1e-6,
    # below which central differences with step 1e-6 are not accurate).
    wl = W.accuracy_1d(n)
    return wl["xi"], wl["h"], wl["hu"], wl["b"], "periodic"


@pytest.mark.parametrize("hydro", [False, True])
def test_adjoint_against_gpu_finite_differences(dev, hydro):
    """Central differences of the GPU forward (alew_run with the same frozen
    steps) along random directions of (h0, hu0, b0).  The hydrostatic form
    takes max(b-, b+) at every face, which has no derivative where the two
    bottom traces tie (bit for bit at the symmetry points of this bottom):
    there the directions are in (h0, hu0) only."""
    n, nsteps, ng = 96, 6, 8
    xi, h, hu, b, bc = _accuracy_case(n)
    gp, op = _params(bc, hydro=hydro)
    dts = np.full(nsteps, 5e-4)  # CFL about 0.45 at these speeds
    rng = np.random.default_rng(5)
    gx = np.sort(rng.uniform(0.03, 0.97, ng))
    gbar = rng.normal(size=ng)
    ctx = alew.Context(n, 1)
    T = {k: _t(v, dev) for k, v in dict(h=h, hu=hu, b=b, x=xi, xi=xi, dts=dts, gx=gx, gb=gbar).items()}
    gh = torch.zeros(ng, dtype=torch.float64, device=dev)
    dh, dhu, db = (torch.zeros(n, dtype=torch.float64, device=dev) for _ in range(3))
    ctx.adjoint(gp, [0, n], T["h"], T["hu"], T["b"], T["x"], T["xi"], nsteps, T["dts"], ng, T["gx"],
                gh, T["gb"], dh, dhu, db, ckpt_every=4)

    def J(vh, vm, vb, eps):
        hh = T["h"] + eps * vh
        mm = T["hu"] + eps * vm
        bb = T["b"] + eps * vb
        x = T["x"].clone()
        ctx.run(gp, [0, n], hh, mm, bb, x, T["xi"], max_steps=[nsteps], dts=T["dts"],
                dts_stride=nsteps)
        idx = torch.clamp(torch.searchsorted(x, T["gx"], right=True) - 1, 0, n - 1)
        return float(torch.dot(T["gb"], hh[idx]))

    for _ in range(4):
        vh, vm, vb = (torch.randn(n, dtype=torch.float64, device=dev) for _ in range(3))
        if hydro:
            vb = torch.zeros_like(vb)
        e = 1e-6
        fd = (J(vh, vm, vb, e) - J(vh, vm, vb, -e)) / (2 * e)
        ad = float(torch.dot(dh, vh) + torch.dot(dhu, vm) + torch.dot(db, vb))
        assert abs(fd - ad) <= 1e-6 * max(1.0, abs(ad)), (fd, ad)


def test_checkpoint_interval_does_not_change_the_gradient(dev):
    n, nsteps, ng = 80, 9, 5
    xi, h, hu, b, bc = _case("step", n)
    gp, _ = _params(bc)
    dts = np.full(nsteps, 1e-3)
    rng = np.random.default_rng(2)
    T = {k: _t(v, dev) for k, v in dict(h=h, hu=hu, b=b, x=xi, xi=xi, dts=dts,
                                         gx=np.sort(rng.uniform(0.05, 0.95, ng)),
                                         gb=rng.normal(size=ng)).items()}
    ctx = alew.Context(n, 1)
    outs = []
    for ck in (1, 4, 9, 16):
        gh = torch.zeros(ng, dtype=torch.float64, device=dev)
        g3 = [torch.zeros(n, dtype=torch.float64, device=dev) for _ in range(3)]
        ctx.adjoint(gp, [0, n], T["h"], T["hu"], T["b"], T["x"], T["xi"], nsteps, T["dts"], ng,
                    T["gx"], gh, T["gb"], *g3, ckpt_every=ck)
        outs.append(torch.cat(g3).cpu().numpy())
    for o in outs[1:]:
        np.testing.assert_allclose(o, outs[0], rtol=0, atol=1e-13 * np.abs(outs[0]).max())


def test_batched_adjoint_equals_single_instances(dev):
    """A ragged batch gives each instance the gradient it has on its own."""
    cases = [_case("smooth", 40), _case("step", 57), _case("smooth", 33)]
    nsteps, ng = 5, 4
    insts = [(xi, h, hu, b) for (xi, h, hu, b, bc) in cases]
    gp, _ = _params("transmissive")
    bt = W.pack(insts)
    off = bt["cell_off"]
    S = int(off[-1])
    ninst = len(insts)
    rng = np.random.default_rng(8)
    gx = np.concatenate([np.sort(rng.uniform(0.05, 0.95, ng)) for _ in range(ninst)])
    gb = rng.normal(size=ninst * ng)
    dts = np.full(ninst * nsteps, 1.2e-3)
    T = {k: _t(v, dev) for k, v in dict(h=bt["h"], hu=bt["hu"], b=bt["b"], x=bt["x"], xi=bt["xi"],
                                         dts=dts, gx=gx, gb=gb).items()}
    ctx = alew.Context(S, ninst)
    gh = torch.zeros(ninst * ng, dtype=torch.float64, device=dev)
    g3 = [torch.zeros(S, dtype=torch.float64, device=dev) for _ in range(3)]
    ctx.adjoint(gp, off, T["h"], T["hu"], T["b"], T["x"], T["xi"], nsteps, T["dts"], ng, T["gx"], gh,
                T["gb"], *g3, ckpt_every=2)
    for i in range(ninst):
        a, e = int(off[i]), int(off[i + 1])
        c1 = alew.Context(e - a, 1)
        gh1 = torch.zeros(ng, dtype=torch.float64, device=dev)
        o3 = [torch.zeros(e - a, dtype=torch.float64, device=dev) for _ in range(3)]
        c1.adjoint(gp, [0, e - a], T["h"][a:e], T["hu"][a:e], T["b"][a:e], T["x"][a + i:e + i + 1],
                   T["xi"][a + i:e + i + 1], nsteps, T["dts"][i * nsteps:(i + 1) * nsteps], ng,
                   T["gx"][i * ng:(i + 1) * ng], gh1, T["gb"][i * ng:(i + 1) * ng], *o3,
                   ckpt_every=2)
        assert torch.equal(gh1, gh[i * ng:(i + 1) * ng])
        for k in range(3):
            scale = float(o3[k].abs().max()) or 1.0
            assert float((o3[k] - g3[k][a:e]).abs().max()) <= 1e-13 * scale


def test_adjoint_many_tiles_deterministic(dev):
    """A batch of many multi-tile instances (far more reverse-stage tiles than
    run at once): two calls agree bit for bit, and every instance has the
    gradient of its own one-instance call."""
    ninst, n, nsteps, ng = 96, 3000, 6, 8
    base = [_case("smooth", n), _case("step", n)]
    insts = [(xi, h, hu, b) for (xi, h, hu, b, bc) in (base[k % 2] for k in range(ninst))]
    gp, _ = _params("transmissive")
    bt = W.pack(insts)
    off = bt["cell_off"]
    S = int(off[-1])
    rng = np.random.default_rng(21)
    gx = np.concatenate([np.sort(rng.uniform(0.02, 0.98, ng)) for _ in range(ninst)])
    gb = rng.normal(size=ninst * ng)
    dts = np.full(ninst * nsteps, 2e-5)  # CFL about 0.2 on 3000 cells
    T = {k: _t(v, dev) for k, v in dict(h=bt["h"], hu=bt["hu"], b=bt["b"], x=bt["x"], xi=bt["xi"],
                                         dts=dts, gx=gx, gb=gb).items()}
    ctx = alew.Context(S, ninst)
    runs = []
    for _ in range(2):
        gh = torch.zeros(ninst * ng, dtype=torch.float64, device=dev)
        g3 = [torch.zeros(S, dtype=torch.float64, device=dev) for _ in range(3)]
        ctx.adjoint(gp, off, T["h"], T["hu"], T["b"], T["x"], T["xi"], nsteps, T["dts"], ng,
                    T["gx"], gh, T["gb"], *g3, ckpt_every=4)
        torch.cuda.synchronize()
        runs.append([g.cpu().numpy() for g in g3])
    for k in range(3):
        assert np.array_equal(runs[0][k], runs[1][k]), k
    c1 = alew.Context(n, 1)
    for i in range(ninst):
        a, e = int(off[i]), int(off[i + 1])
        gh1 = torch.zeros(ng, dtype=torch.float64, device=dev)
        o3 = [torch.zeros(n, dtype=torch.float64, device=dev) for _ in range(3)]
        c1.adjoint(gp, [0, n], T["h"][a:e], T["hu"][a:e], T["b"][a:e], T["x"][a + i:e + i + 1],
                   T["xi"][a + i:e + i + 1], nsteps, T["dts"][i * nsteps:(i + 1) * nsteps], ng,
                   T["gx"][i * ng:(i + 1) * ng], gh1, T["gb"][i * ng:(i + 1) * ng], *o3,
                   ckpt_every=4)
        for k in range(3):
            o = o3[k].cpu().numpy()
            scale = max(float(np.abs(o).max()), 1e-300)
            assert np.abs(o - runs[0][k][a:e]).max() <= 1e-13 * scale, (i, k)


def test_autograd_function_gradients(dev):
    """torch.autograd through the gauge map equals the direct adjoint call and
    central differences of the loss."""
    n, nsteps, ng = 72, 5, 6
    xi, h, hu, b, bc = _accuracy_case(n)
    gp, _ = _params(bc)
    rng = np.random.default_rng(21)
    T = {k: _t(v, dev) for k, v in dict(x=xi, xi=xi, dts=np.full(nsteps, 5e-4),
                                         gx=np.sort(rng.uniform(0.05, 0.95, ng))).items()}
    ctx = alew.Context(n, 1)
    G = alew.GaugeProblem(ctx, gp, [0, n], T["x"], T["xi"], nsteps, T["dts"], T["gx"], ng,
                          ckpt_every=2)
    obs = _t(rng.normal(size=ng) * 0.1 + 6.0, dev)
    h0 = _t(h, dev).requires_grad_()
    hu0 = _t(hu, dev).requires_grad_()
    b0 = _t(b, dev).requires_grad_()
    loss = 0.5 * ((G(h0, hu0, b0) - obs) ** 2).sum()
    loss.backward()
    with torch.no_grad():
        gbar = G(h0, hu0, b0) - obs
        gh = torch.zeros(ng, dtype=torch.float64, device=dev)
        d3 = [torch.zeros(n, dtype=torch.float64, device=dev) for _ in range(3)]
        ctx.adjoint(gp, [0, n], h0.detach(), hu0.detach(), b0.detach(), T["x"], T["xi"], nsteps,
                    T["dts"], ng, T["gx"], gh, gbar, *d3, ckpt_every=2)
        for a, bb in zip((h0.grad, hu0.grad, b0.grad), d3):
            assert torch.allclose(a, bb, rtol=0, atol=1e-14 * float(bb.abs().max() + 1))
        v = [torch.randn(n, dtype=torch.float64, device=dev) for _ in range(3)]
        e = 1e-6

        def L(s):
            return float(0.5 * ((G(h0 + s * v[0], hu0 + s * v[1], b0 + s * v[2]) - obs) ** 2).sum())

        fd = (L(e) - L(-e)) / (2 * e)
        ad = float(sum(torch.dot(g, vv) for g, vv in zip((h0.grad, hu0.grad, b0.grad), v)))
        assert abs(fd - ad) <= 1e-6 * max(1e-3, abs(ad)), (fd, ad)
