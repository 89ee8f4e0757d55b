"""GPU path with an analytic bottom projected onto the moving cells at every
stage (Sec. 3.3, eq. (3.16)) instead of evolved by eq. (3.17), against the
oracle, through the C ABI."""

import numpy as np
import pytest
import torch

import oracle as O
from gpu_common import (assert_parity, class_flips, class_record, gparams, oparams, run_one,
                        t64)
from paper_2208_06588_amd import alew, workloads as W

pytestmark = pytest.mark.gpu

# (library name, oracle code, parameters)
BOTTOMS = {
    "step": ("step", O.BOTTOM_STEP, (4.0, 4.0, 8.0, 0.0)),
    "gauss": ("gauss", O.BOTTOM_GAUSS, (5.0, 0.4, 5.0, 0.0)),
    "sin2": ("sin2", O.BOTTOM_SIN2, (1.0, 1.0, 0.0, 0.0)),
    "bump": ("bump", O.BOTTOM_BUMP, (0.25, 0.1, 1.5, 0.0)),
    "parabola": ("parabola", O.BOTTOM_PARABOLA, (10.0, 3000.0, 0.0, 0.0)),
}


def _both(kind, gflags=0, oflags=0):
    g, o, bp = BOTTOMS[kind]
    return dict(bottom=g, bottom_p=bp, flags=gflags), dict(bottom=o, bottom_p=bp, flags=oflags)


@pytest.fixture(scope="module")
def dev():
    torch.cuda.set_device(0)
    return torch.device("cuda", 0)


@pytest.mark.parametrize("hydro", [False, True])
@pytest.mark.parametrize("kind", ["gauss", "step"])
def test_projected_bottom_still_water(dev, kind, hydro):
    """Example 5.3 with the projected bottom, to t = 0.5: round-off on the GPU and
    the oracle's state (the b array's input is replaced by the projection)."""
    wl = W.still_water_1d(200, "smooth" if kind == "gauss" else "step")
    wl["b"] = np.zeros(200)
    gk, ok = _both(kind, alew.F_HYDROSTATIC if hydro else 0, O.FLAG_HYDROSTATIC if hydro else 0)
    ctx = alew.Context(200, 1)
    g, st = run_one(ctx, gparams(wl, **gk), wl, dev, t_end=[0.5])
    r = O.run(oparams(wl, **ok), wl["h"], wl["hu"], wl["b"], wl["x"], wl["xi"], t_end=0.5)
    assert st.status == 0 and r["status"] == 0 and st.steps == r["stats"].steps
    assert np.abs(g["h"] + g["b"] - 10.0).max() < 1e-12
    assert np.abs(g["hu"]).max() < 1e-11
    assert_parity(g, r)


@pytest.mark.parametrize("scheme", [0, alew.F_HYDROSTATIC, alew.F_NONWB])
def test_projected_bottom_smooth_periodic(dev, scheme):
    """Example 5.1 with b = sin^2(pi x) projected, sine mesh, 200 cells, to t = 0.1,
    for every scheme."""
    of = {0: 0, alew.F_HYDROSTATIC: O.FLAG_HYDROSTATIC, alew.F_NONWB: O.FLAG_NONWB}[scheme]
    wl = W.accuracy_1d(200)
    gk, ok = _both("sin2", scheme, of)
    ctx = alew.Context(200, 1)
    g, st = run_one(ctx, gparams(wl, **gk), wl, dev, t_end=[0.1])
    r = O.run(oparams(wl, **ok), wl["h"], wl["hu"], wl["b"], wl["x"], wl["xi"], t_end=0.1)
    assert st.status == 0 and r["status"] == 0 and st.steps == r["stats"].steps
    assert tuple(st.n_class) == tuple(r["stats"].n_class)
    assert abs(st.mass_b - 0.5) < 1e-14 and abs(st.mass_b0 - 0.5) < 1e-14
    assert_parity(g, r)


def test_projected_bump_ragged_batch(dev):
    """Ragged perturbation batch (Example 5.4 shape) with the bump projected, to
    t = 0.2: every instance equals the oracle, class records included."""
    rng = np.random.default_rng(7)
    sizes = [5, 64, 129, 300, 451]
    insts = [W.perturbation_instance(int(n), float(rng.uniform(1e-3, 1e-2))) for n in sizes]
    bt = W.pack(insts, bc="transmissive", cfl=0.6, weno_eps=1e-9, mesh="sine", mesh_A=0.05,
                mesh_k=1.0, mesh_omega=np.pi)
    off = [int(v) for v in bt["cell_off"]]
    S, ninst = off[-1], len(off) - 1
    gk, ok = _both("bump")
    ctx = alew.Context(S, ninst)
    T = {k: t64(bt[k], dev) for k in ("h", "hu", "b", "x", "xi")}
    cnt = torch.zeros(3 * S, dtype=torch.int32, device=dev)
    sig = torch.zeros(S, dtype=torch.int64, device=dev)
    st = ctx.run(gparams(bt, **gk), off, T["h"], T["hu"], T["b"], T["x"], T["xi"],
                 t_end=[0.2] * ninst, cls_count=cnt, cls_sig=sig)
    torch.cuda.synchronize()
    G = {k: v.cpu().numpy() for k, v in T.items()}
    C = cnt.cpu().numpy().astype(np.int64).reshape(3, S)
    Z = sig.cpu().numpy().view(np.uint64)
    op = oparams(bt, **ok)
    for i in range(ninst):
        a, e = off[i], off[i + 1]
        n = e - a
        r = O.run(op, bt["h"][a:e], bt["hu"][a:e], bt["b"][a:e], bt["x"][a + i:e + i + 1],
                  bt["xi"][a + i:e + i + 1], t_end=0.2, max_steps=20 * n + 100, record_cls=True)
        ns = r["stats"].steps
        assert r["status"] == 0 and st[i].status == 0 and st[i].steps == ns
        rc, rs = class_record(r["cls"][:ns])
        cells, lower = class_flips(C[:, a:e], Z[a:e], rc, rs)
        assert cells == 0 and lower == 0, (i, cells, lower)
        g = dict(h=G["h"][a:e], hu=G["hu"][a:e], b=G["b"][a:e], x=G["x"][a + i:e + i + 1])
        assert_parity(g, r, tag=f"instance {i}")


def test_projected_parabola_bowl_loses_positivity_alike(dev):
    """The wet/dry bowl (fluid-following mesh, CFL 0.08) at 2048 cells with its
    parabola projected onto the cells.  Sec. 3.3 warns that the projection may
    cost positivity on moving meshes: b no longer follows the limited bottom
    traces that Property 3.1 relies on, and a negative mean depth appears at
    the wet/dry front in the first step.  Both sides report it after the same
    step, with the same state."""
    wl = W.bowl_1d(2048)
    gk, ok = _both("parabola")
    ctx = alew.Context(2048, 1)
    g, st = run_one(ctx, gparams(wl, **gk), wl, dev, max_steps=[30], check=False)
    r = O.run(oparams(wl, **ok), wl["h"], wl["hu"], wl["b"], wl["x"], wl["xi"], max_steps=30)
    assert r["status"] == O.ST_NEGDEPTH and st.status == alew.E_NEGDEPTH
    assert st.steps == r["stats"].steps and st.n_limited == r["stats"].n_limited
    assert_parity(g, r)


def test_projected_engines_agree_and_adjoint_refuses(dev):
    """Stage launches and the persistent engine give the same bits with the
    projected bottom; the adjoint refuses it."""
    bt = W.pack([W.perturbation_instance(n, 5e-3) for n in (300, 1000)], bc="transmissive",
                cfl=0.6, weno_eps=1e-9, mesh="sine", mesh_A=0.05, mesh_k=1.0, mesh_omega=np.pi)
    off = [int(v) for v in bt["cell_off"]]
    S = off[-1]
    gk, _ = _both("bump")
    p = gparams(bt, **gk)
    outs = []
    for launch in (dict(engine=alew.ENGINE_STAGES, block=64, cells_per_thread=2),
                   dict(engine=alew.ENGINE_STAGES, block=256, cells_per_thread=1),
                   dict(engine=alew.ENGINE_PERSISTENT, block=256, cells_per_thread=1)):
        ctx = alew.Context(S, 2)
        ctx.set_launch(**launch)
        T = {k: t64(bt[k], dev) for k in ("h", "hu", "b", "x", "xi")}
        ctx.run(p, off, T["h"], T["hu"], T["b"], T["x"], T["xi"], max_steps=[25, 25])
        torch.cuda.synchronize()
        outs.append(T)
    for T in outs[1:]:
        for k in ("h", "hu", "b", "x"):
            assert torch.equal(T[k], outs[0][k]), k
    ctx = alew.Context(S, 2)
    T = outs[0]
    g = torch.zeros(2, dtype=torch.float64, device=dev)
    with pytest.raises(alew.AlewError) as ei:
        ctx.adjoint(p, off, T["h"], T["hu"], T["b"], T["x"], T["xi"], 1,
                    torch.full((2,), 1e-4, dtype=torch.float64, device=dev), 1,
                    torch.tensor([0.5, 0.5], dtype=torch.float64, device=dev), g)
    assert ei.value.status == alew.E_UNSUPPORTED


@pytest.mark.parametrize("scheme,t_end", [(0, 15.0), (alew.F_HYDROSTATIC, 15.0),
                                          (alew.F_NONWB, 15.0), (0, 60.0)])
def test_example_5_5_jump_aligned_mesh(dev, scheme, t_end):
    """Example 5.5 (dam break over the rectangular bump, bottom projected, nodes
    moved by the quartic map of eq. (5.14)) on 104 cells against the oracle:
    equal steps and class counts, the state at the parity tolerance; on the GPU
    as well the nodes on the jump points never move and the projected bottom is
    exactly 0 or 8.  t = 60: the waves have left through both ends."""
    of = {0: 0, alew.F_HYDROSTATIC: O.FLAG_HYDROSTATIC, alew.F_NONWB: O.FLAG_NONWB}[scheme]
    wl = W.dam_break_bump_1d(104, t_end)
    bp = wl["bottom_p"]
    ctx = alew.Context(104, 1)
    g, st = run_one(ctx, gparams(wl, bottom="step", bottom_p=bp, flags=scheme), wl, dev,
                    t_end=[t_end])
    r = O.run(oparams(wl, bottom=O.BOTTOM_STEP, bottom_p=bp, flags=of), wl["h"], wl["hu"],
              np.zeros(104), wl["x"], wl["xi"], t_end=t_end)
    assert st.status == 0 and r["status"] == 0 and st.steps == r["stats"].steps
    assert tuple(st.n_class) == tuple(r["stats"].n_class)
    assert g["x"][39] == 562.5 and g["x"][65] == 937.5
    assert set(np.unique(g["b"]).tolist()) == {0.0, 8.0}
    assert_parity(g, r)
