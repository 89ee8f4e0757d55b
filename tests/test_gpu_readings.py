"""GPU path against the oracle under the alternative readings (flags), the
class record of alew_run, full-length class parity of the 200-cell smooth
case, and the step-buffer capacity error.  All calls go through the C ABI."""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_common import (assert_parity, class_flips, class_record, gparams, oparams, run_one,
                        t64)
from paper_2208_06588_amd import alew, workloads as W

pytestmark = pytest.mark.gpu

FLAG_CASES = {
    "alpha_cellavg": (alew.F_ALPHA_CELLAVG, O.FLAG_ALPHA_CELLAVG),
    "no_hu_limit": (alew.F_NO_HU_LIMIT, O.FLAG_NO_HU_LIMIT),
    "w_tangent": (alew.F_W_TANGENT, O.FLAG_W_TANGENT),
    "all_hydrostatic": (alew.F_ALPHA_CELLAVG | alew.F_NO_HU_LIMIT | alew.F_W_TANGENT
                        | alew.F_HYDROSTATIC,
                        O.FLAG_ALPHA_CELLAVG | O.FLAG_NO_HU_LIMIT | O.FLAG_W_TANGENT
                        | O.FLAG_HYDROSTATIC),
}


@pytest.fixture(scope="module")
def dev():
    torch.cuda.set_device(0)
    return torch.device("cuda", 0)


@pytest.mark.parametrize("case", list(FLAG_CASES))
def test_readings_smooth_periodic_run(dev, case):
    """200-cell smooth periodic case (Example 5.1 data, sine mesh) to t = 0.1."""
    gf, of = FLAG_CASES[case]
    wl = W.accuracy_1d(200)
    ctx = alew.Context(200, 1)
    g, st = run_one(ctx, gparams(wl, flags=gf), wl, dev, t_end=[0.1])
    r = O.run(oparams(wl, flags=of), wl["h"], wl["hu"], wl["b"], wl["x"], wl["xi"], t_end=0.1)
    assert st.status == 0 and r["status"] == 0
    assert st.steps == r["stats"].steps
    assert tuple(st.n_class) == tuple(r["stats"].n_class)
    assert_parity(g, r, tag=case)


@pytest.mark.parametrize("case", list(FLAG_CASES))
def test_readings_wet_dry_bowl(dev, case):
    """2048-cell parabolic bowl, fluid-following mesh, CFL 0.08: the limiter acts
    on the dry shelf every stage.  Status, step count and state as the oracle
    (the limiter on h alone may end in a negative depth; then both report it
    after the same step)."""
    gf, of = FLAG_CASES[case]
    wl = W.bowl_1d(2048)
    ctx = alew.Context(2048, 1)
    g, st = run_one(ctx, gparams(wl, flags=gf), wl, dev, max_steps=[30], check=False)
    r = O.run(oparams(wl, flags=of), wl["h"], wl["hu"], wl["b"], wl["x"], wl["xi"], max_steps=30)
    ost = {O.ST_OK: alew.OK, O.ST_NEGDEPTH: alew.E_NEGDEPTH, O.ST_MESH: alew.E_MESH,
           O.ST_NONFINITE: alew.E_NONFINITE}[r["status"]]
    assert st.status == ost
    assert st.steps == r["stats"].steps and st.n_limited > 0
    assert st.n_limited == r["stats"].n_limited
    assert_parity(g, r, tag=case)


def test_step_log_capacity_is_reported(dev):
    """A step log shorter than the run stops the instance with ALEW_E_CAPACITY
    after dts_stride steps instead of returning OK short of t_end."""
    wl = W.accuracy_1d(64)
    ctx = alew.Context(64, 1)
    log = torch.zeros(5, dtype=torch.float64, device=dev)
    g, st = run_one(ctx, gparams(wl), wl, dev, t_end=[0.1], dt_log=log, dts_stride=5, check=False)
    assert st.status == alew.E_CAPACITY
    assert st.steps == 5 and st.t < 0.1
    assert bool((log > 0).all())
    with pytest.raises(alew.AlewError) as ei:
        run_one(ctx, gparams(wl), wl, dev, t_end=[0.1], dt_log=log, dts_stride=5)
    assert ei.value.status == alew.E_CAPACITY


@pytest.mark.parametrize("hydro", [False, True])
def test_smooth_case_classes_every_step_full_run(dev, hydro):
    """The 200-cell smooth periodic case to t = 0.1 through alew_step, one call
    per step: the detector class of every cell at every stage of every step
    equals the oracle's (no flips over the whole run), and so does the state."""
    wl = W.accuracy_1d(200)
    fl_g = alew.F_HYDROSTATIC if hydro else 0
    fl_o = O.FLAG_HYDROSTATIC if hydro else 0
    r = O.run(oparams(wl, flags=fl_o), wl["h"], wl["hu"], wl["b"], wl["x"], wl["xi"], t_end=0.1,
              max_steps=2000, record_cls=True)
    nsteps = r["stats"].steps
    assert r["status"] == 0 and 300 < nsteps < 2000
    p = gparams(wl, flags=fl_g)
    ctx = alew.Context(200, 1)
    t = {k: t64(wl[k], dev) for k in ("h", "hu", "b", "x", "xi")}
    cls = torch.zeros(3 * 200, dtype=torch.uint8, device=dev)
    got = []
    tt = 0.0
    while tt < 0.1:
        st = ctx.step(p, t["h"], t["hu"], t["b"], t["x"], t["xi"], t=tt, t_end=0.1, cls=cls)
        tt = st.t
        got.append(cls.cpu().numpy().reshape(3, 200).copy())
        assert len(got) <= nsteps
    got = np.stack(got)
    assert got.shape[0] == nsteps
    flips = int((got != r["cls"][:nsteps]).sum())
    assert flips == 0, f"{flips} class flips"
    g = {k: v.cpu().numpy() for k, v in t.items()}
    assert_parity(g, r)


@pytest.mark.parametrize("hydro", [False, True])
def test_run_class_record_matches_oracle(dev, hydro):
    """alew_run's class record (per-cell counts and sequence signatures) of a
    ragged perturbation batch run to t = 0.2 equals the oracle's, instance by
    instance, as do the states and step counts."""
    rng = np.random.default_rng(12)
    sizes = [5, 9, 64, 131, 250, 377]
    insts = [W.perturbation_instance(int(n), float(rng.uniform(1e-3, 1e-2))) for n in sizes]
    bt = W.pack(insts, bc="transmissive", cfl=0.6, weno_eps=1e-9, mesh="sine", mesh_A=0.05,
                mesh_k=1.0, mesh_omega=np.pi)
    off = [int(v) for v in bt["cell_off"]]
    S, ninst = off[-1], len(off) - 1
    fl_g = alew.F_HYDROSTATIC if hydro else 0
    fl_o = O.FLAG_HYDROSTATIC if hydro else 0
    ctx = alew.Context(S, ninst)
    T = {k: t64(bt[k], dev) for k in ("h", "hu", "b", "x", "xi")}
    cnt = torch.zeros(3 * S, dtype=torch.int32, device=dev)
    sig = torch.zeros(S, dtype=torch.int64, device=dev)
    st = ctx.run(gparams(bt, flags=fl_g), off, T["h"], T["hu"], T["b"], T["x"], T["xi"],
                 t_end=[0.2] * ninst, cls_count=cnt, cls_sig=sig)
    torch.cuda.synchronize()
    G = {k: v.cpu().numpy() for k, v in T.items()}
    C = cnt.cpu().numpy().astype(np.int64).reshape(3, S)
    Z = sig.cpu().numpy().view(np.uint64)
    op = oparams(bt, flags=fl_o)
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
        assert tuple(st[i].n_class) == tuple(rc.sum(axis=1))
        g = dict(h=G["h"][a:e], hu=G["hu"][a:e], b=G["b"][a:e], x=G["x"][a + i:e + i + 1])
        assert_parity(g, r, tag=f"instance {i}")
