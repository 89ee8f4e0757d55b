#!/usr/bin/env python3
"""Throughput of the batched FP64 ALE-WENO forward run on one MI355X.

Workload: ragged batch of 4096 independent 1D perturbation-of-still-water
instances (LeVeque bump, Example 5.4 shape), cell counts uniform in
[1000, 20000] from seed 2208065881 (43,017,136 cells), transmissive
boundaries, sine-moving mesh, CFL 0.6, each instance with its own CFL step.
A benchmark "step" advances every instance by one SSP-RK3 time step (three
stages).  Throughput = cells x stages / second over exactly --steps steps
timed after --warmup untimed steps, inputs resident in HBM.

Prints one JSON line (roofline of the dominant kernel, CPU oracle baseline,
batched-vs-per-instance speedup).  --gpus N with N > 1 exits: one GPU only.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import gc
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-updates/s per RK stage (FP64) + %HBM roofline; adjoint/forward time ratio"
HBM_PEAK_GBS = 8000.0
# Algorithmic HBM bytes per cell and time step (FP64 SoA): stage 1 reads q^n, J^n,
# x^n and writes q^(1) (64 B); stage 2 also reads the base state (88 B); stage 3
# writes q^{n+1}, J^{n+1}, x^{n+1} (104 B).
ALG_BYTES_PER_CELL_STEP = 256.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _code_only(text):
    """C++ source without comments and with whitespace runs collapsed (string
    literals here hold no comment markers), so that edits of comments alone
    keep the counters of profiles/counters.json valid."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def source_hash():
    """Hash of the code (comments stripped) of the stage kernels' sources."""
    h = hashlib.sha1()
    for f in ("alew.hip", "alew_device.h", "alew_kernels.h"):
        with open(os.path.join(ROOT, "paper_2208_06588_amd", "csrc", f)) as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def load_counters(kernel):
    """rocprofv3 counter results for this kernel and this library source
    (profiles/counters.json; how each figure is derived from the counters is
    stated in the profile summaries beside it), or None when the library
    source changed since they were taken."""
    try:
        with open(os.path.join(ROOT, "profiles", "counters.json")) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    e = d.get(kernel)
    if not e or e.get("source_hash") != source_hash():
        return None
    return e


def copy_bandwidth(nbytes=4 << 30, reps=10):
    """Device-to-device copy of nbytes, timed with events over reps copies:
    bytes read + written per second (GB/s), the practical HBM rate for
    streaming work on this GPU (context for the 8 TB/s peak)."""
    import torch
    n = nbytes // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    del a, b
    torch.cuda.empty_cache()
    return round(2.0 * n * 8 * reps / (ms / 1e3) / 1e9, 1)


def scheme_id(p):
    """The stage kernels' scheme template argument: 0 special source term,
    1 hydrostatic reconstruction, 2 without well-balancing."""
    from paper_2208_06588_amd import alew
    if p.flags & alew.F_NONWB:
        return 2
    return 1 if p.flags & alew.F_HYDROSTATIC else 0


def roofline(ctx, p, off, T, tnow, L, S, kern_ms, launches, steps, copy_bw=True):
    """Roofline object of the dominant kernel.  For the stage-launch engine the
    same number of steps runs once more with an event pair around every stage
    launch (no graph); achieved = the method's bytes per cell and stage (256/3 B)
    x cells of a launch / average stage-launch time.  Counter results (HBM
    bytes, VALU instructions) come from profiles/counters.json when they were
    taken on this source."""
    from paper_2208_06588_amd import alew
    import torch
    per_stage = ALG_BYTES_PER_CELL_STEP / 3.0
    if L.engine == alew.ENGINE_PERSISTENT:
        blk = L.block or 256
        cpt = L.cells_per_thread or (2 if blk == 64 else 1)
        kernel = f"k_persistent<{blk}, {cpt}, {scheme_id(p)}>"
        ms_launch = kern_ms / max(1, launches)
        achieved = ALG_BYTES_PER_CELL_STEP * S * steps / max(1, launches) / (ms_launch / 1e3) / 1e9
        stage_launches, epi = None, None
    else:
        blk = L.block or 64  # 0 = the library's choice for the stage launches
        cpt = L.cells_per_thread or (2 if blk == 64 else 1)
        kernel = f"k_stage<{blk}, {cpt}, {'true' if L.compact_tiles else 'false'}, {scheme_id(p)}>"
        ctx.set_kernel_timing(True)
        W = {k: v.clone() for k, v in T.items()}
        ctx.run(p, off, W["h"], W["hu"], W["b"], W["x"], W["xi"], t0=tnow,
                max_steps=[steps] * (len(off) - 1))
        torch.cuda.synchronize()
        ctx.set_kernel_timing(False)
        sms, sn, scells = ctx.kernel_timing(0)
        ems, en, _ = ctx.kernel_timing(1)
        del W
        ms_launch = sms / max(1, sn)
        achieved = per_stage * scells / (sms / 1e3) / 1e9
        stage_launches = sn
        epi = dict(kernel="k_final<256>", launches=en, launch_ms=round(ems / max(1, en), 4))
        # RK stage 1 reads the step's state (88 B per cell moved); stages 2 and 3
        # also the previous stage's partial updates (136 B per cell)
        by_stage = []
        for q in (2, 3, 4):
            qms, qn, _ = ctx.kernel_timing(q)
            by_stage.append(round(qms / max(1, qn), 4))
        log(f"kernel timing: {sn} stage launches, {ms_launch:.4f} ms each (by RK stage "
            f"{by_stage}); {en} epilogues, {ems / max(1, en):.4f} ms each")
    roof = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=None, kernel=kernel,
                launch_ms=round(ms_launch, 4), launches=stage_launches,
                alg_bytes_per_cell_stage=round(per_stage, 3),
                timing="HIP events on the library stream around each launch")
    if epi is not None:
        roof["launch_ms_by_rk_stage"] = by_stage
        roof["step_epilogue"] = epi
    if copy_bw:  # (profiler runs calibrate their byte counters with a copy of their own)
        roof["copy_gbs"] = copy_bandwidth()
    c = load_counters(kernel)
    if c is not None:
        cells_per_launch = S
        roof["traffic"] = round(c["hbm_bytes_per_cell_stage"] * cells_per_launch)
        roof["traffic_note"] = ("FETCH_SIZE x %.2f + WRITE_SIZE x %.2f per launch (copy-kernel "
                                "calibration), scaled to this batch" % (c["fetch_factor"],
                                                                         c["write_factor"]))
        # FP64 VALU against the chip: 256 CUs x 4 SIMDs x 2.4 GHz issue one wave64
        # instruction per SIMD every 4 cycles; FP64 peak 78.6 TFLOP/s
        waves = c["waves_per_cell_stage"] * cells_per_launch
        issue_s = c["valu_per_wave"] * waves * 4 / (1024 * 2.4e9)
        flops = c["fp64_flops_per_cell_stage"] * cells_per_launch
        roof["valu"] = dict(valu_insts_per_wave=round(c["valu_per_wave"], 1),
                            fp64_flops_per_cell_stage=round(c["fp64_flops_per_cell_stage"], 1),
                            issue_utilisation=round(issue_s / (ms_launch / 1e3), 4),
                            fp64_tflops=round(flops / (ms_launch / 1e3) / 1e12, 2),
                            fp64_peak_tflops=78.6,
                            fp64_frac=round(flops / (ms_launch / 1e3) / 78.6e12, 4))
    return roof


def bowl_leg(dev, n, steps, warmup):
    """Single 2^24-cell wet/dry run (parabolic bowl, fluid-following mesh,
    limiter active): forward throughput and the HBM fraction of the whole step."""
    import torch
    from paper_2208_06588_amd import alew, workloads as W
    t0 = time.perf_counter()
    wl = W.bowl_1d(n)
    log(f"bowl workload: {n} cells ({time.perf_counter() - t0:.1f} s to build)")
    p = alew.params(bc="transmissive", mesh="fluid", cfl=wl["cfl"], weno_eps=wl["weno_eps"])
    T = {k: torch.tensor(wl[k], dtype=torch.float64, device=dev) for k in ("h", "hu", "b", "x", "xi")}
    ctx = alew.Context(n, 1)
    # the autotuner over the stage-launch shapes (one work-group per instance, the
    # persistent engine, is no candidate for a single 2^24-cell instance)
    from paper_2208_06588_amd import autotune
    best, _ = autotune.tune(ctx, p, [0, n], T, steps=2, use_cache=False, log=log,
                            candidates=[c for c in autotune.CANDIDATES
                                        if c["engine"] == alew.ENGINE_STAGES])
    st = ctx.run(p, [0, n], T["h"], T["hu"], T["b"], T["x"], T["xi"], max_steps=[warmup])
    torch.cuda.synchronize()
    gc.collect()
    a = time.perf_counter()
    st = ctx.run(p, [0, n], T["h"], T["hu"], T["b"], T["x"], T["xi"], t0=[st[0].t], max_steps=[steps])
    torch.cuda.synchronize()
    wall = time.perf_counter() - a
    assert st[0].steps == steps and st[0].status == 0, "bowl run did not complete"
    value = 3.0 * n * steps / wall
    return dict(workload=f"parabolic bowl, {n} cells, transmissive, fluid-following mesh, CFL 0.08",
                steps=steps, value=value, unit="cell-updates/s",
                launch=autotune.name_of(best),
                step_hbm_frac=round(ALG_BYTES_PER_CELL_STEP * n * steps / wall / 1e9 / HBM_PEAK_GBS, 4),
                limited_cells_per_step=round(st[0].n_limited / steps, 1),
                h_min=st[0].h_min)


def guarded(name, fn):
    """Run one of the legs beside the main measurement; a failure there is
    reported in its place instead of costing the whole line."""
    try:
        return fn()
    except (AssertionError, RuntimeError, ValueError) as e:
        log(f"{name} failed: {e!r}")
        return dict(error=f"{type(e).__name__}: {e}")


def hydrostatic_leg(ctx, p, off, T, tnow, L, S, steps):
    """The hydrostatic-reconstruction scheme (Sec. 4.1) on the forward batch,
    in the forward leg's launch: 2 warm-up steps, then `steps` timed steps in
    one call (wall and the library's event time of the call), and its stage
    kernel's roofline from the event-timed pass."""
    import torch
    ninst = len(off) - 1
    W = {k: v.clone() for k, v in T.items()}
    st = ctx.run(p, off, W["h"], W["hu"], W["b"], W["x"], W["xi"], t0=tnow, max_steps=[2] * ninst)
    tnow = [s.t for s in st]
    torch.cuda.synchronize()
    gc.collect()
    a = time.perf_counter()
    st = ctx.run(p, off, W["h"], W["hu"], W["b"], W["x"], W["xi"], t0=tnow,
                 max_steps=[steps] * ninst)
    torch.cuda.synchronize()
    wall = time.perf_counter() - a
    assert all(s.steps == steps and s.status == 0 for s in st), "hydrostatic run did not complete"
    kern_ms, launches = ctx.last_timing()
    roof = roofline(ctx, p, off, W, tnow=[s.t for s in st], L=L, S=S, kern_ms=kern_ms,
                    launches=launches, steps=steps, copy_bw=False)
    del W
    return dict(workload="the forward batch with the hydrostatic reconstruction (Sec. 4.1)",
                steps=steps, value=3.0 * S * steps / wall, unit="cell-updates/s",
                ms_per_step=round(wall * 1e3 / steps, 4),
                kernel_ms_per_step=round(kern_ms / steps, 4), roofline=roof)


def cpu_baseline(bt, ninst_sample, steps):
    """The oracle on the host cores: first ninst_sample instances of the same
    draw, `steps` CFL steps each, one instance per thread."""
    import oracle as O
    off = bt["cell_off"]
    P = O.params(bc=O.BC_TRANSMISSIVE, mesh=O.MESH_SINE, mesh_A=0.05, mesh_k=1.0,
                 mesh_omega=np.pi, cfl=0.6, weno_eps=1e-9)
    O.lib()
    nproc = os.cpu_count() or 1
    try:
        nproc = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        pass
    # the machine's CPU share for one GPU is 16 cores whatever the host shows
    cores = min(16, nproc)

    def one(i):
        a, e = int(off[i]), int(off[i + 1])
        r = O.run(P, bt["h"][a:e], bt["hu"][a:e], bt["b"][a:e], bt["x"][a + i:e + i + 1],
                  bt["xi"][a + i:e + i + 1], max_steps=steps)
        return (e - a) * 3 * r["stats"].steps

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=cores) as ex:
        work = sum(ex.map(one, range(ninst_sample)))
    wall = time.perf_counter() - t0
    ncell = int(off[ninst_sample])
    return dict(value=work / wall, unit="cell-updates/s", cores=cores, kind="oracle",
                per_core=work / wall / cores, nproc=nproc, cpu_model=cpu_model(),
                sample=f"first {ninst_sample} instances of the same draw ({ncell} cells), "
                       f"{steps} CFL steps each, one instance per thread; {wall:.1f} s wall")


def class_flips_leg(dev, bt, ninst_sample, steps):
    """Class flips between the GPU and the oracle on the first ninst_sample
    instances of the batch over `steps` steps: both record the class of every
    cell at every stage (the GPU as per-cell counts and a sequence signature,
    sig <- sig * CLS_SIG_MUL + class + 1 per stage, the oracle as the full
    record, reduced here the same way); a cell whose signatures differ has
    flipped at least once."""
    import torch
    import oracle as O
    from paper_2208_06588_amd import alew
    off = bt["cell_off"][:ninst_sample + 1]
    S = int(off[-1])
    P = O.params(bc=O.BC_TRANSMISSIVE, mesh=O.MESH_SINE, mesh_A=0.05, mesh_k=1.0,
                 mesh_omega=np.pi, cfl=0.6, weno_eps=1e-9)
    mul = np.uint64(alew.CLS_SIG_MUL)

    def one(i):
        a, e = int(off[i]), int(off[i + 1])
        r = O.run(P, bt["h"][a:e], bt["hu"][a:e], bt["b"][a:e], bt["x"][a + i:e + i + 1],
                  bt["xi"][a + i:e + i + 1], max_steps=steps, record_cls=True)
        cl = r["cls"][:r["stats"].steps]
        counts = np.stack([(cl == c).sum(axis=(0, 1)) for c in range(3)]).astype(np.int64)
        sig = np.zeros(e - a, dtype=np.uint64)
        with np.errstate(over="ignore"):
            for k in range(cl.shape[0]):
                for st in range(3):
                    sig = sig * mul + (cl[k, st].astype(np.uint64) + np.uint64(1))
        return counts, sig

    with cf.ThreadPoolExecutor(max_workers=16) as ex:
        ref = list(ex.map(one, range(ninst_sample)))
    rc = np.concatenate([c for c, _ in ref], axis=1)
    rs = np.concatenate([g for _, g in ref])
    T = {k: torch.tensor(np.asarray(bt[k][:S + (ninst_sample if k in ("x", "xi") else 0)]),
                         dtype=torch.float64, device=dev) for k in ("h", "hu", "b", "x", "xi")}
    cnt = torch.zeros(3 * S, dtype=torch.int32, device=dev)
    sig = torch.zeros(S, dtype=torch.int64, device=dev)
    ctx = alew.Context(S, ninst_sample)
    p = alew.params(bc="transmissive", mesh="sine", mesh_A=0.05, mesh_k=1.0, mesh_omega=np.pi,
                    cfl=0.6, weno_eps=1e-9)
    ctx.run(p, list(off), T["h"], T["hu"], T["b"], T["x"], T["xi"], max_steps=[steps] * ninst_sample,
            cls_count=cnt, cls_sig=sig)
    torch.cuda.synchronize()
    gc_ = cnt.cpu().numpy().astype(np.int64).reshape(3, S)
    gs = sig.cpu().numpy().view(np.uint64)
    cells = int((gs != rs).sum())
    return dict(instances=ninst_sample, cells=S, steps=steps, cell_stages=3 * S * steps,
                flipped_cells=cells,
                flipped_cell_stages_at_least=int(np.abs(gc_ - rc).sum()) // 2,
                class_counts=[int(v) for v in rc.sum(axis=1)])


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            return next(l.split(":", 1)[1].strip() for l in f if l.startswith("model name"))
    except (OSError, StopIteration):
        return "unknown"


def oracle_other_configs():
    """Part of the CPU baseline: the oracle, single threaded (one instance per
    call), on the other configurations: the 200-cell periodic smooth run to
    t = 0.1 in full; one perturbation instance of the 4096-instance draw, 30
    steps; the parabolic bowl at 2^22 cells, one step; one 65536-cell instance
    of the inversion batch, 2 steps forward and the tape adjoint of those
    steps."""
    import oracle as O
    from paper_2208_06588_amd import workloads as W
    out = {"cpu": cpu_model(), "threads": 1}
    wl = W.accuracy_1d(200, "sine")
    op = O.params(bc=O.BC_PERIODIC, mesh=O.MESH_SINE, mesh_A=0.05, mesh_k=1.0,
                  mesh_omega=math.pi, cfl=0.6, weno_eps=1e-6)
    a = time.perf_counter()
    r = O.run(op, wl["h"], wl["hu"], wl["b"], wl["x"], wl["xi"], t_end=0.1)
    t_o = time.perf_counter() - a
    st = r["stats"].steps
    out["smooth_200_to_t0.1"] = dict(cells=200, steps=st, wall_s=round(t_o, 3),
                                     value=3.0 * 200 * st / t_o)
    bt = W.perturbation_batch(subset=1)
    n = int(bt["cell_off"][1])
    op = O.params(bc=O.BC_TRANSMISSIVE, mesh=O.MESH_SINE, mesh_A=0.05, mesh_k=1.0,
                  mesh_omega=math.pi, cfl=0.6, weno_eps=1e-9)
    a = time.perf_counter()
    O.run(op, bt["h"], bt["hu"], bt["b"], bt["x"], bt["xi"], max_steps=30)
    out["perturbation_one_instance"] = dict(cells=n, steps=30,
                                            value=3.0 * n * 30 / (time.perf_counter() - a))
    wl = W.bowl_1d(1 << 22)
    op = O.params(bc=O.BC_TRANSMISSIVE, mesh=O.MESH_FLUID, cfl=0.08, weno_eps=1e-6)
    a = time.perf_counter()
    O.run(op, wl["h"], wl["hu"], wl["b"], wl["x"], wl["xi"], max_steps=1)
    out["bowl_2p22_one_step"] = dict(cells=1 << 22, value=3.0 * (1 << 22) / (time.perf_counter() - a))
    bt = W.inversion_batch(ninst=1, n=65536, ngauge=64)
    op = O.params(bc=O.BC_TRANSMISSIVE, mesh=O.MESH_SINE, mesh_A=0.05, mesh_k=1.0,
                  mesh_omega=math.pi, cfl=0.6)
    a = time.perf_counter()
    r = O.run(op, bt["h"], bt["hu"], bt["b"], bt["x"], bt["xi"], max_steps=2)
    t_f = time.perf_counter() - a
    dts = np.full(2, r["stats"].dt_min)
    a = time.perf_counter()
    O.adjoint(op, bt["h"], bt["hu"], bt["b"], bt["x"], bt["xi"], dts, bt["gauge_x"], np.ones(64))
    t_a = time.perf_counter() - a
    out["inversion_one_instance_2_steps"] = dict(cells=65536, forward_s=round(t_f, 3),
                                                 adjoint_s=round(t_a, 3),
                                                 adjoint_over_forward=round(t_a / t_f, 2))
    for v in out.values():
        if isinstance(v, dict) and "value" in v:
            v["unit"] = "cell-updates/s"
    return out


def small_run_leg(dev):
    """The 200-cell smooth periodic run to t = 0.1 on the GPU (one instance:
    bound by launch latency, not by the kernels)."""
    import torch
    from paper_2208_06588_amd import alew, workloads as W
    wl = W.accuracy_1d(200, "sine")
    gp = alew.params(bc="periodic", mesh="sine", mesh_A=0.05, mesh_k=1.0, mesh_omega=math.pi,
                     cfl=0.6, weno_eps=1e-6)
    T = {k: torch.tensor(wl[k], dtype=torch.float64, device=dev) for k in ("h", "hu", "b", "x", "xi")}
    ctx = alew.Context(200, 1)
    ctx.set_launch(engine=alew.ENGINE_STAGES, use_graph=1)
    W1 = {k: v.clone() for k, v in T.items()}
    ctx.run(gp, [0, 200], W1["h"], W1["hu"], W1["b"], W1["x"], W1["xi"], t_end=[0.1])
    torch.cuda.synchronize()
    gc.collect()
    a = time.perf_counter()
    sg = ctx.run(gp, [0, 200], T["h"], T["hu"], T["b"], T["x"], T["xi"], t_end=[0.1])[0]
    torch.cuda.synchronize()
    t_g = time.perf_counter() - a
    ctx.close()
    return dict(cells=200, steps=sg.steps, wall_s=round(t_g, 4), value=3.0 * 200 * sg.steps / t_g,
                unit="cell-updates/s")


def adjoint_leg(dev, ninst, ncell, nsteps, ngauge, ckpt, flags=0):
    """Adjoint/forward time ratio on the bathymetry-inversion batch: ninst
    instances of ncell cells, nsteps frozen CFL steps, gauge misfit at ngauge
    gauges per instance, checkpoints every ckpt steps (flags: the well-balanced
    form)."""
    import torch
    from paper_2208_06588_amd import alew, workloads as W
    t0 = time.perf_counter()
    bt = W.inversion_batch(ninst=ninst, n=ncell, ngauge=ngauge)
    log(f"adjoint workload: {ninst} x {ncell} cells ({time.perf_counter() - t0:.1f} s to build)")
    off = [int(v) for v in bt["cell_off"]]
    S = off[-1]
    p = alew.params(bc="transmissive", mesh="sine", mesh_A=0.05, mesh_k=1.0, mesh_omega=np.pi,
                    cfl=0.6, flags=flags)
    T = {k: torch.tensor(bt[k], dtype=torch.float64, device=dev)
         for k in ("h", "hu", "b", "x", "xi", "gauge_x", "b_true")}
    ctx = alew.Context(S, ninst)
    ctx.set_launch(engine=alew.ENGINE_STAGES, use_graph=1)
    # frozen step sizes: the CFL steps of a run from the initial state
    dts = torch.zeros(ninst * nsteps, dtype=torch.float64, device=dev)
    W0 = {k: T[k].clone() for k in ("h", "hu", "b", "x")}
    ctx.run(p, off, W0["h"], W0["hu"], W0["b"], W0["x"], T["xi"], max_steps=[nsteps] * ninst,
            dt_log=dts, dts_stride=nsteps)
    # observations from the same run over the "true" bottom
    gh_obs = torch.zeros(ninst * ngauge, dtype=torch.float64, device=dev)
    htrue = torch.clamp(T["h"] + T["b"] - T["b_true"], min=0.0)
    ctx.adjoint(p, off, htrue, T["hu"], T["b_true"], T["x"], T["xi"], nsteps, dts, ngauge,
                T["gauge_x"], gh_obs, None, ckpt_every=ckpt)
    # forward alone (same frozen steps)
    W1 = {k: T[k].clone() for k in ("h", "hu", "b", "x")}
    torch.cuda.synchronize()
    gc.collect()
    a = time.perf_counter()
    ctx.run(p, off, W1["h"], W1["hu"], W1["b"], W1["x"], T["xi"], max_steps=[nsteps] * ninst,
            dts=dts, dts_stride=nsteps)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - a
    # gradient of 0.5 |gauge_h - obs|^2: forward value, then the adjoint call
    gh = torch.zeros(ninst * ngauge, dtype=torch.float64, device=dev)
    ctx.adjoint(p, off, T["h"], T["hu"], T["b"], T["x"], T["xi"], nsteps, dts, ngauge,
                T["gauge_x"], gh, None, ckpt_every=ckpt)
    gbar = gh - gh_obs
    d3 = [torch.zeros(S, dtype=torch.float64, device=dev) for _ in range(3)]
    torch.cuda.synchronize()
    gc.collect()
    a = time.perf_counter()
    ctx.adjoint(p, off, T["h"], T["hu"], T["b"], T["x"], T["xi"], nsteps, dts, ngauge,
                T["gauge_x"], gh, gbar, *d3, ckpt_every=ckpt)
    torch.cuda.synchronize()
    t_adj = time.perf_counter() - a
    loss = float(0.5 * (gbar ** 2).sum())
    return dict(instances=ninst, cells=S, steps=nsteps, gauges_per_instance=ngauge,
                ckpt_every=ckpt, forward_s=round(t_fwd, 4), adjoint_s=round(t_adj, 4),
                ratio=round(t_adj / t_fwd, 3), loss=loss,
                grad_b_norm=float(torch.linalg.vector_norm(d3[2])),
                note="adjoint_s covers the checkpointed forward, the segment recomputation "
                     "and the reverse sweep")


def speedup_leg(p, off, T, tnow, L, k=64, steps=3):
    """Batched (one call for k instances) against one call per instance, same
    GPU, same k instances, same launch shape, from the state after the timed
    steps at each instance's own time.  Per-instance calls are timed two ways:
    warm, with one context per instance whose tile tables and step graph were
    built by an untimed call on the same arrays (launches and per-call host
    work only), and cold, with one shared context whose tables and graph are
    rebuilt for every instance (also the set-up a naive caller pays)."""
    import torch
    from paper_2208_06588_amd import alew
    sub_off = off[:k + 1]
    Ssub = sub_off[-1]

    def sub_state():
        return {kk: v[:Ssub + (k if kk in ("x", "xi") else 0)].clone() for kk, v in T.items()}

    def launch_of(c):
        c.set_launch(engine=L.engine, block=L.block, steps_per_launch=L.steps_per_launch,
                     use_graph=L.use_graph, cells_per_thread=L.cells_per_thread,
                     compact_tiles=L.compact_tiles)

    def one(c, Tp, i):
        c0, c1 = sub_off[i], sub_off[i + 1]
        return c.run(p, [0, c1 - c0], Tp["h"][c0:c1], Tp["hu"][c0:c1], Tp["b"][c0:c1],
                     Tp["x"][c0 + i:c1 + i + 1], Tp["xi"][c0 + i:c1 + i + 1], t0=[tnow[i]],
                     max_steps=[steps])

    ctxb = alew.Context(Ssub, k)
    launch_of(ctxb)
    Tb = sub_state()
    ctxb.run(p, sub_off, Tb["h"], Tb["hu"], Tb["b"], Tb["x"], Tb["xi"], t0=tnow[:k],
             max_steps=[steps] * k)  # untimed: tables and graph of the batch
    Tb = sub_state()
    torch.cuda.synchronize()
    gc.collect()
    a0 = time.perf_counter()
    ctxb.run(p, sub_off, Tb["h"], Tb["hu"], Tb["b"], Tb["x"], Tb["xi"], t0=tnow[:k],
             max_steps=[steps] * k)
    torch.cuda.synchronize()
    batched = time.perf_counter() - a0
    # warm: a context per instance, each built by one untimed call on its arrays
    ctxs = []
    Tw = sub_state()
    Tsave = sub_state()
    for i in range(k):
        c = alew.Context(sub_off[i + 1] - sub_off[i], 1)
        launch_of(c)
        one(c, Tw, i)
        ctxs.append(c)
    for kk in Tw:
        Tw[kk].copy_(Tsave[kk])
    torch.cuda.synchronize()
    gc.collect()
    a0 = time.perf_counter()
    for i in range(k):
        one(ctxs[i], Tw, i)
    torch.cuda.synchronize()
    warm = time.perf_counter() - a0
    for kk in ("h", "hu", "b", "x"):
        assert torch.equal(Tw[kk], Tb[kk]), f"per-instance result differs ({kk})"
    for c in ctxs:
        c.close()
    # cold: one context shared by the instances
    Tc = sub_state()
    c1 = alew.Context(max(np.diff(sub_off)), 1)
    launch_of(c1)
    torch.cuda.synchronize()
    gc.collect()
    a0 = time.perf_counter()
    for i in range(k):
        one(c1, Tc, i)
    torch.cuda.synchronize()
    cold = time.perf_counter() - a0
    c1.close()
    ctxb.close()
    return dict(instances=k, steps=steps, cells=int(Ssub), batched_s=round(batched, 4),
                per_instance_warm_s=round(warm, 4), per_instance_cold_s=round(cold, 4),
                speedup=round(warm / batched, 2), speedup_cold=round(cold / batched, 2),
                note="speedup: per-instance calls on warm per-instance contexts (no table or "
                     "graph rebuild); speedup_cold: one shared context rebuilding both per call")



def source_hash_2d():
    """Hash of the code (comments stripped) of the 2D kernels' sources."""
    h = hashlib.sha1()
    for f in ("alew2d.hip", "alew_device.h"):
        with open(os.path.join(ROOT, "paper_2208_06588_amd", "csrc", f)) as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


# FP64 vector peak of the MI355X: 256 CUs x 4 SIMDs x 2.4 GHz x 32 flops per cycle
FP64_PEAK_TFLOPS = 78.6


def tensor2d_leg(dev, n, steps, warmup):
    """The 2D tensor-product workload: n x n cells on [0,1]^2, periodic,
    b = sin 2 pi x + cos 2 pi y, h = 10 + exp(sin 2 pi x) cos 2 pi y,
    hu = sin(cos 2 pi x) sin 2 pi y, hv = cos 2 pi x cos(sin 2 pi y), nodes
    x = xi + 0.02 sin(2 pi xi) sin(pi t) and y likewise, CFL 0.6.  `steps`
    steps from t = 0 in one call (timed on the wall clock and by the library's
    events) after `warmup` untimed steps on a copy; then 3 steps with an event
    pair around every launch for the time split and the roofline of the
    dominant kernel (FP64 VALU-bound: counters from profiles/counters.json
    when they were taken on this source)."""
    import torch
    from paper_2208_06588_amd import alew, workloads as W
    wl = W.smooth_2d(n)
    p = alew.params2(cfl=0.6, Ax=wl["Ax"], kx=wl["kx"], omx=wl["omx"], Ay=wl["Ay"], ky=wl["ky"],
                     omy=wl["omy"])
    ctx = alew.Context2(n, n)
    T0 = {k: torch.tensor(wl[k], dtype=torch.float64, device=dev)
          for k in ("h", "hu", "hv", "b", "xi", "yi")}

    def fresh():
        T = {k: v.clone() for k, v in T0.items()}
        T["x"], T["y"] = T0["xi"].clone(), T0["yi"].clone()
        return T

    def go(T, nsteps, pp=None):
        return ctx.run(pp or p, T["h"], T["hu"], T["hv"], T["b"], T["x"], T["y"], T["xi"], T["yi"],
                       max_steps=nsteps)

    if warmup:
        go(fresh(), warmup)
    T = fresh()
    torch.cuda.synchronize()
    gc.collect()
    a = time.perf_counter()
    st = go(T, steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - a
    ev_ms = ctx.last_timing()
    assert st.status == 0 and st.steps == steps, "2D run did not complete"
    N = n * n
    ctx.set_kernel_timing(True)
    go(fresh(), 3)
    torch.cuda.synchronize()
    ctx.set_kernel_timing(False)
    names = ["k2_kin", "k2_xsweep<s>", "k2_ysweep<s>", "k2_fin"]
    split = {}
    for q, nm in enumerate(names):
        ms, nl = ctx.kernel_timing(q)
        split[nm] = dict(launches=nl, launch_ms=round(ms / max(1, nl), 4), ms_per_step=round(ms / 3, 4))
    dom = max(names, key=lambda k: split[k]["ms_per_step"])
    def variant(flags, name):
        """The same workload with another scheme: 20 steps after 2 untimed ones,
        and the x- and y-sweeps' launch times from a 3-step pass."""
        pv = alew.params2(cfl=0.6, Ax=wl["Ax"], kx=wl["kx"], omx=wl["omx"], Ay=wl["Ay"],
                          ky=wl["ky"], omy=wl["omy"], flags=flags)
        go(fresh(), 2, pv)
        Tv = fresh()
        torch.cuda.synchronize()
        a = time.perf_counter()
        stv = go(Tv, 20, pv)
        torch.cuda.synchronize()
        wall_v = time.perf_counter() - a
        assert stv.status == 0 and stv.steps == 20, f"2D {name} run did not complete"
        del Tv
        ctx.set_kernel_timing(True)
        go(fresh(), 3, pv)
        torch.cuda.synchronize()
        ctx.set_kernel_timing(False)
        xms, xn = ctx.kernel_timing(1)
        yms, yn = ctx.kernel_timing(2)
        return dict(steps=20, value=3.0 * N * 20 / wall_v, unit="cell-updates/s",
                    ms_per_step=round(wall_v * 1e3 / 20, 4),
                    xsweep_launch_ms=round(xms / max(1, xn), 4),
                    ysweep_launch_ms=round(yms / max(1, yn), 4))

    # the hydrostatic reconstruction (Sec. 4.1) and the scheme without
    # well-balancing (Sec. 3, characteristic sweeps)
    hydro = variant(alew.F_HYDROSTATIC, "hydrostatic")
    nonwb = variant(alew.F_NONWB, "nonwb")
    roof = dict(bound="alu", kernel=dom, achieved=None, peak=FP64_PEAK_TFLOPS, unit="TFLOP/s",
                frac=None, traffic=None, launch_ms=split[dom]["launch_ms"],
                timing="HIP events on the library stream around each launch")
    c = None
    try:
        with open(os.path.join(ROOT, "profiles", "counters.json")) as f:
            c = json.load(f).get(dom)
    except (OSError, ValueError):
        c = None
    if c is not None and c.get("source_hash") == source_hash_2d():
        flops = c["fp64_flops_per_cell_stage"] * N
        tf = flops / (split[dom]["launch_ms"] / 1e3) / 1e12
        roof.update(achieved=round(tf, 2), frac=round(tf / FP64_PEAK_TFLOPS, 4),
                    fp64_flops_per_cell_stage=round(c["fp64_flops_per_cell_stage"], 1),
                    valu_insts_per_wave=round(c["valu_per_wave"], 1),
                    traffic=round(c["hbm_bytes_per_cell_stage"] * N),
                    traffic_note="FETCH_SIZE x %.2f + WRITE_SIZE x %.2f per launch (copy-kernel "
                                 "calibration)" % (c["fetch_factor"], c["write_factor"]))
    elif c is not None:
        roof["note"] = "counters in profiles/counters.json were taken on another source"
    return dict(workload=f"2D tensor-product moving mesh, {n} x {n} cells FP64 on [0,1]^2, "
                         "periodic, smooth data of Example 5.6, node maps 0.02 sin(2 pi xi) "
                         "sin(pi t) per direction, CFL 0.6, special source-term scheme",
                steps=steps, value=3.0 * N * steps / wall, unit="cell-updates/s",
                ms_per_step=round(wall * 1e3 / steps, 4),
                event_ms_per_step=round(ev_ms / steps, 4), t_end=st.t,
                n_class=list(st.n_class), kernels=split, roofline=roof, hydrostatic=hydro,
                nonwb=nonwb)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--engine", default="auto", choices=["auto", "tune", "persistent", "stages"],
                    help="auto: the library's automatic launch (stage launches, one-wave tiles "
                         "of two cells per thread); tune: the autotuner's pick")
    ap.add_argument("--no-tune-report", action="store_true",
                    help="skip running the autotuner beside the automatic launch")
    ap.add_argument("--block", type=int, default=256)
    ap.add_argument("--graph", type=int, default=1, help="stage engine: replay steps as a hipGraph")
    ap.add_argument("--cpt", type=int, default=1, help="stage engine: cells per thread (1 or 2)")
    ap.add_argument("--compact", type=int, default=0,
                    help="stage engine: 1 = tiles without the four extra stencil slots")
    ap.add_argument("--ninst", type=int, default=4096)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-inst", type=int, default=64)
    ap.add_argument("--cpu-steps", type=int, default=30)
    ap.add_argument("--no-speedup", action="store_true",
                    help="skip the batched vs per-instance comparison")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint/forward ratio")
    ap.add_argument("--adj-ninst", type=int, default=256)
    ap.add_argument("--adj-cells", type=int, default=65536)
    ap.add_argument("--adj-steps", type=int, default=200)
    ap.add_argument("--no-bowl", action="store_true", help="skip the 2^24-cell wet/dry run")
    ap.add_argument("--oracle-suite", action="store_true",
                    help="CPU baseline: also time the oracle on the other configurations, "
                         "single threaded (about 2 minutes); and the 200-cell run on the GPU")
    ap.add_argument("--no-full-run", action="store_true",
                    help="skip timing the whole batch to t = 0.2 (every instance from t = 0 with "
                         "its own CFL steps, 609-12201 steps; about 45 s)")
    ap.add_argument("--bowl-steps", type=int, default=20)
    ap.add_argument("--scheme", default="special", choices=["special", "hydrostatic"],
                    help="well-balanced form of the timed forward leg (Sec. 4.2 special source "
                         "term, or Sec. 4.1 hydrostatic reconstruction)")
    ap.add_argument("--no-hydrostatic", action="store_true",
                    help="skip the hydrostatic-reconstruction legs (forward and adjoint)")
    ap.add_argument("--hr-steps", type=int, default=20)
    ap.add_argument("--no-2d", action="store_true", help="skip the 2048 x 2048 2D leg")
    ap.add_argument("--only-2d", action="store_true",
                    help="run only the 2D leg and print its object (profiling)")
    ap.add_argument("--n2d", type=int, default=2048)
    ap.add_argument("--steps-2d", type=int, default=100)
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="first copy a buffer of this many MiB (calibrates profiler byte counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the batched instances are independent and the "
              "figure is one GPU's throughput; use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2208_06588_amd import alew, autotune, workloads as W

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.copy_probe > 0:
        n = args.copy_probe * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"copy probe: {n * 8} bytes read, {n * 8} bytes written")
        del a, b
    if args.only_2d:
        print(json.dumps({"tensor2d": tensor2d_leg(dev, args.n2d, args.steps_2d, 2)}), flush=True)
        return
    t0 = time.perf_counter()
    bt = W.perturbation_batch(ninst=args.ninst) if args.ninst == 4096 else \
        W.perturbation_batch(subset=args.ninst)
    off = [int(v) for v in bt["cell_off"]]
    ninst = len(off) - 1
    S = off[-1]
    log(f"workload: {ninst} instances, {S} cells ({time.perf_counter() - t0:.1f} s to build)")
    hydro = args.scheme == "hydrostatic"
    p = alew.params(bc="transmissive", mesh="sine", mesh_A=0.05, mesh_k=1.0, mesh_omega=np.pi,
                    cfl=0.6, weno_eps=1e-9, flags=alew.F_HYDROSTATIC if hydro else 0)
    T = {k: torch.tensor(bt[k], dtype=torch.float64, device=dev) for k in ("h", "hu", "b", "x", "xi")}
    ctx = alew.Context(S, ninst)

    tune_report = None
    if args.engine in ("auto", "tune") and not (args.engine == "auto" and args.no_tune_report):
        best, times = autotune.tune(ctx, p, off, T, steps=2, use_cache=False, log=log)
        log(f"autotune picked {best}")
        tune_report = dict(picked=autotune.name_of(best),
                           first_round_ms={k: round(v * 1e3, 2) for k, v in times.items()})
    if args.engine == "auto":
        ctx.set_launch()  # the library's automatic launch
    elif args.engine == "tune":
        pass
    else:
        eng = alew.ENGINE_PERSISTENT if args.engine == "persistent" else alew.ENGINE_STAGES
        ctx.set_launch(engine=eng, block=args.block, use_graph=args.graph,
                       cells_per_thread=args.cpt, compact_tiles=args.compact)
    L = ctx.get_launch()
    engine_name = "persistent" if L.engine == alew.ENGINE_PERSISTENT else "stage-launches"

    # warmup (untimed), then exactly --steps steps in one call
    tnow = [0.0] * ninst
    if args.warmup > 0:
        st = ctx.run(p, off, T["h"], T["hu"], T["b"], T["x"], T["xi"], t0=tnow,
                     max_steps=[args.warmup] * ninst)
        tnow = [s.t for s in st]
    # the interpreter's cycle collector runs now, not inside the timed call
    gc.collect()
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    st = ctx.run(p, off, T["h"], T["hu"], T["b"], T["x"], T["xi"], t0=tnow,
                 max_steps=[args.steps] * ninst)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    kern_ms, launches = ctx.last_timing()
    assert all(s.steps == args.steps and s.status == 0 for s in st), "run did not complete"
    cell_stages = 3.0 * S * args.steps
    value = cell_stages / wall
    log(f"timed {args.steps} steps: {wall * 1e3:.1f} ms wall, {kern_ms:.1f} ms in {launches} "
        f"compute launch(es); {value:.3e} cell-updates/s")

    roof = roofline(ctx, p, off, T, tnow=[s.t for s in st], L=L, S=S, kern_ms=kern_ms,
                    launches=launches, steps=args.steps, copy_bw=args.copy_probe == 0)
    # the whole step (stage kernels, per-instance reductions, step epilogue,
    # node update and step-size reductions) against the same algorithmic bytes
    step_gbs = ALG_BYTES_PER_CELL_STEP * S * args.steps / wall / 1e9
    roof["step_level"] = dict(achieved=round(step_gbs, 1), frac=round(step_gbs / HBM_PEAK_GBS, 4),
                              alg_bytes_per_cell_step=ALG_BYTES_PER_CELL_STEP,
                              timing="wall clock of the timed call")

    out = {
        "metric": METRIC, "value": value, "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"ragged batch of {ninst} 1D perturbation-of-still-water "
                               f"instances, 1000-20000 cells each (seed 2208065881), {S} cells, "
                               "transmissive, sine-moving mesh, CFL 0.6, FP64 SSP-RK3, "
                               + ("hydrostatic reconstruction" if hydro else
                                  "special source-term treatment"),
                   "ninst": ninst, "cells": S, "engine": engine_name,
                   "block": L.block or (256 if L.engine == alew.ENGINE_PERSISTENT else 64),
                   "cells_per_thread": L.cells_per_thread or
                   (2 if L.engine != alew.ENGINE_PERSISTENT and L.block in (0, 64) else 1),
                   "compact_tiles": int(L.compact_tiles),
                   "parallelism": "single GPU"},
        "roofline": roof,
    }
    if tune_report is not None:
        out["autotune"] = tune_report

    if not hydro and not args.no_hydrostatic and L.engine != alew.ENGINE_PERSISTENT:
        # the hydrostatic-reconstruction scheme on the same batch, same launch
        p_hr = alew.params(bc="transmissive", mesh="sine", mesh_A=0.05, mesh_k=1.0,
                           mesh_omega=np.pi, cfl=0.6, weno_eps=1e-9, flags=alew.F_HYDROSTATIC)
        tn = [s.t for s in st]
        out["hydrostatic"] = guarded("hydrostatic", lambda: hydrostatic_leg(
            ctx, p_hr, off, T, tn, L, S, args.hr_steps))
        log(f"hydrostatic: {out['hydrostatic']}")

    if not args.no_full_run:
        # the whole job: every instance from its initial state at t = 0 to t = 0.2 in one call
        W2 = {k: torch.tensor(bt[k], dtype=torch.float64, device=dev)
              for k in ("h", "hu", "b", "x", "xi")}
        torch.cuda.synchronize()
        gc.collect()
        a0 = time.perf_counter()
        stf = ctx.run(p, off, W2["h"], W2["hu"], W2["b"], W2["x"], W2["xi"], t_end=[0.2] * ninst)
        torch.cuda.synchronize()
        wall_f = time.perf_counter() - a0
        assert all(s.status == 0 and abs(s.t - 0.2) < 1e-12 for s in stf), "full run did not finish"
        ns = np.diff(off)
        work = float(sum(3.0 * int(ns[i]) * stf[i].steps for i in range(ninst)))
        out["full_run"] = dict(t_end=0.2, wall_s=round(wall_f, 3), cell_stages=work,
                               value=work / wall_f, unit="cell-updates/s",
                               steps_min=int(min(s.steps for s in stf)),
                               steps_max=int(max(s.steps for s in stf)))
        log(f"full run: {out['full_run']}")
        del W2

    if not args.no_speedup:
        out["batched_speedup"] = guarded("batched speedup", lambda: speedup_leg(
            p, off, T, [s.t for s in st], L))
        log(f"batched speedup: {out['batched_speedup']}")

    if not args.no_bowl:
        out["bowl"] = guarded("bowl", lambda: bowl_leg(dev, 1 << 24, args.bowl_steps, 2))
        log(f"bowl: {out['bowl']}")

    if not args.no_2d:
        out["tensor2d"] = guarded("2D", lambda: tensor2d_leg(dev, args.n2d, args.steps_2d, 2))
        log(f"2D: {out['tensor2d']}")
        torch.cuda.empty_cache()

    if not args.no_adjoint:
        del ctx, T
        torch.cuda.empty_cache()
        out["adjoint"] = guarded("adjoint", lambda: adjoint_leg(
            dev, args.adj_ninst, args.adj_cells, args.adj_steps, 64, 16))
        out["adjoint_forward_ratio"] = out["adjoint"].get("ratio")
        if not args.no_hydrostatic:
            torch.cuda.empty_cache()
            out["adjoint_hydrostatic"] = guarded("adjoint (hydrostatic)", lambda: adjoint_leg(
                dev, args.adj_ninst, args.adj_cells, args.adj_steps, 64, 16,
                flags=alew.F_HYDROSTATIC))
            log(f"adjoint (hydrostatic reconstruction): {out['adjoint_hydrostatic']}")
        log(f"adjoint: {out['adjoint']}")

    if args.oracle_suite:
        log("smooth 200-cell run on the GPU ...")
        out["smooth_200_gpu"] = guarded("smooth 200-cell run", lambda: small_run_leg(dev))
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = guarded("cpu baseline", lambda: cpu_baseline(
            bt, min(args.cpu_inst, ninst), args.cpu_steps))
        log("class flips against the oracle ...")
        out["class_flips"] = guarded("class flips", lambda: class_flips_leg(
            dev, bt, min(32, ninst), args.cpu_steps))
        log(f"class flips: {out['class_flips']}")
        if args.oracle_suite:
            log("oracle on the other configurations ...")
            out["cpu_baseline"]["other_configs"] = guarded("oracle, other configurations",
                                                           oracle_other_configs)
            log(f"oracle, other configurations: {out['cpu_baseline']['other_configs']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
