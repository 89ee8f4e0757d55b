"""Helpers shared by the GPU test files: device tensors, parameter structs for
both sides (library and oracle) from one workload dict, the parity measure,
and the class record of an oracle run (per-cell counts and sequence
signature, as alew_run defines them)."""
import numpy as np
import torch

import oracle as O
from paper_2208_06588_amd import alew

TOL = 1e-11  # relative L-inf bar of the FP64 parity tests


def t64(a, dev):
    return torch.tensor(np.asarray(a), dtype=torch.float64, device=dev)


def gparams(wl, **kw):
    d = dict(bc=wl["bc"], mesh=wl["mesh"], mesh_A=wl["mesh_A"], mesh_k=wl["mesh_k"],
             mesh_omega=wl["mesh_omega"], cfl=wl["cfl"], weno_eps=wl["weno_eps"])
    d.update(kw)
    return alew.params(**d)


def oparams(wl, **kw):
    bc = dict(periodic=O.BC_PERIODIC, transmissive=O.BC_TRANSMISSIVE, reflective=O.BC_REFLECTIVE)
    mesh = dict(given=O.MESH_GIVEN, sine=O.MESH_SINE, paper=O.MESH_PAPER, fluid=O.MESH_FLUID,
                aligned=O.MESH_ALIGNED)
    d = dict(bc=bc[wl["bc"]], mesh=mesh[wl["mesh"]], mesh_A=wl["mesh_A"], mesh_k=wl["mesh_k"],
             mesh_omega=wl["mesh_omega"], cfl=wl["cfl"], weno_eps=wl["weno_eps"])
    d.update(kw)
    return O.params(**d)


def relerr(g, r):
    g = np.asarray(g)
    r = np.asarray(r)
    return float(np.abs(g - r).max() / max(1.0, np.abs(r).max()))


def assert_parity(g, r, fields=("h", "hu", "b", "x"), tol=TOL, tag=""):
    for k in fields:
        e = relerr(g[k], r[k])
        assert e <= tol, (tag, k, e)


def run_one(ctx, p, wl, dev, **kw):
    """alew_run of one instance; returns host arrays and its stats."""
    n = len(wl["h"])
    t = {k: t64(wl[k], dev) for k in ("h", "hu", "b", "x", "xi")}
    st = ctx.run(p, [0, n], t["h"], t["hu"], t["b"], t["x"], t["xi"], **kw)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in t.items()}, st[0]


def class_record(cls_steps):
    """Per-cell counts ([3, n]) and sequence signature ([n], uint64) of the
    classes an oracle run recorded ([steps, 3 stages, n]), as alew_run
    accumulates them: sig <- sig * CLS_SIG_MUL + class + 1 (mod 2^64) at every
    stage in time order."""
    cls_steps = np.asarray(cls_steps)
    n = cls_steps.shape[-1]
    counts = np.stack([(cls_steps == c).sum(axis=(0, 1)) for c in range(3)]).astype(np.int64)
    sig = np.zeros(n, dtype=np.uint64)
    mul = np.uint64(alew.CLS_SIG_MUL)
    with np.errstate(over="ignore"):
        for k in range(cls_steps.shape[0]):
            for s in range(3):
                sig = sig * mul + (cls_steps[k, s].astype(np.uint64) + np.uint64(1))
    return counts, sig


def class_flips(counts_gpu, sig_gpu, counts_ref, sig_ref):
    """Cells whose class sequences differ (signatures), and a lower bound on the
    number of flipped cell-stages (half the count differences)."""
    cells = int((np.asarray(sig_gpu, dtype=np.uint64) != np.asarray(sig_ref, np.uint64)).sum())
    lower = int(np.abs(np.asarray(counts_gpu, np.int64) - np.asarray(counts_ref, np.int64)).sum()) // 2
    return cells, lower
