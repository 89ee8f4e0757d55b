"""alew_step_noalloc (the step without a context or device allocation) against
alew_step, through the C ABI: two calls in a row, the second on a smaller
instance, each compared bit for bit (same kernels, same arithmetic) with
alew_step on the same inputs, and with the oracle at the parity bar."""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_common import assert_parity, gparams, oparams, t64
from paper_2208_06588_amd import alew, workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    torch.cuda.set_device(0)
    return torch.device("cuda", 0)


def _both(wl, dev, steps, flags=0):
    """steps calls of alew_step_noalloc and of alew_step from the same state."""
    n = len(wl["h"])
    p = gparams(wl, flags=flags)
    A = {k: t64(wl[k], dev) for k in ("h", "hu", "b", "x", "xi")}
    B = {k: t64(wl[k], dev) for k in ("h", "hu", "b", "x", "xi")}
    ca = torch.zeros(3 * n, dtype=torch.uint8, device=dev)
    cb = torch.zeros(3 * n, dtype=torch.uint8, device=dev)
    ctx = alew.Context(n, 1)
    ta = tb = 0.0
    for _ in range(steps):
        sa = alew.step_noalloc(p, A["h"], A["hu"], A["b"], A["x"], A["xi"], t=ta, cls=ca)
        sb = ctx.step(p, B["h"], B["hu"], B["b"], B["x"], B["xi"], t=tb, cls=cb)
        ta, tb = sa.t, sb.t
        assert torch.equal(ca, cb)
    torch.cuda.synchronize()
    ctx.close()
    return A, B, sa, sb


@pytest.mark.parametrize("hydro", [False, True])
def test_noalloc_step_equals_alew_step_twice_shrinking(dev, hydro):
    flags = alew.F_HYDROSTATIC if hydro else 0
    # first call: a 4000-cell perturbation instance; second: the 200-cell smooth case
    big = W.perturbation_instance(4000, 5e-3)
    wl_big = dict(xi=big[0], x=big[0].copy(), h=big[1], hu=big[2], b=big[3], bc="transmissive",
                  cfl=0.6, weno_eps=1e-9, mesh="sine", mesh_A=0.05, mesh_k=1.0, mesh_omega=np.pi)
    wl_small = W.accuracy_1d(200)
    for wl, steps in ((wl_big, 3), (wl_small, 5)):
        A, B, sa, sb = _both(wl, dev, steps, flags)
        for k in ("h", "hu", "b", "x"):
            assert torch.equal(A[k], B[k]), k
        assert sa.steps == sb.steps == 1 and sa.t == sb.t and sa.status == sb.status == 0
        assert tuple(sa.n_class) == tuple(sb.n_class) and sa.n_limited == sb.n_limited
        r = O.run(oparams(wl, flags=O.FLAG_HYDROSTATIC if hydro else 0), wl["h"], wl["hu"],
                  wl["b"], wl["x"], wl["xi"], max_steps=steps)
        assert_parity({k: v.cpu().numpy() for k, v in A.items()}, r)


def test_noalloc_step_rejects_sizes_beyond_its_scratch(dev):
    n = alew.NOALLOC_MAX_CELLS + 1
    z = torch.zeros(n, dtype=torch.float64, device=dev)
    xn = torch.linspace(0.0, 1.0, n + 1, dtype=torch.float64, device=dev)
    with pytest.raises(alew.AlewError) as ei:
        alew.step_noalloc(alew.params(), z + 1.0, z, z, xn, xn.clone())
    assert ei.value.status == alew.E_ARG
    assert "65536" in str(ei.value)
