"""Thin ctypes binding of ``libalew.so`` (C ABI in include/alew.h).

Argument marshalling only: every step of the scheme runs in the HIP kernels.
PyTorch provides device memory and the stream.  If the library is missing
this module raises at load time; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libalew.so")

(OK, E_ARG, E_MESH, E_NEGDEPTH, E_NONFINITE, E_HIP, E_NOMEM, E_UNSUPPORTED, E_NEGWEIGHT,
 E_CAPACITY) = range(10)
BC = {"periodic": 0, "transmissive": 1, "reflective": 2}
MESH = {"given": 0, "sine": 1, "paper": 2, "fluid": 3, "aligned": 4}
F_BETA_LOCAL, F_BETA_FROM_H, F_HYDROSTATIC = 1, 2, 4
F_ALPHA_CELLAVG, F_NO_HU_LIMIT, F_W_TANGENT, F_NONWB = 8, 16, 32, 64
F_SPLIT = 128  # split negative linear weights instead of reporting them
CLS_SIG_MUL = 1099511628211  # multiplier of the class-sequence signature of alew_run
ENGINE_AUTO, ENGINE_PERSISTENT, ENGINE_STAGES = 0, 1, 2


class Params(C.Structure):
    _fields_ = [
        ("g", C.c_double), ("cfl", C.c_double), ("weno_eps", C.c_double), ("pp_eps", C.c_double),
        ("mesh_A", C.c_double), ("mesh_k", C.c_double), ("mesh_omega", C.c_double),
        ("dry_eps", C.c_double),
        ("bc", C.c_int32), ("mesh", C.c_int32), ("flags", C.c_int32), ("bottom", C.c_int32),
        ("bottom_p", C.c_double * 4),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("steps", C.c_int64), ("n_class", C.c_int64 * 3), ("n_limited", C.c_int64),
        ("n_negweight", C.c_int64),
        ("t", C.c_double), ("dt_min", C.c_double), ("dt_max", C.c_double), ("h_min", C.c_double),
        ("mass_eta0", C.c_double), ("mass_eta", C.c_double), ("mass_b0", C.c_double),
        ("mass_b", C.c_double),
        ("status", C.c_int32), ("pad", C.c_int32),
    ]

    def as_dict(self):
        return {k: (list(getattr(self, k)) if k == "n_class" else getattr(self, k))
                for k, _ in self._fields_ if k != "pad"}


class Launch(C.Structure):
    _fields_ = [("engine", C.c_int32), ("block", C.c_int32), ("steps_per_launch", C.c_int32),
                ("use_graph", C.c_int32), ("cells_per_thread", C.c_int32),
                ("compact_tiles", C.c_int32)]


class Params2(C.Structure):
    """alew2d_params: the 2D tensor-product scheme (nodes move per direction,
    x = xi + Ax sin(2 pi kx xi) sin(omx t), y likewise)."""
    _fields_ = [
        ("g", C.c_double), ("cfl", C.c_double), ("weno_eps", C.c_double), ("dry_eps", C.c_double),
        ("Ax", C.c_double), ("kx", C.c_double), ("omx", C.c_double),
        ("Ay", C.c_double), ("ky", C.c_double), ("omy", C.c_double),
        ("bcx", C.c_int32), ("bcy", C.c_int32), ("flags", C.c_int32), ("pad", C.c_int32),
        ("Vx", C.c_double), ("Vy", C.c_double),
    ]


class Stats2(C.Structure):
    _fields_ = [
        ("steps", C.c_int64), ("t", C.c_double), ("dt_min", C.c_double), ("dt_max", C.c_double),
        ("mass0", C.c_double), ("mass_b0", C.c_double), ("mass", C.c_double),
        ("mass_b", C.c_double), ("n_class", C.c_int64 * 3), ("n_limited", C.c_int64),
        ("status", C.c_int32), ("pad", C.c_int32),
    ]

    def as_dict(self):
        return {k: (list(getattr(self, k)) if k == "n_class" else getattr(self, k))
                for k, _ in self._fields_ if k != "pad"}


class AlewError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"alew status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() first")
        L = C.CDLL(LIB_PATH)
        vp, dp, i64 = C.c_void_p, C.POINTER(C.c_double), C.c_int64
        L.alew_create.argtypes = [C.POINTER(vp), i64, i64, vp]
        L.alew_destroy.argtypes = [vp]
        L.alew_set_stream.argtypes = [vp, vp]
        L.alew_set_launch.argtypes = [vp, C.POINTER(Launch)]
        L.alew_get_launch.argtypes = [vp, C.POINTER(Launch)]
        L.alew_step.argtypes = [vp, C.POINTER(Params), i64, vp, vp, vp, vp, vp, vp, C.c_double,
                                C.c_double, C.c_double, vp, C.POINTER(Stats)]
        L.alew_run.argtypes = [vp, C.POINTER(Params), i64, C.POINTER(C.c_int64), vp, vp, vp, vp, vp,
                               dp, dp, C.POINTER(C.c_int64), vp, vp, i64, vp, vp,
                               C.POINTER(Stats)]
        L.alew_adjoint_reserve.argtypes = [vp, i64, i64, i64]
        L.alew_step_noalloc.argtypes = [C.POINTER(Params), i64, vp, vp, vp, vp, vp, vp, C.c_double,
                                        C.c_double, C.c_double, vp, C.POINTER(Stats), vp]
        L.alew_adjoint.argtypes = [vp, C.POINTER(Params), i64, C.POINTER(C.c_int64), vp, vp, vp,
                                   vp, vp, C.c_double, i64, vp, i64, i64, vp, vp, vp, vp, vp, vp]
        L.alew_last_timing.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.alew_last_timing.restype = C.c_int
        L.alew_set_kernel_timing.argtypes = [vp, C.c_int]
        L.alew_set_kernel_timing.restype = C.c_int
        L.alew_kernel_timing.argtypes = [vp, C.c_int, C.POINTER(C.c_double),
                                         C.POINTER(C.c_int64), C.POINTER(C.c_double)]
        L.alew_kernel_timing.restype = C.c_int
        L.alew2d_create.argtypes = [C.POINTER(vp), i64, i64, vp]
        L.alew2d_destroy.argtypes = [vp]
        L.alew2d_set_stream.argtypes = [vp, vp]
        L.alew2d_set_launch.argtypes = [vp, C.c_int32, C.c_int32]
        L.alew2d_last_timing.argtypes = [vp, C.POINTER(C.c_double)]
        L.alew2d_set_kernel_timing.argtypes = [vp, C.c_int]
        L.alew2d_kernel_timing.argtypes = [vp, C.c_int, C.POINTER(C.c_double),
                                           C.POINTER(C.c_int64)]
        L.alew2d_run.argtypes = [vp, C.POINTER(Params2), i64, i64, vp, vp, vp, vp, vp, vp, vp, vp,
                                 C.c_double, C.c_double, i64, vp, vp, vp, C.POINTER(Stats2)]
        L.alew_last_error.restype = C.c_char_p
        L.alew_version.restype = C.c_char_p
        for f in ("alew_create", "alew_set_stream", "alew_set_launch", "alew_get_launch",
                  "alew_step", "alew_run", "alew_adjoint", "alew_adjoint_reserve",
                  "alew_step_noalloc", "alew2d_create", "alew2d_set_stream",
                  "alew2d_set_launch", "alew2d_last_timing", "alew2d_run",
                  "alew2d_set_kernel_timing", "alew2d_kernel_timing"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


BOTTOM = {"ale": 0, "step": 1, "gauss": 2, "sin2": 3, "bump": 4, "parabola": 5}


def params(g=9.812, cfl=0.6, weno_eps=1e-6, pp_eps=1e-11, dry_eps=1e-8, bc="periodic",
           mesh="sine", mesh_A=0.05, mesh_k=1.0, mesh_omega=3.141592653589793, flags=0,
           bottom="ale", bottom_p=(0.0, 0.0, 0.0, 0.0)) -> Params:
    return Params(g, cfl, weno_eps, pp_eps, mesh_A, mesh_k, mesh_omega, dry_eps,
                  BC[bc] if isinstance(bc, str) else int(bc),
                  MESH[mesh] if isinstance(mesh, str) else int(mesh), int(flags),
                  BOTTOM[bottom] if isinstance(bottom, str) else int(bottom),
                  (C.c_double * 4)(*[float(v) for v in bottom_p]))


def _ptr(t: Optional[torch.Tensor], dtype=torch.float64):
    if t is None:
        return None
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"expected a contiguous {dtype} CUDA tensor, got {t.dtype} "
                         f"{'cuda' if t.is_cuda else 'cpu'} contiguous={t.is_contiguous()}")
    return C.c_void_p(t.data_ptr())


def _sizes(ncell, ninst, h, hu, b, x, xi, w):
    """Host-side shape checks: the kernels index exactly these extents."""
    for name, t in (("h", h), ("hu", hu), ("b", b)):
        if t.numel() != ncell:
            raise ValueError(f"{name} has {t.numel()} entries, expected {ncell}")
    for name, t in (("x", x), ("xi", xi), ("w", w)):
        if t is not None and t.numel() != ncell + ninst:
            raise ValueError(f"{name} has {t.numel()} entries, expected {ncell + ninst}")


def _check(st):
    if st != OK:
        raise AlewError(st, lib().alew_last_error().decode())


class Context:
    """Owns the library's scratch memory for up to max_cells cells in
    max_inst instances; work goes to the current torch stream."""

    def __init__(self, max_cells: int, max_inst: int = 1, device=None):
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.max_cells, self.max_inst = int(max_cells), int(max_inst)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream().cuda_stream
            _check(lib().alew_create(C.byref(h), self.max_cells, self.max_inst, C.c_void_p(stream)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().alew_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync_stream(self):
        _check(lib().alew_set_stream(self._h, C.c_void_p(torch.cuda.current_stream().cuda_stream)))

    def set_launch(self, engine=ENGINE_AUTO, block=0, steps_per_launch=0, use_graph=1,
                   cells_per_thread=0, compact_tiles=0):
        _check(lib().alew_set_launch(self._h, C.byref(Launch(engine, block, steps_per_launch,
                                                             use_graph, cells_per_thread,
                                                             compact_tiles))))

    def last_timing(self):
        """(milliseconds, launches) of the compute launches of the last call."""
        ms, n = C.c_double(), C.c_int64()
        _check(lib().alew_last_timing(self._h, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def set_kernel_timing(self, on=True):
        """Event pairs around every stage launch and step epilogue of later
        runs (the step sequence then runs without a graph)."""
        _check(lib().alew_set_kernel_timing(self._h, 1 if on else 0))

    def kernel_timing(self, which=0):
        """(milliseconds, launches, cells) summed over the stage launches
        (which=0), the step epilogues (which=1) or the stage launches of RK
        stage 1, 2, 3 (which=2, 3, 4) of the last timed run."""
        ms, n, cells = C.c_double(), C.c_int64(), C.c_double()
        _check(lib().alew_kernel_timing(self._h, which, C.byref(ms), C.byref(n), C.byref(cells)))
        return ms.value, n.value, cells.value

    def get_launch(self) -> Launch:
        l = Launch()
        _check(lib().alew_get_launch(self._h, C.byref(l)))
        return l

    def step(self, p: Params, h, hu, b, x, xi=None, w=None, t=0.0, dt=0.0, t_end=0.0, cls=None,
             check=True) -> Stats:
        """One SSP-RK3 step of one instance; tensors are updated in place."""
        n = h.numel()
        _sizes(n, 1, h, hu, b, x, xi, w)
        if n > self.max_cells:
            raise ValueError("more cells than the context holds")
        if cls is not None and cls.numel() != 3 * n:
            raise ValueError("cls must hold 3 * ncell entries")
        self._sync_stream()
        S = Stats()
        st = lib().alew_step(self._h, C.byref(p), h.numel(), _ptr(h), _ptr(hu), _ptr(b), _ptr(x),
                             _ptr(xi), _ptr(w), float(t), float(dt), float(t_end),
                             _ptr(cls, torch.uint8), C.byref(S))
        if check:
            _check(st)
        S.status = st if st else S.status
        return S

    def run(self, p: Params, cell_off: Sequence[int], h, hu, b, x, xi, t0=None, t_end=None,
            max_steps=None, dts=None, dt_log=None, dts_stride=0, cls_count=None, cls_sig=None,
            check=True):
        """Run a packed ragged batch; returns the per-instance Stats (a ctypes
        array: index it or iterate over it).  cls_count
        (int32, 3 * cells) and cls_sig (int64, cells) accumulate the class record
        of every cell and stage (see alew_run)."""
        ninst = len(cell_off) - 1
        S = int(cell_off[-1])
        _sizes(S, ninst, h, hu, b, x, xi, None)
        for d in (dts, dt_log):
            if d is not None and d.numel() < ninst * dts_stride:
                raise ValueError("dts/dt_log must hold ninst * dts_stride entries")
        if (cls_count is None) != (cls_sig is None):
            raise ValueError("cls_count and cls_sig go together")
        if cls_count is not None and (cls_count.numel() != 3 * S or cls_sig.numel() != S):
            raise ValueError("cls_count must hold 3 * cells entries and cls_sig one per cell")
        self._sync_stream()
        off = (C.c_int64 * len(cell_off))(*[int(v) for v in cell_off])
        n = len(cell_off) - 1

        def darr(v):
            if v is None:
                return None
            v = [float(a) for a in (v if hasattr(v, "__len__") else [v] * n)]
            return (C.c_double * n)(*v)

        def iarr(v):
            if v is None:
                return None
            v = [int(a) for a in (v if hasattr(v, "__len__") else [v] * n)]
            return (C.c_int64 * n)(*v)

        stats = (Stats * n)()
        st = lib().alew_run(self._h, C.byref(p), n, off, _ptr(h), _ptr(hu), _ptr(b), _ptr(x),
                            _ptr(xi), darr(t0), darr(t_end), iarr(max_steps), _ptr(dts),
                            _ptr(dt_log), int(dts_stride), _ptr(cls_count, torch.int32),
                            _ptr(cls_sig, torch.int64), stats)
        if check:
            _check(st)
        # the ctypes array itself (indexable, iterable): no per-instance Python
        # objects are made inside the call
        return stats

    def adjoint_reserve(self, nsteps, ngauge, ckpt_every=16):
        """Allocate the adjoint workspace for up to nsteps steps and ngauge gauges
        per instance at the context's capacity."""
        _check(lib().alew_adjoint_reserve(self._h, int(nsteps), int(ckpt_every), int(ngauge)))

    def adjoint(self, p: Params, cell_off, h0, hu0, b0, x0, xi, nsteps, dts, ngauge, gauge_x,
                gauge_h, gauge_bar=None, dh0=None, dhu0=None, db0=None, ckpt_every=16, t0=0.0):
        """Gauge depths after nsteps frozen steps (gauge_h, out) and, when
        gauge_bar is given, the gradients of sum(gauge_bar * gauge_h) with
        respect to h0, hu0, b0 (written into dh0, dhu0, db0)."""
        ninst = len(cell_off) - 1
        S = int(cell_off[-1])
        _sizes(S, ninst, h0, hu0, b0, x0, xi, None)
        if dts.numel() < ninst * nsteps:
            raise ValueError("dts must hold ninst * nsteps step sizes")
        for t in (gauge_x, gauge_h, gauge_bar):
            if t is not None and t.numel() != ninst * ngauge:
                raise ValueError("gauge arrays must hold ninst * ngauge entries")
        for t in (dh0, dhu0, db0):
            if t is not None and t.numel() != S:
                raise ValueError("gradient arrays must hold one entry per cell")
        self._sync_stream()
        off = (C.c_int64 * len(cell_off))(*[int(v) for v in cell_off])
        st = lib().alew_adjoint(self._h, C.byref(p), ninst, off, _ptr(h0), _ptr(hu0),
                                _ptr(b0), _ptr(x0), _ptr(xi), float(t0), int(nsteps), _ptr(dts),
                                int(ckpt_every), int(ngauge), _ptr(gauge_x), _ptr(gauge_h),
                                _ptr(gauge_bar), _ptr(dh0), _ptr(dhu0), _ptr(db0))
        _check(st)


NOALLOC_MAX_CELLS = 65536


def step_noalloc(p: Params, h, hu, b, x, xi=None, w=None, t=0.0, dt=0.0, t_end=0.0, cls=None,
                 check=True) -> Stats:
    """alew_step_noalloc: one step of one instance without a context and without
    device allocation (the library's static scratch; ncell <= 65536), on the
    current torch stream."""
    n = h.numel()
    _sizes(n, 1, h, hu, b, x, xi, w)
    if cls is not None and cls.numel() != 3 * n:
        raise ValueError("cls must hold 3 * ncell entries")
    S = Stats()
    st = lib().alew_step_noalloc(C.byref(p), n, _ptr(h), _ptr(hu), _ptr(b), _ptr(x), _ptr(xi),
                                 _ptr(w), float(t), float(dt), float(t_end),
                                 _ptr(cls, torch.uint8), C.byref(S),
                                 C.c_void_p(torch.cuda.current_stream().cuda_stream))
    if check:
        _check(st)
    S.status = st if st else S.status
    return S


def params2(g=9.812, cfl=0.6, weno_eps=1e-6, dry_eps=1e-8, Ax=0.02, kx=1.0,
            omx=3.141592653589793, Ay=0.02, ky=1.0, omy=3.141592653589793, bcx="periodic",
            bcy="periodic", flags=0, Vx=0.0, Vy=0.0) -> Params2:
    """flags: 0 (special source term), F_HYDROSTATIC (hydrostatic reconstruction)
    or F_NONWB (without well-balancing, characteristic sweeps)."""
    bc = lambda v: BC[v] if isinstance(v, str) else int(v)
    return Params2(g, cfl, weno_eps, dry_eps, Ax, kx, omx, Ay, ky, omy, bc(bcx), bc(bcy),
                   int(flags), 0, float(Vx), float(Vy))


class Context2:
    """Workspace of the 2D tensor-product scheme for grids up to max_nx x
    max_ny cells; work goes to the current torch stream."""

    def __init__(self, max_nx: int, max_ny: int, device=None):
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.max_nx, self.max_ny = int(max_nx), int(max_ny)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream().cuda_stream
            _check(lib().alew2d_create(C.byref(h), self.max_nx, self.max_ny, C.c_void_p(stream)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().alew2d_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_launch(self, rows=16, check_every=8):
        _check(lib().alew2d_set_launch(self._h, int(rows), int(check_every)))

    def last_timing(self) -> float:
        """Device milliseconds of the last run (events around its launches)."""
        ms = C.c_double()
        _check(lib().alew2d_last_timing(self._h, C.byref(ms)))
        return ms.value

    def set_kernel_timing(self, on=True):
        """Event pairs around every launch of later runs."""
        _check(lib().alew2d_set_kernel_timing(self._h, 1 if on else 0))

    def kernel_timing(self, which):
        """(milliseconds, launches) of the last run for which = 0 kinematics,
        1 x-sweeps, 2 y-sweeps, 3 step epilogues (with kernel timing on)."""
        ms, n = C.c_double(), C.c_int64()
        _check(lib().alew2d_kernel_timing(self._h, int(which), C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def run(self, p: Params2, h, hu, hv, b, x, y, xi, yi, t0=0.0, t_end=0.0, max_steps=0,
            cls=None, cls_count=None, cls_sig=None, check=True) -> Stats2:
        """Advance the [ny, nx] state in place; returns Stats2.  cls (uint8,
        3 nx ny): classes of the last step; cls_count (int32, 3 nx ny) and
        cls_sig (int64, nx ny): the class record of the run."""
        if h.dim() != 2:
            raise ValueError("state tensors are [ny, nx]")
        ny, nx = h.shape
        for name, t in (("hu", hu), ("hv", hv), ("b", b)):
            if tuple(t.shape) != (ny, nx):
                raise ValueError(f"{name} must be [{ny}, {nx}]")
        for name, t, n in (("x", x, nx + 1), ("xi", xi, nx + 1), ("y", y, ny + 1),
                           ("yi", yi, ny + 1)):
            if t.numel() != n:
                raise ValueError(f"{name} must hold {n} nodes")
        for name, t, n in (("cls", cls, 3 * nx * ny), ("cls_count", cls_count, 3 * nx * ny),
                           ("cls_sig", cls_sig, nx * ny)):
            if t is not None and t.numel() != n:
                raise ValueError(f"{name} must hold {n} entries")
        _check(lib().alew2d_set_stream(self._h, C.c_void_p(torch.cuda.current_stream().cuda_stream)))
        S = Stats2()
        st = lib().alew2d_run(self._h, C.byref(p), nx, ny, _ptr(h), _ptr(hu), _ptr(hv), _ptr(b),
                              _ptr(x), _ptr(y), _ptr(xi), _ptr(yi), float(t0), float(t_end),
                              int(max_steps), _ptr(cls, torch.uint8), _ptr(cls_count, torch.int32),
                              _ptr(cls_sig, torch.int64), C.byref(S))
        if check:
            _check(st)
        S.status = st if st else S.status
        return S


def version() -> str:
    return lib().alew_version().decode()


class _GaugeFn(torch.autograd.Function):
    """gauge_h = G(h0, hu0, b0); backward runs alew_adjoint with the incoming
    gradient as gauge_bar (checkpointed recomputation of the forward)."""

    @staticmethod
    def forward(fctx, h0, hu0, b0, problem):
        gh = torch.empty(problem.ninst * problem.ngauge, dtype=torch.float64, device=h0.device)
        problem.ctx.adjoint(problem.p, problem.cell_off, h0.contiguous(), hu0.contiguous(),
                            b0.contiguous(), problem.x0, problem.xi, problem.nsteps, problem.dts,
                            problem.ngauge, problem.gauge_x, gh, None, ckpt_every=problem.ckpt_every,
                            t0=problem.t0)
        fctx.save_for_backward(h0, hu0, b0)
        fctx.problem = problem
        return gh

    @staticmethod
    def backward(fctx, grad):
        h0, hu0, b0 = fctx.saved_tensors
        pr = fctx.problem
        gh = torch.empty_like(grad)
        dh, dhu, db = (torch.empty_like(h0) for _ in range(3))
        pr.ctx.adjoint(pr.p, pr.cell_off, h0.contiguous(), hu0.contiguous(), b0.contiguous(), pr.x0,
                       pr.xi, pr.nsteps, pr.dts, pr.ngauge, pr.gauge_x, gh,
                       grad.contiguous().to(torch.float64), dh, dhu, db,
                       ckpt_every=pr.ckpt_every, t0=pr.t0)
        return dh, dhu, db, None


class GaugeProblem:
    """Differentiable map from an initial state (h0, hu0, b0) to the mean depths
    at gauges after nsteps frozen steps on a prescribed moving mesh.

    >>> G = GaugeProblem(ctx, params, cell_off, x0, xi, nsteps, dts, gauge_x, ngauge)
    >>> loss = 0.5 * ((G(h0, hu0, b0) - obs) ** 2).sum(); loss.backward()
    """

    def __init__(self, ctx: Context, p: Params, cell_off, x0, xi, nsteps, dts, gauge_x, ngauge,
                 ckpt_every=16, t0=0.0):
        self.ctx, self.p, self.cell_off = ctx, p, [int(v) for v in cell_off]
        self.ninst = len(self.cell_off) - 1
        self.x0, self.xi, self.nsteps, self.dts = x0, xi, int(nsteps), dts
        self.gauge_x, self.ngauge = gauge_x, int(ngauge)
        self.ckpt_every, self.t0 = int(ckpt_every), float(t0)

    def __call__(self, h0, hu0, b0):
        return _GaugeFn.apply(h0, hu0, b0, self)
