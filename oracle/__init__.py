"""Oracle for the 1D well-balanced ALE-WENO hybrid scheme (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: a plain, slow, serial FP64 CPU implementation of
the scheme of Zhang, Xia & Xu (arXiv 2208.06588) in ``alew_oracle.cpp``.
Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  It shares no code with the GPU library.

Every function documents the passage of the paper it follows; the readings
of ambiguous passages are listed at the top of ``alew_oracle.cpp``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "alew_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
# ALEW_ORACLE_LIB: load a separately built copy (the sanitizer test's build of
# the same source) instead of building and loading liboracle.so
_LIB_OVERRIDE = os.environ.get("ALEW_ORACLE_LIB")

BC_PERIODIC, BC_TRANSMISSIVE, BC_REFLECTIVE = 0, 1, 2
MESH_GIVEN, MESH_SINE, MESH_PAPER, MESH_FLUID, MESH_ALIGNED = 0, 1, 2, 3, 4
ST_OK, ST_ARG, ST_MESH, ST_NEGDEPTH, ST_NONFINITE, ST_NEGWEIGHT = 0, 1, 2, 3, 4, 8
FLAG_BETA_LOCAL, FLAG_BETA_FROM_H, FLAG_HYDROSTATIC = 1, 2, 4
FLAG_ALPHA_CELLAVG, FLAG_NO_HU_LIMIT, FLAG_W_TANGENT, FLAG_NONWB = 8, 16, 32, 64
FLAG_SPLIT = 128  # negative linear weights split instead of reported (R29)


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


class Params2(C.Structure):
    """Constants of the 2D tensor-product scheme (nodes move per direction:
    x = xi + Ax sin(2 pi kx xi) sin(omx t), y likewise)."""
    _fields_ = [
        ("g", C.c_double), ("cfl", C.c_double), ("weno_eps", C.c_double), ("dry_eps", C.c_double),
        ("Ax", C.c_double), ("kx", C.c_double), ("omx", C.c_double),
        ("Ay", C.c_double), ("ky", C.c_double), ("omy", C.c_double),
        ("bcx", C.c_int32), ("bcy", C.c_int32), ("flags", C.c_int32), ("pad", C.c_int32),
        ("Vx", C.c_double), ("Vy", C.c_double),
    ]


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (no FMA contraction, IEEE division/sqrt)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        # a name of its own per process: worker processes that start together
        # may build at once, and each renames a complete library into place
        tmp = f"{_LIB}.{os.getpid()}.tmp"
        subprocess.check_call(
            ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
             "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            L = C.CDLL(_LIB_OVERRIDE)
        else:
            build()
            L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        u8p = C.POINTER(C.c_uint8)
        L.orc_geometry.argtypes = [dp, dp, dp, dp, dp]
        L.orc_reconstruct.argtypes = [dp, dp, dp, dp, dp, C.c_double, C.c_double, dp, dp, dp]
        L.orc_limit.argtypes = [C.c_double, C.c_double, dp, C.c_double, C.c_int, dp]
        L.orc_bottom_average.argtypes = [C.POINTER(Params), C.c_double, C.c_double]
        L.orc_bottom_average.restype = C.c_double
        L.orc_nonlinear_weights.argtypes = [dp, dp, C.c_int, dp]
        L.orc_nonlinear_weights.restype = None
        L.orc_reconstruct_char.argtypes = [dp, dp, dp, dp, C.c_double, C.c_double, C.c_double,
                                           C.c_double, dp]
        L.orc_hydro_source.argtypes = [C.c_double, dp, dp]
        L.orc_hydro_source.restype = C.c_double
        L.orc_residual.argtypes = [C.POINTER(Params), C.c_int64, dp, dp, dp, dp, dp, dp, dp, u8p]
        L.orc_mesh_velocity.argtypes = [C.POINTER(Params), C.c_int64, dp, dp, dp, dp, C.c_double,
                                        C.c_double, dp]
        L.orc_run.argtypes = [C.POINTER(Params), C.c_int64, dp, dp, dp, dp, dp, dp, C.c_double,
                              C.c_double, C.c_int64, dp, dp, u8p, C.POINTER(Stats)]
        L.orc_adjoint.argtypes = [C.POINTER(Params), C.c_int64, dp, dp, dp, dp, dp, C.c_double,
                                  C.c_int64, dp, C.c_int64, dp, dp, dp, dp, dp, dp]
        L.orc2_run.argtypes = [C.POINTER(Params2), C.c_int64, C.c_int64, dp, dp, dp, dp, dp, dp,
                               dp, dp, C.c_double, C.c_double, C.c_int64, dp,
                               C.POINTER(C.c_int64), u8p, C.POINTER(C.c_int64), dp,
                               C.POINTER(C.c_int64), dp, C.c_int64]
        L.orc2_limit_edges.argtypes = [C.c_double, C.c_double, C.c_double, dp]
        L.orc2_limit_edges.restype = C.c_int
        L.orc2_sweep.argtypes = [dp, C.c_double, C.c_double, dp, dp, dp, dp, dp, dp, dp]
        L.orc2_residual.argtypes = [C.POINTER(Params2), C.c_int64, C.c_int64, dp, dp, dp, dp, dp,
                                    dp, dp, dp, dp]
        L.orc2_residual.restype = C.c_double
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


BOTTOM_ALE, BOTTOM_STEP, BOTTOM_GAUSS, BOTTOM_SIN2, BOTTOM_BUMP, BOTTOM_PARABOLA = range(6)


def params(g=9.812, cfl=0.6, weno_eps=1e-6, pp_eps=1e-11, bc=BC_PERIODIC, mesh=MESH_SINE,
           mesh_A=0.05, mesh_k=1.0, mesh_omega=np.pi, flags=0, dry_eps=1e-8, bottom=BOTTOM_ALE,
           bottom_p=(0.0, 0.0, 0.0, 0.0)) -> Params:
    """Scheme constants: g (Sec. 5), CFL, WENO epsilon (Sec. 2.2 Step 2),
    positivity epsilon (eq. (3.20)), boundary type, mesh motion, the dry
    tolerance of the trace velocity, and the bottom (evolved by eq. (3.17), or
    an analytic b(x) projected onto the cells, eq. (3.16))."""
    return Params(g, cfl, weno_eps, pp_eps, mesh_A, mesh_k, mesh_omega, dry_eps, bc, mesh, flags,
                  bottom, (C.c_double * 4)(*[float(v) for v in bottom_p]))


def geometry(widths5):
    """Stencil polynomials and linear weights of one cell (Sec. 2.2, Step 1).

    Returns (d[4,3], c[3,4,3], cd[3,4,3], a[3,3,3]) at the 4 Gauss-Lobatto
    points s = 0, 1/2 -+ sqrt(5)/10, 1 of the cell."""
    w = _f64(widths5)
    d = np.zeros((4, 3)); c = np.zeros((3, 4, 3)); cd = np.zeros((3, 4, 3)); a = np.zeros((3, 3, 3))
    lib().orc_geometry(_p(w), _p(d), _p(c), _p(cd), _p(a))
    return d, c, cd, a


def reconstruct(widths5, h5, m5, b5, dx, eps=1e-6, v5=None):
    """Unlimited hybrid WENO values of one cell (Sec. 2.2 Steps 2-4, eq. (2.10)).

    v5 is the first indicator variable (default eta = h + b).
    Returns (vals[16] = h[4], hu[4], b[4], b_x[4]; cls; beta[3]; gamma)."""
    h5, m5, b5 = _f64(h5), _f64(m5), _f64(b5)
    v5 = h5 + b5 if v5 is None else _f64(v5)
    out = np.zeros(16); beta = np.zeros(3); gam = np.zeros(1)
    cls = lib().orc_reconstruct(_p(_f64(widths5)), _p(v5), _p(h5), _p(m5), _p(b5),
                                float(dx), float(eps), _p(out), _p(beta), _p(gam))
    return out, cls, beta, float(gam[0])


def bottom_average(P: Params, xl, xr):
    """Average over [xl, xr] of the analytic bottom of P (eq. (3.16))."""
    return float(lib().orc_bottom_average(C.byref(P), float(xl), float(xr)))


def nonlinear_weights(d, K, split=True):
    """Nonlinear weights of one point from linear weights d[3] and the factors
    K[3] = 1 + (tau / (beta_r + eps))^2 (split: the splitting of R29)."""
    phi = np.zeros(3)
    lib().orc_nonlinear_weights(_p(_f64(d)), _p(_f64(K)), 1 if split else 0, _p(phi))
    return phi


def limit_edges2(hbar, mbar, nbar, e):
    """The directional positivity limiter of one cell (eq. (3.21) / (3.22))
    on its two opposite edges: e[2][4][4] = (side, Gauss-Lobatto
    point, h / hu / hv / b).  Returns (limited copy, acted)."""
    t = np.array(e, dtype=np.float64).reshape(32).copy()
    r = lib().orc2_limit_edges(C.c_double(hbar), C.c_double(mbar), C.c_double(nbar), _p(t))
    return t.reshape(2, 4, 4), bool(r)


def reconstruct_char(widths5, eta5, m5, b5, dx, eps=1e-6, g=9.812, dry_eps=1e-8):
    """Unlimited reconstruction of one cell of the scheme without
    well-balancing (Sec. 3; characteristic variables of the cell's mean
    state, b on its own).  Returns (vals[16] = h[4], hu[4], b[4], b_x[4]; cls)."""
    out = np.zeros(16)
    cls = lib().orc_reconstruct_char(_p(_f64(widths5)), _p(_f64(eta5)), _p(_f64(m5)),
                                     _p(_f64(b5)), float(dx), float(eps), float(g),
                                     float(dry_eps), _p(out))
    return out, cls


def limit(hbar, mbar, traces6, pp_eps=1e-11, hu_lim=True):
    """1D positivity limiter (eq. (3.20)-(3.21), Remark 4.1) on (hL,huL,bL,hR,huR,bR);
    hu_lim=False leaves the hu traces alone."""
    out = np.zeros(6)
    r = lib().orc_limit(float(hbar), float(mbar), _p(_f64(traces6)), float(pp_eps),
                        1 if hu_lim else 0, _p(out))
    return out, r


def hydro_source(g, eta4, b4):
    """Hydrostatic source of one cell (Sec. 4.1, after eq. (4.3)) from eta and b
    at the 4 Gauss-Lobatto points (cell ends first and last)."""
    return float(lib().orc_hydro_source(float(g), _p(_f64(eta4)), _p(_f64(b4))))


def residual(P: Params, eta, hu, b, J, w):
    """Semi-discrete right-hand side (eq. (3.12), (3.17), (4.7)-(4.10)).

    Returns (R[3,n] for (eta, hu, b), alpha, cls[n])."""
    eta, hu, b, J, w = map(_f64, (eta, hu, b, J, w))
    n = eta.size
    R = np.zeros(3 * n); al = np.zeros(1); cls = np.zeros(n, np.uint8)
    lib().orc_residual(C.byref(P), n, _p(eta), _p(hu), _p(b), _p(J), _p(w), _p(R), _p(al),
                       cls.ctypes.data_as(C.POINTER(C.c_uint8)))
    return R.reshape(3, n), float(al[0]), cls


def mesh_velocity(P: Params, h, hu, b, xi, t, dt):
    """Node speeds of the step [t, t+dt] for the prescribed or fluid mesh."""
    h, hu, b, xi = map(_f64, (h, hu, b, xi))
    w = np.zeros(h.size + 1)
    lib().orc_mesh_velocity(C.byref(P), h.size, _p(h), _p(hu), _p(b), _p(xi), float(t), float(dt),
                            _p(w))
    return w


def run(P: Params, h, hu, b, x, xi=None, w=None, t0=0.0, t_end=0.0, max_steps=0, dts=None,
        record_cls=False):
    """Time-march the scheme (eq. (3.14)-(3.15)) from t0 to t_end and/or for
    max_steps steps.  Returns dict(h, hu, b, x, t, stats, status, cls)."""
    h, hu, b, x = (_f64(a).copy() for a in (h, hu, b, x))
    n = h.size
    xi_a = None if xi is None else _f64(xi)
    w_a = None if w is None else _f64(w)
    dts_a = None if dts is None else _f64(dts)
    nrec = max_steps if max_steps > 0 else 0
    cls = np.zeros((nrec, 3, n), np.uint8) if (record_cls and nrec > 0) else None
    S = Stats()
    t = np.zeros(1)
    st = lib().orc_run(C.byref(P), n, _p(h), _p(hu), _p(b), _p(x), _p(xi_a), _p(w_a), float(t0),
                       float(t_end), int(max_steps), _p(dts_a), _p(t),
                       None if cls is None else cls.ctypes.data_as(C.POINTER(C.c_uint8)),
                       C.byref(S))
    return dict(h=h, hu=hu, b=b, x=x, t=float(t[0]), stats=S, status=st, cls=cls)


def adjoint(P: Params, h0, hu0, b0, x0, xi, dts, gauge_x, gauge_bar, t0=0.0):
    """Exact discrete adjoint of the oracle run with frozen step sizes.

    gauge_h[g] = hbar(T) of the cell containing gauge_x[g]; returns
    (gauge_h, dh0, dhu0, db0) for the functional sum_g gauge_bar[g] gauge_h[g]."""
    h0, hu0, b0, x0, xi, dts, gx, gb = map(_f64, (h0, hu0, b0, x0, xi, dts, gauge_x, gauge_bar))
    n = h0.size
    gh = np.zeros(gx.size); dh = np.zeros(n); dhu = np.zeros(n); db = np.zeros(n)
    st = lib().orc_adjoint(C.byref(P), n, _p(h0), _p(hu0), _p(b0), _p(x0), _p(xi), float(t0),
                           dts.size, _p(dts), gx.size, _p(gx), _p(gh), _p(gb), _p(dh), _p(dhu),
                           _p(db))
    return gh, dh, dhu, db, st


# ---------------------------------------------------------------------------
# 2D tensor-product extension
# ---------------------------------------------------------------------------
def params2(g=9.812, cfl=0.6, weno_eps=1e-6, dry_eps=1e-8, Ax=0.02, kx=1.0, omx=np.pi, Ay=0.02,
            ky=1.0, omy=np.pi, bcx=BC_PERIODIC, bcy=BC_PERIODIC, flags=0, Vx=0.0,
            Vy=0.0) -> Params2:
    """2D scheme constants; flags: 0 (special source term, Sec. 4.2) or
    FLAG_HYDROSTATIC (hydrostatic reconstruction, Sec. 4.1, R31)."""
    return Params2(g, cfl, weno_eps, dry_eps, Ax, kx, omx, Ay, ky, omy, bcx, bcy, int(flags), 0,
                   float(Vx), float(Vy))


def sweep2(widths5, e5, mx5, my5, h5, b5, dx, eps=1e-6, ext5=None):
    """One sweep of the 2D dimension-by-dimension reconstruction on 5 cells.
    Returns (out[6, 4] = h, hu, hv, b, db/ds, ext at the 4 Gauss-Lobatto
    points of the middle cell; class)."""
    out = np.zeros(24)
    ext = None if ext5 is None else _f64(ext5)
    c = lib().orc2_sweep(_p(_f64(widths5)), float(dx), float(eps), _p(_f64(e5)), _p(_f64(mx5)),
                         _p(_f64(my5)), _p(_f64(h5)), _p(_f64(b5)), _p(ext), _p(out))
    return out.reshape(6, 4), c


def residual2(P: Params2, eta, hu, hv, b, dx, dy, wx, wy):
    """Semi-discrete right-hand side of the 2D scheme; arrays [ny, nx]."""
    eta, hu, hv, b = (_f64(a) for a in (eta, hu, hv, b))
    ny, nx = eta.shape
    R = np.zeros(4 * nx * ny)
    al = lib().orc2_residual(C.byref(P), nx, ny, _p(eta), _p(hu), _p(hv), _p(b), _p(_f64(dx)),
                             _p(_f64(dy)), _p(_f64(wx)), _p(_f64(wy)), _p(R))
    return R.reshape(4, ny, nx), al


def run2(P: Params2, h, hu, hv, b, x, y, xi, yi, t0=0.0, t_end=0.0, max_steps=0,
         record_cls=False, record_dts=0):
    """Time-march the 2D scheme; arrays [ny, nx] (row j, column i).  Returns
    dict(h, hu, hv, b, x, y, t, steps, status, n_class, mass, cls, n_limited,
    dts: the step sizes of the first record_dts steps)."""
    h, hu, hv, b, x, y = (_f64(a).copy() for a in (h, hu, hv, b, x, y))
    ny, nx = h.shape
    t = np.zeros(1)
    steps = C.c_int64()
    ncls = (C.c_int64 * 3)()
    mass = np.zeros(4)
    cls = np.zeros((max_steps, 3, ny, nx), np.uint8) if (record_cls and max_steps > 0) else None
    nlim = C.c_int64()
    dts = np.zeros(int(record_dts)) if record_dts > 0 else None
    st = lib().orc2_run(C.byref(P), nx, ny, _p(h), _p(hu), _p(hv), _p(b), _p(x), _p(y),
                        _p(_f64(xi)), _p(_f64(yi)), float(t0), float(t_end), int(max_steps),
                        _p(t), C.byref(steps), None if cls is None else
                        cls.ctypes.data_as(C.POINTER(C.c_uint8)), ncls, _p(mass), C.byref(nlim),
                        _p(dts), int(record_dts))
    if dts is not None:
        dts = dts[:min(steps.value, dts.size)]
    return dict(h=h, hu=hu, hv=hv, b=b, x=x, y=y, t=float(t[0]), steps=steps.value, status=st,
                n_class=list(ncls), mass=mass, cls=cls, n_limited=nlim.value, dts=dts)
