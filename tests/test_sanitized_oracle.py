"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (host
code only; g++), driven through its Python binding in a subprocess on small
cases of every scheme, the jump-aligned mesh with the projected step, the tape
adjoint and the 2D scheme in its three forms (a dry bed included): no invalid
access, overflow or undefined behaviour is reported."""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "alew_oracle.cpp")

DRIVER = r'''
import numpy as np
import oracle as O
from paper_2208_06588_amd import workloads as W

assert O.lib()._name.endswith("liboracle_san.so"), O.lib()._name
wl = W.accuracy_1d(32)
for fl in (0, O.FLAG_HYDROSTATIC, O.FLAG_NONWB, O.FLAG_ALPHA_CELLAVG | O.FLAG_NO_HU_LIMIT,
           O.FLAG_W_TANGENT):
    P = O.params(bc=O.BC_PERIODIC, mesh=O.MESH_SINE, mesh_A=0.05, mesh_k=1.0,
                 mesh_omega=np.pi, flags=fl)
    r = O.run(P, wl["h"], wl["hu"], wl["b"], wl["x"], wl["xi"], max_steps=4, record_cls=True)
    assert r["status"] == 0, (fl, r["status"])
P = O.params(bc=O.BC_PERIODIC, mesh=O.MESH_SINE, mesh_A=0.05, mesh_k=1.0, mesh_omega=np.pi,
             bottom=O.BOTTOM_SIN2, bottom_p=(1.0, 1.0, 0.0, 0.0))
assert O.run(P, wl["h"], wl["hu"], wl["b"], wl["x"], wl["xi"], max_steps=3)["status"] == 0
wb = W.bowl_1d(64)
P = O.params(bc=O.BC_TRANSMISSIVE, mesh=O.MESH_FLUID, cfl=0.08)
r = O.run(P, wb["h"], wb["hu"], wb["b"], wb["x"], wb["xi"], max_steps=3)
for bc in (O.BC_TRANSMISSIVE, O.BC_REFLECTIVE):
    P = O.params(bc=bc, mesh=O.MESH_SINE, mesh_A=0.05, mesh_k=1.0, mesh_omega=np.pi)
    O.run(P, wl["h"], wl["hu"], wl["b"], wl["x"], wl["xi"], max_steps=2)
P = O.params(bc=O.BC_PERIODIC, mesh=O.MESH_SINE, mesh_A=0.05, mesh_k=1.0, mesh_omega=np.pi)
gx = np.array([0.2, 0.5, 0.8])
out = O.adjoint(P, wl["h"], wl["hu"], wl["b"], wl["x"], wl["xi"], [1e-3] * 3, gx, np.ones(3))
assert out[-1] == 0
wd = W.dam_break_bump_1d(24, 15.0)
P = O.params(bc=O.BC_TRANSMISSIVE, mesh=O.MESH_ALIGNED, mesh_A=1.0, mesh_k=0.0,
             mesh_omega=wd["mesh_omega"], bottom=O.BOTTOM_STEP, bottom_p=wd["bottom_p"])
assert O.run(P, wd["h"], wd["hu"], wd["b"], wd["x"], wd["xi"], max_steps=3)["status"] == 0
w2 = W.accuracy_2d(8)
for fl in (0, O.FLAG_HYDROSTATIC, O.FLAG_NONWB):
    P2 = O.params2(Ax=w2["Ax"], kx=1.0, omx=w2["omx"], Ay=w2["Ay"], ky=1.0, omy=w2["omy"],
                   bcy=O.BC_TRANSMISSIVE, flags=fl)
    r2 = O.run2(P2, w2["h"], w2["hu"], w2["hv"], w2["b"], w2["xi"], w2["yi"], w2["xi"], w2["yi"],
                max_steps=2, record_cls=True)
    assert r2["status"] == 0, (fl, r2["status"])
wdb = W.dam_break_2d(8, 8, t_end=1.75)
P2 = O.params2(cfl=0.08, dry_eps=1e-6, Ax=wdb["Ax"], kx=wdb["kx"], omx=wdb["omx"], Ay=wdb["Ay"],
               ky=wdb["ky"], omy=wdb["omy"], bcx=O.BC_TRANSMISSIVE, bcy=O.BC_TRANSMISSIVE,
               flags=O.FLAG_NONWB)
r2 = O.run2(P2, wdb["h"], wdb["hu"], wdb["hv"], wdb["b"], wdb["xi"], wdb["yi"], wdb["xi"],
            wdb["yi"], max_steps=3)
assert r2["status"] == 0, r2["status"]
print("sanitized oracle ok")
'''


@pytest.mark.slow
def test_oracle_under_asan_and_ubsan():
    with tempfile.TemporaryDirectory() as d:
        lib = os.path.join(d, "liboracle_san.so")
        subprocess.check_call(
            ["g++", "-O1", "-g", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
             "-shared", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
             "-fno-omit-frame-pointer", "-o", lib, SRC])
        asan = subprocess.check_output(["g++", "-print-file-name=libasan.so"], text=True).strip()
        ubsan = subprocess.check_output(["g++", "-print-file-name=libubsan.so"], text=True).strip()
        env = dict(os.environ, ALEW_ORACLE_LIB=lib, LD_PRELOAD=f"{asan}:{ubsan}",
                   ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1",
                   PYTHONPATH=ROOT + os.pathsep + os.environ.get("PYTHONPATH", ""))
        r = subprocess.run([sys.executable, "-c", DRIVER], cwd=ROOT, env=env, capture_output=True,
                           text=True, timeout=600)
        assert r.returncode == 0 and "sanitized oracle ok" in r.stdout, r.stdout + r.stderr[-4000:]
        assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
