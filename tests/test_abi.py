"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every
entry point declared in include/alew.h, and the ctypes structures have the
header's layout."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "alew.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(alew(?:2d)?_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("alew_create", "alew_destroy", "alew_step", "alew_run", "alew_adjoint",
              "alew_last_error", "alew_set_launch", "alew2d_create", "alew2d_run"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2208_06588_amd import alew
    L = alew.lib()
    for n in _declared():
        assert hasattr(L, n), n
    assert alew.version().startswith("alew")
    assert L.alew_last_error() is not None


def test_struct_layout_matches_header():
    from paper_2208_06588_amd import alew
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "alew.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu\n", sizeof(alew_params), offsetof(alew_params, bc),
         offsetof(alew_params, dry_eps), sizeof(alew_stats), offsetof(alew_stats, t),
         offsetof(alew_stats, status), sizeof(alew_launch));
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(alew2d_params), offsetof(alew2d_params, bcx),
         offsetof(alew2d_params, omy), sizeof(alew2d_stats), offsetof(alew2d_stats, n_class),
         offsetof(alew2d_stats, status));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), "-o", exe, c])
        got = [int(v) for v in subprocess.check_output([exe]).split()]
    P, S, L = alew.Params, alew.Stats, alew.Launch
    P2, S2 = alew.Params2, alew.Stats2
    want = [C.sizeof(P), P.bc.offset, P.dry_eps.offset, C.sizeof(S), S.t.offset, S.status.offset,
            C.sizeof(L), C.sizeof(P2), P2.bcx.offset, P2.omy.offset, C.sizeof(S2),
            S2.n_class.offset, S2.status.offset]
    assert got == want


def test_binding_rejects_host_tensors():
    import torch
    from paper_2208_06588_amd import alew
    with pytest.raises(ValueError):
        alew._ptr(torch.zeros(4, dtype=torch.float64))
