"""C-ABI checks that need no GPU: the library loads, exports every symbol
the header declares, validates arguments before touching a device, and its
structs have the layout the header gives them."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1011_2775_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wcmg.h")


def header_symbols():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(wcmg_\w+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    syms = header_symbols()
    assert len(syms) >= 20
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIBPATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (wcmg_\w+)", out))
    missing = [s for s in syms if s not in exported]
    assert not missing, missing
    for s in syms:
        getattr(_lib.LIB, s)


def test_params_default():
    p = _lib.MGParams()
    assert _lib.LIB.wcmg_mg_params_default(ctypes.byref(p)) == _lib.OK
    assert p.nlevels == 1 and p.nvec[0] == 24 and list(p.block[0]) == [4, 4, 4, 4]
    assert abs(p.tol[0] - 0.1) < 1e-15 and p.nu_post == 4 and p.smoother_prec == _lib.F32
    assert _lib.LIB.wcmg_mg_params_default(None) == _lib.EINVAL


def test_create_validates_before_device():
    lat = (_lib.Lattice * 1)()
    for m, d in enumerate((4, 4, 5, 4)):
        lat[0].dims[m] = d
    lat[0].t_bc = -1
    h = ctypes.c_void_p()
    assert _lib.LIB.wcmg_create(lat, 1, None, ctypes.byref(h)) == _lib.EDIM
    assert b"even" in _lib.LIB.wcmg_last_error()
    lat[0].dims[2] = 4
    lat[0].t_bc = 0
    assert _lib.LIB.wcmg_create(lat, 1, None, ctypes.byref(h)) == _lib.EINVAL
    assert _lib.LIB.wcmg_create(lat, 0, None, ctypes.byref(h)) == _lib.EINVAL
    assert _lib.LIB.wcmg_create(lat, 1, None, None) == _lib.EINVAL


def test_null_context_rejected():
    L = _lib.LIB
    assert L.wcmg_destroy(None) == _lib.EINVAL
    assert L.wcmg_set_gauge(None, 0, None, 0) == _lib.EINVAL
    assert L.wcmg_set_clover(None, 0, 0.0, 1.0, None, 0) == _lib.EINVAL
    assert L.wcmg_apply_D(None, 0, 0, 0, None, None, 1) == _lib.EINVAL
    assert L.wcmg_solve(None, 0, 0, None, None, 1, 1e-10, None) == _lib.EINVAL
    assert L.wcmg_build_null_vectors(None, 0, 0) == _lib.EINVAL
    assert L.wcmg_timer_enable(None, 1) == _lib.EINVAL


def test_create_without_gpu_reports_enodev():
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is visible")
    lat = (_lib.Lattice * 1)()
    for m in range(4):
        lat[0].dims[m] = 4
    lat[0].t_bc = -1
    h = ctypes.c_void_p()
    assert _lib.LIB.wcmg_create(lat, 1, None, ctypes.byref(h)) == _lib.ENODEV


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text('''
#include <stdio.h>
#include <stddef.h>
#include "wcmg.h"
int main(void) {
  printf("%zu %zu %zu\\n", sizeof(wcmg_lattice), sizeof(wcmg_mg_params), sizeof(wcmg_stats));
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", offsetof(wcmg_mg_params, tol), offsetof(wcmg_mg_params, nu_post),
         offsetof(wcmg_mg_params, setup_rq_tol), offsetof(wcmg_mg_params, seed), offsetof(wcmg_mg_params, coarsest),
         offsetof(wcmg_mg_params, cycle_mode), offsetof(wcmg_mg_params, setup_prec),
         offsetof(wcmg_mg_params, coarse_launch), offsetof(wcmg_mg_params, plain_max_iter), offsetof(wcmg_mg_params, mp_inner_tol),
         offsetof(wcmg_mg_params, coarse_fp16), offsetof(wcmg_mg_params, transfer_fp16));
  printf("%zu %zu %zu %zu\\n", offsetof(wcmg_stats, inner_iters), offsetof(wcmg_stats, true_rel_res),
         offsetof(wcmg_stats, status), offsetof(wcmg_stats, inner_status));
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    lines = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    sizes = [int(v) for v in lines[0].split()]
    assert sizes == [ctypes.sizeof(_lib.Lattice), ctypes.sizeof(_lib.MGParams), ctypes.sizeof(_lib.Stats)]
    offs = [int(v) for v in lines[1].split()]
    M = _lib.MGParams
    assert offs == [M.tol.offset, M.nu_post.offset, M.setup_rq_tol.offset, M.seed.offset, M.coarsest.offset,
                    M.cycle_mode.offset, M.setup_prec.offset, M.coarse_launch.offset, M.plain_max_iter.offset,
                    M.mp_inner_tol.offset, M.coarse_fp16.offset, M.transfer_fp16.offset]
    offs = [int(v) for v in lines[2].split()]
    S = _lib.Stats
    assert offs == [S.inner_iters.offset, S.true_rel_res.offset, S.status.offset, S.inner_status.offset]
