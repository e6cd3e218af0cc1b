"""CPU checks of the boundary: the HIP library loads and exports every function
include/vpp.h declares, and the header compiles as C."""
import ctypes
import os
import subprocess

import pytest

import paper_2401_07805_amd as vpp
from paper_2401_07805_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _ensure_built():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2401_07805_amd import build
        build.build(verbose=False)


def test_library_exports_every_declared_symbol():
    _ensure_built()
    names = _lib.declared_functions()
    assert len(names) >= 20
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert vpp.load().vpp_abi_version() == 1


def test_header_is_plain_c(tmp_path):
    src = tmp_path / "t.c"
    src.write_text('#include "vpp.h"\nint main(void){vpp_desc d; (void)d; (void)&vpp_abi_version; return 0;}\n')
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Werror", "-fsyntax-only",
                           "-I", os.path.join(ROOT, "include"), str(src)])


def test_struct_layouts_match_header(tmp_path):
    """Sizes and field offsets of the ctypes mirrors equal the C compiler's."""
    src = tmp_path / "l.c"
    src.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "vpp.h"
int main(void){
  printf("%zu %zu %zu %zu %zu\n", sizeof(vpp_desc), offsetof(vpp_desc, origin), offsetof(vpp_desc, degree),
         offsetof(vpp_desc, rho_l), offsetof(vpp_desc, device));
  printf("%zu %zu %zu %zu %zu\n", sizeof(vpp_cg_opts), offsetof(vpp_cg_opts, inner_rtol), offsetof(vpp_cg_opts, check_every),
         offsetof(vpp_cg_opts, deflate), offsetof(vpp_cg_opts, deflate_history));
  printf("%zu %zu %zu %zu\n", sizeof(vpp_cg_info), offsetof(vpp_cg_info, rel_residual),
         offsetof(vpp_cg_info, deflation_corrections), offsetof(vpp_cg_info, deflation_first_change));
  printf("%zu %zu\n", sizeof(vpp_kernel_config), offsetof(vpp_kernel_config, variant));
  printf("%zu %zu %zu\n", sizeof(vpp_cp_opts), offsetof(vpp_cp_opts, max_iter), offsetof(vpp_cp_opts, normal_steps));
  printf("%zu %zu\n", sizeof(vpp_reinit_opts), offsetof(vpp_reinit_opts, max_iter));
  return 0;}
''')
    exe = tmp_path / "l"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split("\n")
    D, O, I, K = _lib.Desc, _lib.CgOpts, _lib.CgInfo, _lib.KernelConfig
    assert out[0].split() == [str(v) for v in (ctypes.sizeof(D), D.origin.offset, D.degree.offset,
                                                D.rho_l.offset, D.device.offset)]
    assert out[1].split() == [str(v) for v in (ctypes.sizeof(O), O.inner_rtol.offset, O.check_every.offset,
                                               O.deflate.offset, O.deflate_history.offset)]
    assert out[2].split() == [str(v) for v in (ctypes.sizeof(I), I.rel_residual.offset,
                                               I.deflation_corrections.offset, I.deflation_first_change.offset)]
    assert out[3].split() == [str(v) for v in (ctypes.sizeof(K), K.variant.offset)]
    P = _lib.CpOpts
    assert out[4].split() == [str(v) for v in (ctypes.sizeof(P), P.max_iter.offset, P.normal_steps.offset)]
    R = _lib.ReinitOpts
    assert out[5].split() == [str(v) for v in (ctypes.sizeof(R), R.max_iter.offset)]


def test_candidates_listed_without_gpu():
    _ensure_built()
    for k in (2, 3, 4):
        c = vpp.config_candidates(k)
        assert len(c) >= 2
        assert all(len(x["tile"]) == 3 for x in c)


def test_create_rejects_bad_arguments_before_touching_the_gpu():
    """Argument checks run before any device call, so they work without a GPU."""
    _ensure_built()
    lib = vpp.load()
    d = _lib.Desc()
    d.ncells[:] = [2, 2, 2]
    d.extent[:] = [1, 1, 1]
    d.degree = 5
    d.rho_l, d.rho_g = 1.0, 1.0
    h = ctypes.c_void_p()
    assert lib.vpp_create(ctypes.byref(d), ctypes.byref(h)) == 1
    assert b"degree" in lib.vpp_last_error()
    d.degree = 2
    d.rho_g = -1.0
    assert lib.vpp_create(ctypes.byref(d), ctypes.byref(h)) == 1
    d.rho_g = 1.0
    d.ncells[1] = 0
    assert lib.vpp_create(ctypes.byref(d), ctypes.byref(h)) == 1
    d.ncells[1] = 2
    d.bc[2] = 7
    assert lib.vpp_create(ctypes.byref(d), ctypes.byref(h)) == 1
    assert lib.vpp_create(None, ctypes.byref(h)) == 1
    assert lib.vpp_num_dofs(None) == -1
    # the largest meshes: node indices are 32-bit (4 * 400 + 1 = 1601 nodes per
    # side is 4.1e9 nodes), refused on the host
    d.degree = 4
    d.bc[2] = 0
    d.ncells[:] = [400, 400, 400]
    assert lib.vpp_create(ctypes.byref(d), ctypes.byref(h)) == 1
    assert b"too large" in lib.vpp_last_error()
