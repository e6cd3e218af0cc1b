"""The bounds-checked library (libvpp_debug.so: the same sources with every
global and LDS access of the apply tile kernels and of the shared-node
assembly checked against its buffer, see vpp_debug_bounds_violations) runs
every instantiated configuration on ragged meshes, in FP64 and FP32, with
and without the x . Ax partials (inside CG), with the mass shift, the
arithmetic density mean, the batched apply (Q2 and Q3) and the allocation-free apply:
no access falls outside its buffer, and every configuration gives the same
result.  The release library reports -1 (no checks compiled in).

The debug library is loaded in a child process (the library choice is made
once per process, and this process holds the release library)."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

vpp = pytest.importorskip("paper_2401_07805_amd")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import ctypes as C
import json, sys
import numpy as np
import torch
sys.path.insert(0, ROOT)
import workloads as W
import paper_2401_07805_amd as vpp
from paper_2401_07805_amd import _lib as L

lib = L.load()
assert L.LIB_PATH.endswith("libvpp_debug.so"), L.LIB_PATH
dev = torch.device("cuda", 0)
out = {"cases": 0, "violations": 0, "max_rel": 0.0}

def check(tag):
    v = int(lib.vpp_debug_bounds_violations())
    print(tag, "violations", v, flush=True)
    assert v >= 0, v
    out["violations"] += v

def rel(a, b):
    return float(torch.linalg.norm(a - b) / max(float(torch.linalg.norm(b)), 1e-300))

MESHES = {2: [(13, 7, 5), (9, 10, 3)], 3: [(7, 5, 3), (5, 6, 2)], 4: [(5, 3, 3), (3, 4, 2)]}
for k, shapes in MESHES.items():
    for shape in shapes:
        for law, ratio in ((0, 1000.0), (1, 100.0)):
            m = W.Mesh(ncells=shape, degree=k, bc=(0, 1, 0, 0, 1, 0), rho_l=ratio, rho_g=1.0, heaviside=law)
            m.eps = 0.1
            phi = torch.from_numpy(W.droplet_phi(m, 0.3, 0.08, centre=(0.45, 0.52, 0.5))).to(dev)
            x = torch.from_numpy(W.uniform_vectors(7, 1, m.ndofs)[0]).to(dev)
            p = vpp.Problem.from_mesh(m)
            p.set_phi(phi)
            ref64 = ref32 = None
            for cfg in vpp.config_candidates(k):
                p.set_config(cfg["variant"], cfg["tile"])
                y = p.apply(x)
                y32 = p.apply(x.float())
                torch.cuda.synchronize()
                check(f"k={k} {shape} law {law} {cfg}")
                if ref64 is None:
                    ref64, ref32 = y, y32
                ry = rel(y, ref64)
                if ry > 1e-13:
                    print("config", cfg, "rel", ry, flush=True)
                out["max_rel"] = max(out["max_rel"], ry)
                assert rel(y32.double(), ref32.double()) < 1e-5
                out["cases"] += 1
            # the x . Ax instantiations (inside CG), both precisions
            b = p.apply(x)
            p.cg_solve(b, rtol=1e-6, max_iter=20, raise_on_failure=False)
            p.cg_solve(b, rtol=1e-6, max_iter=20, precision="mixed", raise_on_failure=False)
            check(f"k={k} {shape} law {law} cg")
            # mass shift (its own instantiations)
            p.set_mass(1.0)
            p.apply(x)
            p.cg_solve(b, rtol=1e-6, max_iter=20, raise_on_failure=False)
            check(f"k={k} {shape} law {law} mass")
        # arithmetic density mean
        m = W.Mesh(ncells=shape, degree=k, bc=(0, 1, 0, 0, 1, 0), rho_l=1000.0, rho_g=1.0)
        q = vpp.Problem(m.ncells, k, m.origin, m.extent, m.bc, m.rho_l, m.rho_g, 2)
        phq = torch.from_numpy(W.droplet_phi(m, 0.3, 0.08)).to(dev)
        q.set_phi(phq)
        xq = torch.from_numpy(W.uniform_vectors(8, 1, m.ndofs)[0]).to(dev)
        q.apply(xq)
        check(f"k={k} {shape} arithmetic")
        # the allocation-free apply (its fixed configuration, static partials)
        d = L.Desc()
        d.ncells[:] = list(m.ncells)
        d.origin[:] = list(m.origin)
        d.extent[:] = list(m.extent)
        d.degree = k
        d.bc[:] = list(m.bc)
        d.rho_l, d.rho_g, d.heaviside, d.device = m.rho_l, m.rho_g, 0, 0
        pz = vpp.Problem.from_mesh(m)
        pz.set_phi(phq)
        yz = torch.empty_like(xq)
        st = lib.vpp_apply_noalloc(C.byref(d), C.c_void_p(phq.data_ptr()), C.c_void_p(xq.data_ptr()),
                                   C.c_void_p(yz.data_ptr()), C.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert st == 0, st
        torch.cuda.synchronize()
        rz = rel(yz, pz.apply(xq))
        out["max_rel"] = max(out["max_rel"], rz)
        check(f"k={k} {shape} noalloc rel {rz:.1e}")
# batched apply (k = 2 and 3) over two ragged meshes, two right-hand sides each
for k, shapes in ((2, ((13, 7, 5), (6, 9, 4))), (3, ((9, 5, 3), (4, 6, 5)))):
    probs, xs, ys = [], [], []
    for shape in shapes:
        m = W.Mesh(ncells=shape, degree=k, bc=(0,) * 6, rho_l=1000.0, rho_g=1.0)
        pr = vpp.Problem.from_mesh(m)
        pr.set_phi(torch.from_numpy(W.droplet_phi(m, 0.3, 0.08)).to(dev))
        probs.append(pr)
        for r in range(2):
            xs.append(torch.from_numpy(W.uniform_vectors(9 + r, 1, m.ndofs)[0]).to(dev))
            ys.append(torch.empty_like(xs[-1]))
    bt = vpp.Batch(probs, [2, 2])
    bt.apply(xs, ys)
    torch.cuda.synchronize()
    check(f"batch k={k} {bt.config}")
    i = 0
    for pr in probs:
        for r in range(2):
            rb = rel(ys[i], pr.apply(xs[i]))
            print("batch k", k, "rhs", i, "rel", rb, flush=True)
            out["max_rel"] = max(out["max_rel"], rb)
            i += 1
print("RESULT", json.dumps(out), flush=True)
"""


def test_release_library_reports_no_checks():
    from paper_2401_07805_amd import _lib as L
    assert L.load().vpp_debug_bounds_violations() == -1


def test_bounds_checked_kernels_stay_in_bounds():
    lib = os.path.join(ROOT, "paper_2401_07805_amd", "libvpp_debug.so")
    assert os.path.exists(lib), "build() links libvpp_debug.so beside libvpp.so"
    env = dict(os.environ, VPP_DEBUG_BOUNDS="1")
    proc = subprocess.run([sys.executable, "-u", "-c", "ROOT = %r\n" % ROOT + CHILD], env=env,
                          capture_output=True, text=True, timeout=600)
    print(proc.stdout[-6000:], proc.stderr[-4000:])
    assert proc.returncode == 0, proc.stderr[-4000:]
    res = json.loads(proc.stdout.split("RESULT", 1)[1])
    assert res["cases"] > 0
    assert res["violations"] == 0
    assert res["max_rel"] < 1e-13
