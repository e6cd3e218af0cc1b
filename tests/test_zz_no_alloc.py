"""vpp_apply_noalloc (shared-face partials in the library's static device
array, no allocation) against vpp_apply on the same problem: two calls in a
row, the second on a smaller mesh, so the second reads an array the first
filled; 1e-12 relative (2-norm and max-norm) like every FP64 apply.  Each
output vector starts as NaN, so every entry must be written.  Sizes whose
partials do not fit the static array, and bad arguments, are refused before
any launch."""
import ctypes as C

import numpy as np
import pytest
import torch

import workloads as W
from gpu_util import dev, host, rel, rel_max, say

pytestmark = pytest.mark.gpu

vpp = pytest.importorskip("paper_2401_07805_amd")
from paper_2401_07805_amd import _lib as L  # noqa: E402


def _desc(m, law=None):
    d = L.Desc()
    d.ncells[:] = list(m.ncells)
    d.origin[:] = list(m.origin)
    d.extent[:] = list(m.extent)
    d.degree = m.degree
    d.bc[:] = list(m.bc)
    d.rho_l, d.rho_g = m.rho_l, m.rho_g
    d.heaviside = m.heaviside if law is None else law
    d.device = 0
    return d


def _noalloc(d, phi, x):
    y = torch.full_like(x, float("nan"))
    st = L.load().vpp_apply_noalloc(C.byref(d), C.c_void_p(phi.data_ptr()), C.c_void_p(x.data_ptr()),
                                    C.c_void_p(y.data_ptr()),
                                    C.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, y


@pytest.mark.parametrize("k,sizes,law", [(2, ((24, 20, 16), (7, 9, 5)), None), (3, ((14, 11, 12), (4, 3, 5)), None),
                                         (4, ((9, 8, 10), (3, 2, 4)), None), (2, ((17, 12, 9), (5, 6, 3)), 2)])
def test_noalloc_matches_apply_twice(k, sizes, law):
    for n in sizes:
        m = W.Mesh(ncells=n, degree=k, bc=(0, 1, 1, 0, 0, 1), rho_l=1000.0, rho_g=1.0,
                   heaviside=W.H_PAPER if k == 3 else W.H_LINEAR)
        m.eps = 2.0 / max(n)
        phi = dev(W.droplet_phi(m, 0.3, m.eps, centre=(0.45, 0.5, 0.55)))
        x = dev(W.uniform_vectors(5 + k, 1, m.ndofs)[0])
        d = _desc(m, law)
        prob = vpp.Problem(m.ncells, k, m.origin, m.extent, m.bc, m.rho_l, m.rho_g, d.heaviside)
        prob.set_phi(phi)
        yref = host(prob.apply(x))
        say("noalloc", k, n, law)
        st, y = _noalloc(d, phi, x)
        assert st == 0, L.load().vpp_last_error()
        y = host(y)
        assert np.isfinite(y).all()
        assert rel(y, yref) < 1e-12 and rel_max(y, yref) < 1e-12, (rel(y, yref), rel_max(y, yref))


def test_noalloc_refuses_before_launch():
    lib = L.load()
    m = W.unit_cube(4, 2, 1000.0, 1.0)
    x = dev(np.ones(m.ndofs + 1))
    y = torch.zeros_like(x)
    phi = dev(np.zeros(m.ndofs + 1))
    d = _desc(m)
    P = lambda t, off=0: C.c_void_p(t.data_ptr() + off)
    say("noalloc refusals")
    assert lib.vpp_apply_noalloc(None, P(phi), P(x), P(y), None) == 1
    assert lib.vpp_apply_noalloc(C.byref(d), P(phi), P(x, 4), P(y), None) == 1
    assert lib.vpp_apply_noalloc(C.byref(d), P(phi), P(x), P(x), None) == 1
    bad = _desc(m)
    bad.degree = 5
    assert lib.vpp_apply_noalloc(C.byref(bad), P(phi), P(x), P(y), None) == 1
    big = _desc(W.unit_cube(96, 3, 1000.0, 1.0))      # 24.1M DoFs: partials beyond the static array
    assert lib.vpp_apply_noalloc(C.byref(big), P(phi), P(x), P(y), None) == 2
    assert b"static scratch" in lib.vpp_last_error()
    torch.cuda.synchronize()
    assert float(y.abs().max()) == 0.0                  # nothing was launched
