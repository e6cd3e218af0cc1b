"""FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It wraps the plain C oracle in ``oracle.c`` (full-quadrature
assembly, CSR SpMV, Jacobi PCG, adjoint gradient) through ctypes and adds the
analytic right-hand sides used by the pins.  It shares no code with the HIP
library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc + OpenMP into liboracle.so (in-tree)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-D_GNU_SOURCE", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


class _Desc(C.Structure):
    _fields_ = [("ncells", C.c_int32 * 3), ("origin", C.c_double * 3),
                ("extent", C.c_double * 3), ("degree", C.c_int32), ("bc", C.c_int32 * 6),
                ("rho_l", C.c_double), ("rho_g", C.c_double), ("heaviside", C.c_int32),
                ("eps", C.c_double), ("mass", C.c_double)]


_lib = None
_D = C.POINTER(C.c_double)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build()
    L = C.CDLL(_SO)
    P = C.POINTER(_Desc)
    vp = C.c_void_p
    sig = {
        "orc_gll_points": (None, [C.c_int, _D]),
        "orc_gauss_rule": (None, [C.c_int, _D, _D]),
        "orc_lagrange": (C.c_double, [C.c_int, _D, C.c_int, C.c_double]),
        "orc_lagrange_deriv": (C.c_double, [C.c_int, _D, C.c_int, C.c_double]),
        "orc_heaviside": (C.c_double, [P, C.c_double]),
        "orc_heaviside_deriv": (C.c_double, [P, C.c_double]),
        "orc_coefficient": (C.c_double, [P, C.c_double]),
        "orc_num_dofs": (C.c_int64, [P]),
        "orc_num_qpoints": (C.c_int64, [P]),
        "orc_coef_qp": (None, [P, _D, _D]),
        "orc_assemble": (vp, [P, _D, C.c_int]),
        "orc_assemble_cq": (vp, [P, _D, C.c_int]),
        "orc_free": (None, [vp]),
        "orc_rows": (C.c_int64, [vp]),
        "orc_nnz": (C.c_int64, [vp]),
        "orc_export": (None, [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64), _D]),
        "orc_spmv": (None, [vp, _D, _D]),
        "orc_diag": (None, [vp, _D]),
        "orc_pcg": (C.c_int, [vp, _D, _D, C.c_double, C.c_double, C.c_int,
                              C.POINTER(C.c_int), _D]),
        "orc_rhs_qp": (None, [P, _D, _D]),
        "orc_rhs_flux": (None, [P, _D, _D, _D, _D]),
        "orc_qp_coords": (None, [P, C.c_int, _D, _D, _D, _D]),
        "orc_eval_qp": (None, [P, C.c_int, _D, _D]),
        "orc_grad_coef": (None, [P, _D, _D, _D]),
        "orc_grad_phi": (None, [P, _D, _D, _D]),
        "orc_num_threads": (C.c_int, []),
        "orc_set_num_threads": (None, [C.c_int]),
        "orc_apply_rows": (None, [P, _D, _D, C.POINTER(C.c_int64), C.c_int64, _D]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def desc_of(mesh) -> _Desc:
    """Oracle descriptor from a ``workloads.Mesh``."""
    d = _Desc()
    d.ncells[:] = list(mesh.ncells)
    d.origin[:] = list(mesh.origin)
    d.extent[:] = list(mesh.extent)
    d.degree = mesh.degree
    d.bc[:] = list(mesh.bc)
    d.rho_l = mesh.rho_l
    d.rho_g = mesh.rho_g
    d.heaviside = mesh.heaviside
    d.eps = mesh.eps if mesh.eps > 0 else 1.0
    d.mass = float(getattr(mesh, "mass", 0.0))
    return d


def num_threads() -> int:
    return _load().orc_num_threads()


def set_num_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on (n > 0)."""
    _load().orc_set_num_threads(int(n))


# -- 1D tables ----------------------------------------------------------------

def gll_points(k: int) -> np.ndarray:
    out = np.zeros(k + 1)
    _load().orc_gll_points(k, _ptr(out))
    return out


def gauss_rule(n: int):
    x, w = np.zeros(n), np.zeros(n)
    _load().orc_gauss_rule(n, _ptr(x), _ptr(w))
    return x, w


def lagrange(k: int, nodes, a: int, x: float, deriv: bool = False) -> float:
    nd = _f64(nodes)
    f = _load().orc_lagrange_deriv if deriv else _load().orc_lagrange
    return f(k, _ptr(nd), a, float(x))


# -- coefficient law ----------------------------------------------------------

def heaviside(mesh, phi: float, deriv: bool = False) -> float:
    d = desc_of(mesh)
    f = _load().orc_heaviside_deriv if deriv else _load().orc_heaviside
    return f(C.byref(d), float(phi))


def coefficient(mesh, phi: float) -> float:
    d = desc_of(mesh)
    return _load().orc_coefficient(C.byref(d), float(phi))


def coef_qp(mesh, phi) -> np.ndarray:
    d = desc_of(mesh)
    out = np.zeros(_load().orc_num_qpoints(C.byref(d)))
    _load().orc_coef_qp(C.byref(d), _ptr(_f64(phi)), _ptr(out))
    return out


def coef_qp_arith(mesh, phi, paper: bool = False) -> np.ndarray:
    """The arithmetic density mean App. D contrasts with Eq. rhoEff, at every
    Gauss point (cell-major, like coef_qp): phi_h(x_q) interpolated from the
    nodal phi, clamped to [-1, 1] (reading R3), H linear (phi+1)/2 or the sine
    ramp of Eq. heaviside (paper=True), rho = H rho_l + (1 - H) rho_g, c = 1/rho."""
    ph = np.clip(eval_qp(mesh, phi), -1.0, 1.0)
    if paper:
        d = desc_of(mesh)
        d.heaviside = 1
        H = np.array([_load().orc_heaviside(C.byref(d), float(v)) for v in ph])
    else:
        H = 0.5 * (ph + 1.0)
    return 1.0 / (H * mesh.rho_l + (1.0 - H) * mesh.rho_g)


# -- assembled operator -------------------------------------------------------

class Operator:
    """Assembled FP64 CSR matrix of the pressure-Poisson operator."""

    def __init__(self, mesh, phi=None, cq=None, constrained: bool = True):
        L = _load()
        self.mesh = mesh
        self._d = desc_of(mesh)
        if cq is not None:
            self._h = L.orc_assemble_cq(C.byref(self._d), _ptr(_f64(cq)), int(constrained))
        else:
            self._h = L.orc_assemble(C.byref(self._d), _ptr(_f64(phi)), int(constrained))
        self.n = L.orc_rows(self._h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_free(h)
            self._h = None

    @property
    def nnz(self) -> int:
        return _load().orc_nnz(self._h)

    def matvec(self, x) -> np.ndarray:
        x = _f64(x)
        y = np.zeros(self.n)
        _load().orc_spmv(self._h, _ptr(x), _ptr(y))
        return y

    def diagonal(self) -> np.ndarray:
        d = np.zeros(self.n)
        _load().orc_diag(self._h, _ptr(d))
        return d

    def to_scipy(self):
        import scipy.sparse as sp
        nnz = self.nnz
        rp = np.zeros(self.n + 1, dtype=np.int64)
        col = np.zeros(nnz, dtype=np.int64)
        val = np.zeros(nnz)
        _load().orc_export(self._h, rp.ctypes.data_as(C.POINTER(C.c_int64)),
                           col.ctypes.data_as(C.POINTER(C.c_int64)), _ptr(val))
        return sp.csr_matrix((val, col, rp), shape=(self.n, self.n))

    def pcg(self, b, x0=None, rtol=1e-10, atol=0.0, max_iter=100000):
        b = _f64(b)
        x = np.zeros(self.n) if x0 is None else _f64(x0).copy()
        it = C.c_int(0)
        rr = C.c_double(0.0)
        st = _load().orc_pcg(self._h, _ptr(b), _ptr(x), rtol, atol, max_iter,
                             C.byref(it), C.byref(rr))
        return x, {"status": st, "iterations": it.value, "rel_residual": rr.value}


# -- load vectors / evaluation / adjoint -------------------------------------

def rhs_qp(mesh, fq) -> np.ndarray:
    d = desc_of(mesh)
    b = np.zeros(mesh.ndofs)
    _load().orc_rhs_qp(C.byref(d), _ptr(_f64(fq)), _ptr(b))
    return b


def rhs_flux(mesh, fx, fy, fz) -> np.ndarray:
    d = desc_of(mesh)
    b = np.zeros(mesh.ndofs)
    _load().orc_rhs_flux(C.byref(d), _ptr(_f64(fx)), _ptr(_f64(fy)), _ptr(_f64(fz)), _ptr(b))
    return b


def qp_coords(mesh, nq: Optional[int] = None):
    """(x, y, z, w) of the nq-point Gauss rule in every cell (default nq = k+1)."""
    nq = mesh.degree + 1 if nq is None else nq
    d = desc_of(mesh)
    n = int(np.prod(mesh.ncells)) * nq ** 3
    x, y, z, w = (np.zeros(n) for _ in range(4))
    _load().orc_qp_coords(C.byref(d), nq, _ptr(x), _ptr(y), _ptr(z), _ptr(w))
    return x, y, z, w


def eval_qp(mesh, u, nq: Optional[int] = None) -> np.ndarray:
    nq = mesh.degree + 1 if nq is None else nq
    d = desc_of(mesh)
    out = np.zeros(int(np.prod(mesh.ncells)) * nq ** 3)
    _load().orc_eval_qp(C.byref(d), nq, _ptr(_f64(u)), _ptr(out))
    return out


def apply_rows(mesh, phi, x, rows) -> np.ndarray:
    """Rows `rows` of y = A_D x, assembled cell by cell around each node."""
    d = desc_of(mesh)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.zeros(rows.size)
    _load().orc_apply_rows(C.byref(d), _ptr(_f64(phi)), _ptr(_f64(x)),
                           rows.ctypes.data_as(C.POINTER(C.c_int64)), rows.size, _ptr(out))
    return out


def grad_coef(mesh, p, lam) -> np.ndarray:
    d = desc_of(mesh)
    out = np.zeros(_load().orc_num_qpoints(C.byref(d)))
    _load().orc_grad_coef(C.byref(d), _ptr(_f64(p)), _ptr(_f64(lam)), _ptr(out))
    return out


def grad_phi(mesh, phi, gq) -> np.ndarray:
    d = desc_of(mesh)
    out = np.zeros(mesh.ndofs)
    _load().orc_grad_phi(C.byref(d), _ptr(_f64(phi)), _ptr(_f64(gq)), _ptr(out))
    return out


# -- right-hand sides for the pins and the solves -----------------------------

def constrain_rhs(op_full, mesh, ell, g_bnd=None) -> np.ndarray:
    """Symmetric elimination of Dirichlet values: b_D = g_D, b_I = ell_I - A_ID g_D.

    ``op_full`` is the unconstrained operator (``Operator(..., constrained=False)``)."""
    mask = mesh.boundary_mask()
    g = np.zeros(mesh.ndofs) if g_bnd is None else np.where(mask, g_bnd, 0.0)
    b = ell - op_full.matvec(g)
    b[mask] = g[mask]
    return b


def manufactured_sine_rhs(mesh, radius: float, eps: float, centre=(0.5, 0.5, 0.5),
                          sign: float = 1.0) -> np.ndarray:
    """Load vector of f = -div(c grad p*) for p* = sin(pi x) sin(pi y) sin(pi z).

    c is the analytic coefficient of the droplet field phi = tanh(sign*(r-|x-c0|)/(2 eps))
    (sign=-1: bubble), so f = 3 pi^2 c p* - grad c . grad p*, with
    grad c = (1/rho_l - 1/rho_g) H'(phi) grad phi and grad phi = (1-phi^2)/(2 eps) grad d.
    Homogeneous Dirichlet values (p* vanishes on the cube faces)."""
    x, y, z, _ = qp_coords(mesh)
    dx, dy, dz = x - centre[0], y - centre[1], z - centre[2]
    r = np.sqrt(dx * dx + dy * dy + dz * dz)
    rs = np.where(r > 0, r, 1.0)
    d = sign * (radius - r)
    phi = np.tanh(d / (2 * eps))
    Hd = np.array([heaviside(mesh, v, deriv=True) for v in phi]) if mesh.heaviside else 0.5
    dcdphi = (1.0 / mesh.rho_l - 1.0 / mesh.rho_g) * Hd
    Hv = np.array([heaviside(mesh, v) for v in phi]) if mesh.heaviside else 0.5 * (phi + 1)
    c = Hv / mesh.rho_l + (1 - Hv) / mesh.rho_g
    dphi = (1 - phi * phi) / (2 * eps) * sign
    gd = np.where(r > 0, -1.0, 0.0)
    gx, gy, gz = gd * dx / rs * dphi * dcdphi, gd * dy / rs * dphi * dcdphi, gd * dz / rs * dphi * dcdphi
    pi = np.pi
    s = np.sin(pi * x) * np.sin(pi * y) * np.sin(pi * z)
    px = pi * np.cos(pi * x) * np.sin(pi * y) * np.sin(pi * z)
    py = pi * np.sin(pi * x) * np.cos(pi * y) * np.sin(pi * z)
    pz = pi * np.sin(pi * x) * np.sin(pi * y) * np.cos(pi * z)
    f = 3 * pi * pi * c * s - (gx * px + gy * py + gz * pz)
    b = rhs_qp(mesh, f)
    b[mesh.boundary_mask()] = 0.0
    return b


def manufactured_sine_rhs_spheres(mesh, centres, radii, eps: float) -> np.ndarray:
    """Load vector of f = -div(c grad p*) for p* = sin(pi x) sin(pi y) sin(pi z) on a
    union of liquid spheres: d = max_i (r_i - |x - c_i|) with ties to the lowest
    i, phi = tanh(d/(2 eps)), and grad d = -(x - c_i)/|x - c_i| of the sphere
    that attains the maximum; c is the analytic coefficient of Eq. rhoEff for
    that phi, so f = 3 pi^2 c p* - grad c . grad p* as for one sphere.
    Homogeneous Dirichlet values (p* vanishes on the cube faces)."""
    x, y, z, _ = qp_coords(mesh)
    centres = np.asarray(centres, dtype=np.float64)
    radii = np.asarray(radii, dtype=np.float64)
    dist = np.stack([r - np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
                     for c, r in zip(centres, radii)])
    owner = np.argmax(dist, axis=0)                   # first maximum: lowest sphere index
    d = dist[owner, np.arange(x.size)]
    cx, cy, cz = centres[owner, 0], centres[owner, 1], centres[owner, 2]
    dx, dy, dz = x - cx, y - cy, z - cz
    r = np.sqrt(dx * dx + dy * dy + dz * dz)
    rs = np.where(r > 0, r, 1.0)
    phi = np.tanh(d / (2 * eps))
    Hd = np.array([heaviside(mesh, v, deriv=True) for v in phi]) if mesh.heaviside else 0.5
    Hv = np.array([heaviside(mesh, v) for v in phi]) if mesh.heaviside else 0.5 * (phi + 1)
    dcdphi = (1.0 / mesh.rho_l - 1.0 / mesh.rho_g) * Hd
    c = Hv / mesh.rho_l + (1 - Hv) / mesh.rho_g
    dphi = (1 - phi * phi) / (2 * eps)
    gd = np.where(r > 0, -1.0, 0.0)
    gx, gy, gz = (gd * dd / rs * dphi * dcdphi for dd in (dx, dy, dz))
    pi = np.pi
    s = np.sin(pi * x) * np.sin(pi * y) * np.sin(pi * z)
    px = pi * np.cos(pi * x) * np.sin(pi * y) * np.sin(pi * z)
    py = pi * np.sin(pi * x) * np.cos(pi * y) * np.sin(pi * z)
    pz = pi * np.sin(pi * x) * np.sin(pi * y) * np.cos(pi * z)
    f = 3 * pi * pi * c * s - (gx * px + gy * py + gz * pz)
    b = rhs_qp(mesh, f)
    b[mesh.boundary_mask()] = 0.0
    return b


def sine_load(mesh) -> np.ndarray:
    """Load vector of f0 = 3 pi^2 sin sin sin (phi-independent), zero on Dirichlet rows."""
    x, y, z, _ = qp_coords(mesh)
    f = 3 * np.pi ** 2 * np.sin(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z)
    b = rhs_qp(mesh, f)
    b[mesh.boundary_mask()] = 0.0
    return b


def discrete_manufactured_rhs(op, mesh, p_nodal) -> np.ndarray:
    """b = A_D p* for a nodal p* with zero Dirichlet values (exact discrete solution p*)."""
    p = np.array(p_nodal, dtype=np.float64)
    p[mesh.boundary_mask()] = 0.0
    return op.matvec(p)


from .closest_point import band_nodes, closest_points, node_coords  # noqa: E402  (closest-point projection)
from .reinit import reinit_matrix, reinit_rhs, reinit_rows  # noqa: E402  (reinitialization step)
