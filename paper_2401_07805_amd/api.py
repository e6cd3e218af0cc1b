"""Python face of the C ABI: problems, batches and the autograd Function.

Torch provides device memory and streams only; every step of the operator,
solver and adjoint runs in the HIP library.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import torch

from . import _lib as L


class VppError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{L.STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_PREC = {"fp64": L.VPP_FP64, "fp32": L.VPP_FP32}
# Largest number of Ritz vectors of the first FP32 phase that mixed-precision
# solves deflate (0: none; only isolated small Ritz values are used)
DEFLATE = 4


def _check(status: int):
    if status != L.VPP_OK:
        raise VppError(status, L.load().vpp_last_error().decode())


def _stream(device: torch.device) -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _vec(t: torch.Tensor, n: int, dtype: torch.dtype, device: torch.device, name: str) -> C.c_void_p:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device != device:
        raise ValueError(f"{name} must be on {device}, got {t.device}")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if t.numel() != n or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous vector of {n} entries")
    return C.c_void_p(t.data_ptr())


def _info(ci: L.CgInfo) -> dict:
    return {"iterations": ci.iterations, "outer_iterations": ci.outer_iterations, "status": ci.status,
            "status_name": L.STATUS_NAMES.get(ci.status, str(ci.status)),
            "rel_residual": ci.rel_residual, "true_rel_residual": ci.true_rel_residual,
            "deflation_corrections": ci.deflation_corrections, "deflation_first_change": ci.deflation_first_change}


class Problem:
    """One mesh + degree + material law on one GPU (vpp_create)."""

    def __init__(self, ncells: Sequence[int], degree: int, origin=(0.0, 0.0, 0.0), extent=(1.0, 1.0, 1.0),
                 bc=(0, 0, 0, 0, 0, 0), rho_l: float = 1000.0, rho_g: float = 1.0, heaviside: int = 0,
                 device: int = 0):
        lib = L.load()
        d = L.Desc()
        d.ncells[:] = [int(v) for v in ncells]
        d.origin[:] = [float(v) for v in origin]
        d.extent[:] = [float(v) for v in extent]
        d.degree = int(degree)
        d.bc[:] = [int(v) for v in bc]
        d.rho_l = float(rho_l)
        d.rho_g = float(rho_g)
        d.heaviside = int(heaviside)
        d.device = int(device)
        self._h = C.c_void_p()
        _check(lib.vpp_create(C.byref(d), C.byref(self._h)))
        self.device = torch.device("cuda", int(device))
        self.degree = int(degree)
        self.ncells = tuple(int(v) for v in ncells)
        self.n = lib.vpp_num_dofs(self._h)
        self.nq = lib.vpp_num_qpoints(self._h)
        self.last_grad_coef: Optional[torch.Tensor] = None
        self._phi_version = 0

    @classmethod
    def from_mesh(cls, mesh, device: int = 0) -> "Problem":
        """From any object with ncells, degree, origin, extent, bc, rho_l, rho_g, heaviside."""
        return cls(mesh.ncells, mesh.degree, mesh.origin, mesh.extent, mesh.bc, mesh.rho_l, mesh.rho_g,
                   mesh.heaviside, device)

    def close(self):
        h = getattr(self, "_h", None)
        if h and h.value and L._lib is not None:
            L._lib.vpp_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self) -> C.c_void_p:
        return self._h

    def set_phi(self, phi: torch.Tensor):
        _check(L.load().vpp_set_phi(self._h, _vec(phi, self.n, torch.float64, self.device, "phi"),
                                    _stream(self.device)))
        self._phi_version += 1

    def closest_points(self, eps: float, pts: Optional[torch.Tensor] = None, phi_lim: float = 0.9,
                       tol: float = 1e-11, max_iter: int = 50, normal_steps: int = 3,
                       normal: Optional[Sequence[torch.Tensor]] = None):
        """Closest points on {phi_h = 0} (vpp_closest_points).  pts: (P, 3) float64
        on the device, or None for the narrow band |phi| < phi_lim of the mesh
        nodes.  normal: three nodal fields (the filtered normal) to take the
        normal from (vpp_closest_points_normal), or None for the gradient of
        phi_h.  Returns (y (P, 3), info (P,) int32: outer steps to convergence,
        0 not converged, -1 outside the band)."""
        o = L.CpOpts(float(eps), float(phi_lim), float(tol), int(max_iter), int(normal_steps))
        if normal is not None:
            if len(normal) != 3:
                raise ValueError("normal must hold three nodal fields")
            nptr = [_vec(c, self.n, torch.float64, self.device, "normal") for c in normal]
        if pts is None:
            n, ptr = self.n, None
        else:
            if pts.dtype != torch.float64 or pts.device != self.device or pts.dim() != 2 or pts.shape[1] != 3:
                raise ValueError("pts must be a (P, 3) float64 tensor on the problem's device")
            pts = pts.contiguous()
            n, ptr = pts.shape[0], C.c_void_p(pts.data_ptr())
            if n == 0:
                return (torch.empty((0, 3), dtype=torch.float64, device=self.device),
                        torch.empty(0, dtype=torch.int32, device=self.device))
        y = torch.empty((n, 3), dtype=torch.float64, device=self.device)
        info = torch.empty(n, dtype=torch.int32, device=self.device)
        if normal is None:
            _check(L.load().vpp_closest_points(self._h, ptr, n, C.byref(o), C.c_void_p(y.data_ptr()),
                                               C.c_void_p(info.data_ptr()), _stream(self.device)))
        else:
            _check(L.load().vpp_closest_points_normal(self._h, ptr, n, *nptr, C.byref(o),
                                                      C.c_void_p(y.data_ptr()), C.c_void_p(info.data_ptr()),
                                                      _stream(self.device)))
        return y, info

    def extend(self, y: torch.Tensor, info: torch.Tensor, f: torch.Tensor) -> torch.Tensor:
        """f extended from the closest points (vpp_extend): f_h(y_g) on the band, f elsewhere."""
        if y.shape != (self.n, 3) or info.shape != (self.n,) or info.dtype != torch.int32:
            raise ValueError("y, info must be the node-mode output of closest_points")
        out = torch.empty_like(f)
        _check(L.load().vpp_extend(self._h, C.c_void_p(y.contiguous().data_ptr()),
                                   C.c_void_p(info.contiguous().data_ptr()),
                                   _vec(f, self.n, torch.float64, self.device, "f"),
                                   _vec(out, self.n, torch.float64, self.device, "out"), _stream(self.device)))
        return out

    def normal_rhs(self, phi: torch.Tensor):
        """(n_bar_d, v) for d = x, y, z with n_bar = grad phi_h / |grad phi_h| (vpp_normal_rhs)."""
        bs = [torch.empty(self.n, dtype=torch.float64, device=self.device) for _ in range(3)]
        _check(L.load().vpp_normal_rhs(self._h, _vec(phi, self.n, torch.float64, self.device, "phi"),
                                       *[_vec(b, self.n, torch.float64, self.device, "b") for b in bs],
                                       _stream(self.device)))
        return bs

    def curvature_rhs(self, n0: torch.Tensor, n1: torch.Tensor, n2: torch.Tensor) -> torch.Tensor:
        """(-div n_h, v) for the nodal normal components (vpp_curvature_rhs)."""
        b = torch.empty(self.n, dtype=torch.float64, device=self.device)
        _check(L.load().vpp_curvature_rhs(self._h, *[_vec(v, self.n, torch.float64, self.device, "n")
                                                     for v in (n0, n1, n2)],
                                          _vec(b, self.n, torch.float64, self.device, "b"), _stream(self.device)))
        return b

    def reinit_step(self, psi: torch.Tensor, normal, eps: float, dtau: float, rtol: float = 1e-12,
                    atol: float = 1e-20, max_iter: int = 100000, raise_on_failure: bool = True):
        """One semi-implicit reinitialization step (vpp_reinit_step); normal: the three
        nodal components.  Returns (psi', info)."""
        out = torch.empty_like(psi)
        o = L.ReinitOpts(float(eps), float(dtau), float(rtol), float(atol), int(max_iter))
        ci = L.CgInfo()
        st = L.load().vpp_reinit_step(self._h, _vec(psi, self.n, torch.float64, self.device, "psi"),
                                      *[_vec(c, self.n, torch.float64, self.device, "normal") for c in normal],
                                      C.byref(o), _vec(out, self.n, torch.float64, self.device, "psi_out"),
                                      C.byref(ci), _stream(self.device))
        if st != L.VPP_OK and (raise_on_failure or st not in (5, 6)):
            _check(st)
        return out, _info(ci)

    def _reinit_opts(self, eps: float, dtau: float):
        return L.ReinitOpts(float(eps), float(dtau), 0.0, 0.0, 0)

    def reinit_apply(self, x: torch.Tensor, normal, eps: float, dtau: float) -> torch.Tensor:
        """y = (M/dtau + eps K_n) x, the reinitialization step's operator (vpp_reinit_apply)."""
        y = torch.empty_like(x)
        o = self._reinit_opts(eps, dtau)
        _check(L.load().vpp_reinit_apply(self._h, *[_vec(c, self.n, torch.float64, self.device, "normal")
                                                    for c in normal], C.byref(o),
                                         _vec(x, self.n, torch.float64, self.device, "x"),
                                         _vec(y, self.n, torch.float64, self.device, "y"), _stream(self.device)))
        return y

    def reinit_diagonal(self, normal, eps: float, dtau: float) -> torch.Tensor:
        """diag(M/dtau + eps K_n) (vpp_reinit_diagonal)."""
        d = torch.empty(self.n, dtype=torch.float64, device=self.device)
        o = self._reinit_opts(eps, dtau)
        _check(L.load().vpp_reinit_diagonal(self._h, *[_vec(c, self.n, torch.float64, self.device, "normal")
                                                       for c in normal], C.byref(o),
                                            _vec(d, self.n, torch.float64, self.device, "diag"),
                                            _stream(self.device)))
        return d

    def reinit_rhs(self, psi: torch.Tensor, normal, eps: float, dtau: float) -> torch.Tensor:
        """(psi, v)/dtau + ((1 - psi_h^2)/2 n, grad v) (vpp_reinit_rhs)."""
        b = torch.empty(self.n, dtype=torch.float64, device=self.device)
        o = self._reinit_opts(eps, dtau)
        _check(L.load().vpp_reinit_rhs(self._h, _vec(psi, self.n, torch.float64, self.device, "psi"),
                                       *[_vec(c, self.n, torch.float64, self.device, "normal") for c in normal],
                                       C.byref(o), _vec(b, self.n, torch.float64, self.device, "b"),
                                       _stream(self.device)))
        return b

    def set_mass(self, mu: float):
        """Operator mu M + K_c (vpp_set_mass); mu = 0 is the pressure operator."""
        _check(L.load().vpp_set_mass(self._h, float(mu), _stream(self.device)))

    def apply(self, x: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        prec = L.VPP_FP64 if x.dtype == torch.float64 else L.VPP_FP32
        if x.dtype not in (torch.float64, torch.float32):
            raise ValueError("x must be float64 or float32")
        y = torch.empty_like(x) if out is None else out
        _check(L.load().vpp_apply(self._h, prec, _vec(x, self.n, x.dtype, self.device, "x"),
                                  _vec(y, self.n, x.dtype, self.device, "y"), _stream(self.device)))
        return y

    def diagonal(self) -> torch.Tensor:
        d = torch.empty(self.n, dtype=torch.float64, device=self.device)
        _check(L.load().vpp_diagonal(self._h, _vec(d, self.n, torch.float64, self.device, "diag"),
                                     _stream(self.device)))
        return d

    def cg_solve(self, b: torch.Tensor, x0: Optional[torch.Tensor] = None, rtol: float = 1e-8,
                 atol: float = 0.0, max_iter: int = 100000, precision: str = "fp64",
                 inner_rtol: float = 1e-2, inner_max_iter: int = 0, check_every: int = 0,
                 raise_on_failure: bool = True, deflate: int = DEFLATE, deflate_history: int = 0):
        """Jacobi PCG; precision "mixed" runs FP32 recurrences with FP64
        residual replacements, and with deflate > 0 a Galerkin correction in the
        span of that many Ritz vectors of the first FP32 phase at every
        replacement (vpp_cg_opts)."""
        x = torch.zeros_like(b) if x0 is None else x0.clone()
        o = L.CgOpts(rtol, atol, int(max_iter), L.VPP_MIXED if precision == "mixed" else L.VPP_FP64,
                     inner_rtol, int(inner_max_iter), int(check_every), int(deflate), int(deflate_history))
        ci = L.CgInfo()
        st = L.load().vpp_cg_solve(self._h, _vec(b, self.n, torch.float64, self.device, "b"),
                                   _vec(x, self.n, torch.float64, self.device, "x"), C.byref(o),
                                   C.byref(ci), _stream(self.device))
        if st != L.VPP_OK and (raise_on_failure or st not in (5, 6)):
            _check(st)
        return x, _info(ci)

    def grad_coef(self, p: torch.Tensor, lam: torch.Tensor) -> torch.Tensor:
        g = torch.empty(self.nq, dtype=torch.float64, device=self.device)
        _check(L.load().vpp_grad_coef(self._h, _vec(p, self.n, torch.float64, self.device, "p"),
                                      _vec(lam, self.n, torch.float64, self.device, "lam"),
                                      _vec(g, self.nq, torch.float64, self.device, "g_q"),
                                      _stream(self.device)))
        return g

    def grad_phi(self, g_q: torch.Tensor) -> torch.Tensor:
        out = torch.empty(self.n, dtype=torch.float64, device=self.device)
        _check(L.load().vpp_grad_phi(self._h, _vec(g_q, self.nq, torch.float64, self.device, "g_q"),
                                     _vec(out, self.n, torch.float64, self.device, "g_phi"),
                                     _stream(self.device)))
        return out

    @property
    def config(self) -> dict:
        """Kernel configuration of the FP64 apply."""
        return self.config_for("fp64")

    def config_for(self, precision: str) -> dict:
        c = L.KernelConfig()
        _check(L.load().vpp_get_config_for(self._h, _PREC[precision], C.byref(c)))
        return {"variant": c.variant, "tile": tuple(c.tile)}

    def set_config(self, variant: int, tile: Sequence[int], precision: Optional[str] = None):
        """Sets the kernel configuration of one precision ("fp64", "fp32") or of both (None)."""
        c = L.KernelConfig()
        c.variant = int(variant)
        c.tile[:] = [int(v) for v in tile]
        if precision is None:
            _check(L.load().vpp_set_config(self._h, C.byref(c)))
        else:
            _check(L.load().vpp_set_config_for(self._h, _PREC[precision], C.byref(c)))

    def tune(self, cache_path: Optional[str] = None) -> dict:
        """Autotunes both precisions; returns the FP64 choice."""
        _check(L.load().vpp_tune(self._h, cache_path.encode() if cache_path else None, _stream(self.device)))
        return self.config


def config_candidates(degree: int) -> list:
    lib = L.load()
    n = lib.vpp_config_candidates(int(degree), None, 0)
    arr = (L.KernelConfig * max(n, 1))()
    lib.vpp_config_candidates(int(degree), arr, n)
    return [{"variant": arr[i].variant, "tile": tuple(arr[i].tile)} for i in range(n)]


class Batch:
    """Independent problems applied together by one persistent graph launch."""

    def __init__(self, problems: Sequence[Problem], nrhs: Sequence[int], tune_cache: Optional[str] = None):
        lib = L.load()
        self.problems = list(problems)
        self.nrhs = [int(v) for v in nrhs]
        hs = (C.c_void_p * len(problems))(*[p.handle.value for p in problems])
        nr = (C.c_int32 * len(problems))(*self.nrhs)
        self._h = C.c_void_p()
        _check(lib.vpp_batch_create(hs, nr, len(problems), tune_cache.encode() if tune_cache else None,
                                    C.byref(self._h)))
        self.device = problems[0].device

    def close(self):
        h = getattr(self, "_h", None)
        if h and h.value and L._lib is not None:
            L._lib.vpp_batch_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _tables(self, xs, ys):
        ptr_x, ptr_y = [], []
        i = 0
        for p, nr in zip(self.problems, self.nrhs):
            for _ in range(nr):
                ptr_x.append(_vec(xs[i], p.n, torch.float64, self.device, "x").value)
                ptr_y.append(_vec(ys[i], p.n, torch.float64, self.device, "y").value)
                i += 1
        if i != len(xs) or i != len(ys):
            raise ValueError("one vector per (problem, rhs) pair expected")
        tx = (C.c_void_p * i)(*ptr_x)
        ty = (C.c_void_p * i)(*ptr_y)
        return tx, ty

    def apply(self, xs: Sequence[torch.Tensor], ys: Sequence[torch.Tensor]):
        tx, ty = self._tables(xs, ys)
        _check(L.load().vpp_batch_apply(self._h, tx, ty, _stream(self.device)))

    def cg_solve(self, bs, xs, rtol=1e-8, atol=0.0, max_iter=100000, precision="fp64", inner_rtol=1e-2,
                 check_every=0, raise_on_failure=True, deflate=DEFLATE):
        """Solve A_i x = b for every (problem, rhs) pair; xs hold the initial
        guesses and receive the solutions.  Returns one info dict per pair."""
        tb, tx = self._tables(bs, xs)
        n = len(bs)
        o = L.CgOpts(rtol, atol, int(max_iter), L.VPP_MIXED if precision == "mixed" else L.VPP_FP64,
                     inner_rtol, 0, int(check_every), int(deflate), 0)
        infos = (L.CgInfo * n)()
        st = L.load().vpp_batch_cg_solve(self._h, tb, tx, C.byref(o), infos, _stream(self.device))
        if st != L.VPP_OK and (raise_on_failure or st not in (5, 6)):
            _check(st)
        return [_info(infos[i]) for i in range(n)]

    @property
    def config(self) -> dict:
        c = L.KernelConfig()
        _check(L.load().vpp_batch_get_config(self._h, C.byref(c)))
        return {"variant": c.variant, "tile": tuple(c.tile)}


class AmrProblem:
    """A box whose marked coarse cells are refined once, with hanging-node
    constraints (vpp_amr_create).  Vectors hold the coarse lattice and then the
    fine lattice (num_dofs entries)."""

    def __init__(self, ncells: Sequence[int], degree: int, refined, origin=(0.0, 0.0, 0.0),
                 extent=(1.0, 1.0, 1.0), bc=(0, 0, 0, 0, 0, 0), rho_l: float = 1000.0, rho_g: float = 1.0,
                 heaviside: int = 0, device: int = 0):
        import numpy as np
        lib = L.load()
        d = L.Desc()
        d.ncells[:] = [int(v) for v in ncells]
        d.origin[:] = [float(v) for v in origin]
        d.extent[:] = [float(v) for v in extent]
        d.degree = int(degree)
        d.bc[:] = [int(v) for v in bc]
        d.rho_l = float(rho_l)
        d.rho_g = float(rho_g)
        d.heaviside = int(heaviside)
        d.device = int(device)
        mask = np.ascontiguousarray(np.asarray(refined, dtype=np.uint8).ravel())
        if mask.size != int(np.prod(ncells)):
            raise ValueError("refined must hold one entry per coarse cell")
        self._h = C.c_void_p()
        _check(lib.vpp_amr_create(C.byref(d), mask.ctypes.data_as(C.c_void_p), C.byref(self._h)))
        self.device = torch.device("cuda", int(device))
        self.n = lib.vpp_amr_num_dofs(self._h)
        self.nfree = lib.vpp_amr_num_free(self._h)

    def close(self):
        h = getattr(self, "_h", None)
        if h and h.value and L._lib is not None:
            L._lib.vpp_amr_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_phi(self, phi: torch.Tensor):
        _check(L.load().vpp_amr_set_phi(self._h, _vec(phi, self.n, torch.float64, self.device, "phi"),
                                        _stream(self.device)))

    def apply(self, x: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        y = torch.empty_like(x) if out is None else out
        _check(L.load().vpp_amr_apply(self._h, _vec(x, self.n, torch.float64, self.device, "x"),
                                      _vec(y, self.n, torch.float64, self.device, "y"), _stream(self.device)))
        return y

    def diagonal(self) -> torch.Tensor:
        d = torch.empty(self.n, dtype=torch.float64, device=self.device)
        _check(L.load().vpp_amr_diagonal(self._h, _vec(d, self.n, torch.float64, self.device, "diag"),
                                         _stream(self.device)))
        return d

    def cg_solve(self, b: torch.Tensor, x0: Optional[torch.Tensor] = None, rtol: float = 1e-8, atol: float = 0.0,
                 max_iter: int = 100000, check_every: int = 0, raise_on_failure: bool = True):
        x = torch.zeros_like(b) if x0 is None else x0.clone()
        o = L.CgOpts(rtol, atol, int(max_iter), L.VPP_FP64, 0.0, 0, int(check_every))
        ci = L.CgInfo()
        st = L.load().vpp_amr_cg_solve(self._h, _vec(b, self.n, torch.float64, self.device, "b"),
                                       _vec(x, self.n, torch.float64, self.device, "x"), C.byref(o), C.byref(ci),
                                       _stream(self.device))
        if st != L.VPP_OK and (raise_on_failure or st not in (5, 6)):
            _check(st)
        return x, _info(ci)


class PoissonSolve(torch.autograd.Function):
    """p = A_D(phi)^{-1} b with a hand-written adjoint.

    backward: lam = A_D^{-1} dJ/dp (A_D symmetric), dJ/dc_q from vpp_grad_coef (kept
    on problem.last_grad_coef), dJ/dphi from vpp_grad_phi, dJ/db = lam."""

    @staticmethod
    def forward(ctx, phi: torch.Tensor, b: torch.Tensor, problem: Problem, opts: Optional[dict] = None):
        opts = dict(opts or {})
        problem.set_phi(phi.detach())
        p, info = problem.cg_solve(b.detach(), **opts)
        ctx.problem = problem
        ctx.opts = opts
        ctx.version = problem._phi_version
        ctx.save_for_backward(phi.detach(), p)
        return p

    @staticmethod
    def backward(ctx, gp: torch.Tensor):
        phi, p = ctx.saved_tensors
        problem: Problem = ctx.problem
        if problem._phi_version != ctx.version:
            problem.set_phi(phi)
            ctx.version = problem._phi_version
        lam, _ = problem.cg_solve(gp.contiguous().to(torch.float64), **ctx.opts)
        g_q = problem.grad_coef(p, lam)
        problem.last_grad_coef = g_q
        g_phi = problem.grad_phi(g_q)
        return g_phi, lam, None, None


def poisson_solve(phi: torch.Tensor, b: torch.Tensor, problem: Problem, **opts) -> torch.Tensor:
    return PoissonSolve.apply(phi, b, problem, opts)
