"""Seeded synthetic inputs shared by the GPU library's callers and by the CPU oracle.

This module holds no part of the operator's arithmetic (no basis evaluation, no
quadrature, no coefficient law). It only places the lattice nodes, samples the
analytic level-set fields at them, and draws seeded random vectors, so that both
sides of a parity test receive bit-identical inputs.

Node placement: Q_k Lagrange elements on a uniform Cartesian box; inside each cell
the k+1 support points per direction are the Gauss-Lobatto-Legendre points of
[0,1] (for k=2 they are equidistant).  The paper only says "Lagrange
polynomials" (Sec. "Numerical framework"); the GLL choice is a reading.
Global numbering is lexicographic with x fastest: g = i + Nx*(j + Ny*l).

Level-set fields follow Eq. (initial_phi): phi = tanh(d / (2 eps)) for a signed
distance d that is positive in the liquid (phi > 0 liquid, Sec. "Level-set field").
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional, Sequence, Tuple

import numpy as np

# Closed forms of the GLL support points on [0,1] (reading of the node placement).
_GLL = {
    1: (0.0, 1.0),
    2: (0.0, 0.5, 1.0),
    3: (0.0, 0.5 - math.sqrt(5.0) / 10.0, 0.5 + math.sqrt(5.0) / 10.0, 1.0),
    4: (0.0, 0.5 - math.sqrt(21.0) / 14.0, 0.5, 0.5 + math.sqrt(21.0) / 14.0, 1.0),
}

BC_DIRICHLET = 0
BC_NEUMANN = 1
H_LINEAR = 0
H_PAPER = 1


def support_points(k: int) -> np.ndarray:
    """GLL support points of one cell on [0,1], ascending."""
    if k not in _GLL:
        raise ValueError(f"degree {k} not supported")
    return np.array(_GLL[k], dtype=np.float64)


@dataclass
class Mesh:
    """A uniform box of hexahedral cells carrying Q_k elements."""
    ncells: Tuple[int, int, int]
    degree: int
    origin: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    extent: Tuple[float, float, float] = (1.0, 1.0, 1.0)
    bc: Tuple[int, int, int, int, int, int] = (0, 0, 0, 0, 0, 0)   # x-,x+,y-,y+,z-,z+
    rho_l: float = 1000.0
    rho_g: float = 1.0
    heaviside: int = H_LINEAR
    eps: float = 0.0          # interface thickness; only the field generators use it
    mass: float = 0.0         # mass shift mu of the operator mu M + K_c (0: pressure operator)

    @property
    def nnodes(self) -> Tuple[int, int, int]:
        k = self.degree
        return tuple(k * n + 1 for n in self.ncells)

    @property
    def ndofs(self) -> int:
        nx, ny, nz = self.nnodes
        return nx * ny * nz

    @property
    def h(self) -> Tuple[float, float, float]:
        return tuple(e / n for e, n in zip(self.extent, self.ncells))

    def axis_coords(self, d: int) -> np.ndarray:
        """Coordinates of the node planes along direction d."""
        k = self.degree
        xi = support_points(k)
        n = self.ncells[d]
        h = self.extent[d] / n
        out = np.empty(k * n + 1)
        for c in range(n):
            out[k * c: k * c + k + 1] = self.origin[d] + (c + xi) * h
        out[-1] = self.origin[d] + self.extent[d]
        return out

    def node_grid(self):
        """(X, Y, Z) arrays of shape (Nz, Ny, Nx) so that ravel() is the global order."""
        x, y, z = (self.axis_coords(d) for d in range(3))
        Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
        return X, Y, Z

    def boundary_mask(self) -> np.ndarray:
        """True on nodes of Dirichlet faces (global order)."""
        Nx, Ny, Nz = self.nnodes
        m = np.zeros((Nz, Ny, Nx), dtype=bool)
        if self.bc[0] == BC_DIRICHLET: m[:, :, 0] = True
        if self.bc[1] == BC_DIRICHLET: m[:, :, -1] = True
        if self.bc[2] == BC_DIRICHLET: m[:, 0, :] = True
        if self.bc[3] == BC_DIRICHLET: m[:, -1, :] = True
        if self.bc[4] == BC_DIRICHLET: m[0, :, :] = True
        if self.bc[5] == BC_DIRICHLET: m[-1, :, :] = True
        return m.ravel()


# ----------------------------------------------------------------------------------
# Level-set fields (Eq. initial_phi), sampled at the lattice nodes.

def _tanh_profile(d: np.ndarray, eps: float) -> np.ndarray:
    return np.tanh(d / (2.0 * eps))


def droplet_phi(mesh: Mesh, radius: float, eps: float,
                centre: Sequence[float] = (0.5, 0.5, 0.5)) -> np.ndarray:
    """Liquid sphere: d = r - |x - c| (positive inside)."""
    X, Y, Z = mesh.node_grid()
    r = np.sqrt((X - centre[0]) ** 2 + (Y - centre[1]) ** 2 + (Z - centre[2]) ** 2)
    return _tanh_profile(radius - r, eps).ravel()


def bubble_phi(mesh: Mesh, radius: float, eps: float,
               centre: Sequence[float] = (0.5, 0.5, 0.5)) -> np.ndarray:
    """Gas sphere in liquid: the droplet field with the phases swapped."""
    return -droplet_phi(mesh, radius, eps, centre)


def spheres_phi(mesh: Mesh, centres: np.ndarray, radii: np.ndarray, eps: float) -> np.ndarray:
    """Union of liquid spheres: d = max_i (r_i - |x - c_i|)."""
    X, Y, Z = mesh.node_grid()
    d = np.full(X.shape, -np.inf)
    for c, r in zip(centres, radii):
        di = r - np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2)
        np.maximum(d, di, out=d)
    return _tanh_profile(d, eps).ravel()


def slab_phi(mesh: Mesh, x_interface: float, eps: float) -> np.ndarray:
    """Flat interface normal to x, liquid at x < x_interface."""
    X, _, _ = mesh.node_grid()
    return _tanh_profile(x_interface - X, eps).ravel()


def sine_field(mesh: Mesh) -> np.ndarray:
    """sin(pi x) sin(pi y) sin(pi z) at the nodes (manufactured pressure)."""
    X, Y, Z = mesh.node_grid()
    return (np.sin(np.pi * X) * np.sin(np.pi * Y) * np.sin(np.pi * Z)).ravel()


def normal_field(mesh: Mesh, centre=(0.5, 0.5, 0.5)) -> List[np.ndarray]:
    """The three components of the unit vector (c0 - x)/|x - c0| at the nodes
    (the interface normal of a droplet field centred at c0; 0 at the centre)."""
    X, Y, Z = mesh.node_grid()
    D = [X - centre[0], Y - centre[1], Z - centre[2]]
    r = np.sqrt(D[0] ** 2 + D[1] ** 2 + D[2] ** 2)
    inv = np.where(r > 0, 1.0 / np.where(r > 0, r, 1.0), 0.0)
    return [(-d * inv).ravel() for d in D]


def uniform_vectors(seed: int, count: int, n: int) -> np.ndarray:
    """`count` vectors with entries uniform in [-1,1] (rows of the returned array)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(count, n))


# ----------------------------------------------------------------------------------
# Workloads: the droplet / bubble / spheres setups of the paper's examples at the
# mesh sizes the measurements use.

@dataclass
class Workload:
    name: str
    mesh: Mesh
    phi: np.ndarray
    vectors: Optional[np.ndarray] = None
    note: str = ""
    extra: dict = field(default_factory=dict)


def unit_cube(n: int, k: int, rho_l: float, rho_g: float, **kw) -> Mesh:
    return Mesh(ncells=(n, n, n), degree=k, rho_l=rho_l, rho_g=rho_g, **kw)


def small_droplet(n: int = 8, k: int = 2, seed: int = 0, nvec: int = 1) -> Workload:
    """Droplet r=0.25 at the cube centre, eps=2h, rho 1000/1 (8^3 Q2 by default)."""
    m = unit_cube(n, k, 1000.0, 1.0)
    eps = 2.0 / n
    m.eps = eps
    phi = droplet_phi(m, 0.25, eps)
    vec = uniform_vectors(seed, nvec, m.ndofs)
    return Workload(f"droplet{n}^3-Q{k}", m, phi, vec)


def droplet_at_scale(k: int = 2, nvec: int = 100, seed: int = 1,
                     n: Optional[int] = None, bubble: bool = False) -> Workload:
    """About 2.15M DoFs: 64^3 Q2, 43^3 Q3 or 32^3 Q4; droplet (or bubble) r=0.25, eps=2h."""
    if n is None:
        n = {2: 64, 3: 43, 4: 32}[k]
    m = unit_cube(n, k, 1000.0, 1.0)
    eps = 2.0 / n
    m.eps = eps
    phi = (bubble_phi if bubble else droplet_phi)(m, 0.25, eps)
    vec = uniform_vectors(seed, nvec, m.ndofs) if nvec else None
    return Workload(f"{'bubble' if bubble else 'droplet'}{n}^3-Q{k}", m, phi, vec)


def spheres_mixed(n: int = 96, k: int = 3, seed: int = 2) -> Workload:
    """Union of 20 seeded spheres (centres drawn first, then radii), rho 7430/0.743, eps=1.5h."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.15, 0.85, size=(20, 3))
    radii = rng.uniform(0.05, 0.15, size=20)
    m = unit_cube(n, k, 7430.0, 0.743)
    eps = 1.5 / n
    m.eps = eps
    phi = spheres_phi(m, centres, radii, eps)
    return Workload(f"spheres{n}^3-Q{k}", m, phi, None,
                    extra={"centres": centres, "radii": radii})


BATCH_SIZES = (16, 24, 32, 40, 48, 56, 64, 64)


def batch_meshes(sizes: Sequence[int] = BATCH_SIZES, nrhs: int = 4, k: int = 2,
                 with_vectors: bool = True) -> List[Workload]:
    """Independent single-sphere meshes; mesh m draws radius, ratio, then its RHS from seed 300+m."""
    out = []
    for mi, n in enumerate(sizes):
        rng = np.random.default_rng(300 + mi)
        radius = float(rng.uniform(0.15, 0.35))
        ratio = float(rng.choice([100.0, 1000.0, 10000.0]))
        m = unit_cube(n, k, ratio, 1.0)
        eps = 2.0 / n
        m.eps = eps
        phi = droplet_phi(m, radius, eps)
        vec = rng.uniform(-1.0, 1.0, size=(nrhs, m.ndofs)) if with_vectors else None
        out.append(Workload(f"batch{mi}-{n}^3-Q{k}", m, phi, vec,
                            extra={"radius": radius, "ratio": ratio}))
    return out


def adjoint_case(n: int = 48, k: int = 2):
    """Droplet r=0.3 (forward) and r=0.28 (target), eps=2h, rho 1000/1."""
    m = unit_cube(n, k, 1000.0, 1.0)
    eps = 2.0 / n
    m.eps = eps
    return m, droplet_phi(m, 0.3, eps), droplet_phi(m, 0.28, eps)


def fd_nodes(mesh: Mesh, count: int = 32, seed: int = 4) -> np.ndarray:
    """`count` distinct seeded node indices that are not Dirichlet nodes."""
    rng = np.random.default_rng(seed)
    free = np.flatnonzero(~mesh.boundary_mask())
    return np.sort(rng.choice(free, size=count, replace=False))
