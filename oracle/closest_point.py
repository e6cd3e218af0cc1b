"""Closest-point projection onto the zero isosurface of the FE level set.

TEST INFRASTRUCTURE ONLY, like the rest of this package: only the tests, the
smoke check and the benchmark's CPU-baseline leg may use it.  It shares no code
with the HIP library.

Follows the appendix "Extension of solution quantities from a level-set
isosurface using closest point projection" (Eq. cpp).  For a point x (a
support point in the narrow band |phi| < phi_lim), y^(0) = x and every outer
step k takes
  (i)  `normal_steps` corrections along the normal, y <- y - d(y) n(y), with the
       signed distance d = eps log((1 + phi_h)/(1 - phi_h)) of Eq. distance and
       n = grad phi_h / |grad phi_h|, and
  (ii) one tangential correction y <- y - sum_j ((y - x) . t_j) t_j with the
       unit tangents t_0 = (v - (v.n) n) / |v - (v.n) n| and t_1 = n x t_0, all
       evaluated at the y that step (ii) starts from; v = e_x, or e_y when
       |n_x| > 0.9 (e_x nearly parallel to n),
until |y^(k+1) - y^(k)| < tol, at most max_iter outer steps.  phi_h and its
gradient at an arbitrary point come from the Q_k Lagrange basis on the GLL
support points of the cell holding the point (product formula).  Readings
where the appendix is silent: y is clipped to the domain box after every
correction; phi_h is clipped to +-(1 - 1e-12) inside the logarithm; a step
whose normal vanishes leaves y unchanged.

The normal n_Gamma of Eq. cpp is the filtered interface normal of Eq.
normal_vector_regularized.  With a nodal normal field given (`normal`, three
arrays), n(y) = n_h(y)/|n_h(y)| with n_h its Q_k interpolant; without it n is
the normalised gradient of phi_h (the unfiltered normal of Eq. normal_vector).
"""
from __future__ import annotations

import numpy as np

_PHI_CLIP = 1.0 - 1e-12


def _gll(k: int) -> np.ndarray:
    """GLL support points of [0,1]: the end points and the roots of P_k'."""
    inner = np.polynomial.legendre.Legendre.basis(k).deriv().roots()
    return np.concatenate(([0.0], np.sort((inner.real + 1.0) / 2.0), [1.0]))


def _lagrange_1d(nodes: np.ndarray, t: np.ndarray):
    """Values and derivatives of the Lagrange polynomials on `nodes` at t: (P, n) each."""
    n = len(nodes)
    V = np.ones((len(t), n))
    D = np.zeros((len(t), n))
    for a in range(n):
        for b in range(n):
            if b == a:
                continue
            V[:, a] *= (t - nodes[b]) / (nodes[a] - nodes[b])
        for m in range(n):
            if m == a:
                continue
            term = np.full(len(t), 1.0 / (nodes[a] - nodes[m]))
            for b in range(n):
                if b != a and b != m:
                    term *= (t - nodes[b]) / (nodes[a] - nodes[b])
            D[:, a] += term
    return V, D


def evaluate(mesh, phi: np.ndarray, pts: np.ndarray):
    """phi_h and grad phi_h at points pts (P, 3) inside the box."""
    k = mesh.degree
    nodes = _gll(k)
    origin = np.asarray(mesh.origin, dtype=np.float64)
    h = np.asarray(mesh.h, dtype=np.float64)
    nc = np.asarray(mesh.ncells)
    Nx, Ny, _ = mesh.nnodes
    s = (pts - origin) / h
    cell = np.clip(np.floor(s), 0, nc - 1).astype(np.int64)
    xi = s - cell
    V, D = [], []
    for d in range(3):
        v, dv = _lagrange_1d(nodes, xi[:, d])
        V.append(v)
        D.append(dv / h[d])
    val = np.zeros(len(pts))
    grad = np.zeros((len(pts), 3))
    for a2 in range(k + 1):
        for a1 in range(k + 1):
            for a0 in range(k + 1):
                g = (k * cell[:, 0] + a0) + Nx * ((k * cell[:, 1] + a1) + Ny * (k * cell[:, 2] + a2))
                f = phi[g]
                val += V[0][:, a0] * V[1][:, a1] * V[2][:, a2] * f
                grad[:, 0] += D[0][:, a0] * V[1][:, a1] * V[2][:, a2] * f
                grad[:, 1] += V[0][:, a0] * D[1][:, a1] * V[2][:, a2] * f
                grad[:, 2] += V[0][:, a0] * V[1][:, a1] * D[2][:, a2] * f
    return val, grad


def _unit_normal(mesh, phi, normal, y):
    """phi_h(y), the unit normal at y (P, 3) and where it is defined (P,)."""
    val, grad = evaluate(mesh, phi, y)
    if normal is not None:
        grad = np.stack([evaluate(mesh, normal[d], y)[0] for d in range(3)], axis=1)
    gn = np.linalg.norm(grad, axis=1)
    ok = gn > 0
    n = np.where(ok[:, None], grad / np.where(ok, gn, 1.0)[:, None], 0.0)
    return val, n, ok


def closest_points(mesh, phi, pts, eps: float, max_iter: int = 20, normal_steps: int = 3,
                   tol: float = 1e-12, normal=None):
    """Closest points y (P, 3) of pts on {phi_h = 0}, the outer steps taken (P,)
    and whether |y^(k+1) - y^(k)| < tol was reached (P,).  normal: None (the
    gradient of phi_h) or three nodal fields of the filtered normal."""
    phi = np.asarray(phi, dtype=np.float64)
    if normal is not None:
        normal = [np.asarray(c, dtype=np.float64) for c in normal]
    x = np.array(pts, dtype=np.float64).reshape(-1, 3)
    lo = np.asarray(mesh.origin, dtype=np.float64)
    hi = lo + np.asarray(mesh.extent, dtype=np.float64)
    y = x.copy()
    steps = np.zeros(len(x), dtype=np.int64)
    done = np.zeros(len(x), dtype=bool)
    for _ in range(max_iter):
        act = ~done
        if not act.any():
            break
        ya = y[act]
        prev = ya.copy()
        for _ in range(normal_steps):
            val, n, ok = _unit_normal(mesh, phi, normal, ya)
            pc = np.clip(val, -_PHI_CLIP, _PHI_CLIP)
            dist = eps * np.log((1.0 + pc) / (1.0 - pc))
            ya = np.clip(ya - np.where(ok, dist, 0.0)[:, None] * n, lo, hi)
        _, n, ok = _unit_normal(mesh, phi, normal, ya)
        v = np.zeros_like(n)
        use_y = np.abs(n[:, 0]) > 0.9
        v[~use_y, 0] = 1.0
        v[use_y, 1] = 1.0
        t0 = v - np.sum(v * n, axis=1)[:, None] * n
        t0 /= np.linalg.norm(t0, axis=1)[:, None]
        t1 = np.cross(n, t0)
        r = ya - x[act]
        corr = np.sum(r * t0, axis=1)[:, None] * t0 + np.sum(r * t1, axis=1)[:, None] * t1
        ya = np.clip(np.where(ok[:, None], ya - corr, ya), lo, hi)
        y[act] = ya
        steps[act] += 1
        conv = np.linalg.norm(ya - prev, axis=1) < tol
        idx = np.flatnonzero(act)
        done[idx[conv]] = True
    return y, steps, done


def band_nodes(mesh, phi, phi_lim: float) -> np.ndarray:
    """Indices of the support points with |phi| < phi_lim (the narrow band), ascending."""
    return np.flatnonzero(np.abs(np.asarray(phi)) < phi_lim)


def node_coords(mesh, idx: np.ndarray) -> np.ndarray:
    """Coordinates (P, 3) of global nodes idx."""
    x, y, z = (mesh.axis_coords(d) for d in range(3))
    Nx, Ny, _ = mesh.nnodes
    i = idx % Nx
    j = (idx // Nx) % Ny
    l = idx // (Nx * Ny)
    return np.stack([x[i], y[j], z[l]], axis=1)
