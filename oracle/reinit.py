"""Reinitialization step of the conservative level set (oracle).

TEST INFRASTRUCTURE ONLY, like the rest of this package.  It shares no code
with the HIP library.

One semi-implicit Euler step in pseudo-time of Eq. reinitialization, the
compressive flux explicit and the diffusion implicit (Sec. "Level-set field"):
  (psi^{k+1}, v)/dtau + eps ((grad psi^{k+1} . n)(grad v . n))
      = (psi^k, v)/dtau + ((1 - (psi^k)^2)/2 n, grad v),
with the boundary terms of both integrations by parts dropped (natural
conditions of the weak form), n the nodal (filtered) normal interpolated at
the Gauss points as it is (not renormalised), and the (k+1)^3 Gauss rule.  The
matrix is assembled cell by cell from the basis values and gradients at every
Gauss point, evaluated by the product formula of the 1D Lagrange polynomials.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .closest_point import _gll, _lagrange_1d


def _cell_tables(mesh):
    """Values (nq, nb) and physical gradients (3, nq, nb) of the cell basis at the
    Gauss points, Gauss weights W_q (nq,), local-to-global offsets (nb,)."""
    k = mesh.degree
    n1 = k + 1
    gx, gw = np.polynomial.legendre.leggauss(n1)
    gx, gw = (gx + 1.0) / 2.0, gw / 2.0
    V, D = _lagrange_1d(_gll(k), gx)          # (nq1, n1)
    h = mesh.h
    Nx, Ny, _ = mesh.nnodes
    nq, nb = n1 ** 3, n1 ** 3
    val = np.zeros((nq, nb))
    grad = np.zeros((3, nq, nb))
    W = np.zeros(nq)
    off = np.zeros(nb, dtype=np.int64)
    for a2 in range(n1):
        for a1 in range(n1):
            for a0 in range(n1):
                off[a0 + n1 * (a1 + n1 * a2)] = a0 + Nx * (a1 + Ny * a2)
    for q2 in range(n1):
        for q1 in range(n1):
            for q0 in range(n1):
                q = q0 + n1 * (q1 + n1 * q2)
                W[q] = gw[q0] * gw[q1] * gw[q2] * h[0] * h[1] * h[2]
                for a2 in range(n1):
                    for a1 in range(n1):
                        for a0 in range(n1):
                            a = a0 + n1 * (a1 + n1 * a2)
                            val[q, a] = V[q0, a0] * V[q1, a1] * V[q2, a2]
                            grad[0, q, a] = D[q0, a0] * V[q1, a1] * V[q2, a2] / h[0]
                            grad[1, q, a] = V[q0, a0] * D[q1, a1] * V[q2, a2] / h[1]
                            grad[2, q, a] = V[q0, a0] * V[q1, a1] * D[q2, a2] / h[2]
    return val, grad, W, off


def _cells(mesh):
    k = mesh.degree
    nx, ny, nz = mesh.ncells
    Nx, Ny, _ = mesh.nnodes
    for cz in range(nz):
        for cy in range(ny):
            for cx in range(nx):
                yield k * cx + Nx * (k * cy + Ny * k * cz)


def reinit_matrix(mesh, normal, eps: float, dtau: float):
    """CSR matrix of (u, v)/dtau + eps ((grad u . n)(grad v . n)) (no constraint)."""
    val, grad, W, off = _cell_tables(mesh)
    nq, nb = val.shape
    rows, cols, vals = [], [], []
    for base in _cells(mesh):
        g = base + off
        nqv = np.stack([val @ np.asarray(normal[d])[g] for d in range(3)])     # (3, nq)
        dn = np.einsum("dq,dqa->qa", nqv, grad)                                # grad N_a . n at q
        Ke = (val.T * (W / dtau)) @ val + eps * (dn.T * W) @ dn
        rows.append(np.repeat(g, nb))
        cols.append(np.tile(g, nb))
        vals.append(Ke.ravel())
    n = mesh.ndofs
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))


def reinit_rhs(mesh, psi, normal, dtau: float) -> np.ndarray:
    """(psi, v)/dtau + ((1 - psi_h^2)/2 n, grad v)."""
    val, grad, W, off = _cell_tables(mesh)
    psi = np.asarray(psi, dtype=np.float64)
    b = np.zeros(mesh.ndofs)
    for base in _cells(mesh):
        g = base + off
        pq = val @ psi[g]
        nqv = np.stack([val @ np.asarray(normal[d])[g] for d in range(3)])
        flux = 0.5 * (1.0 - pq * pq) * nqv                                     # (3, nq)
        be = val.T @ (W * pq / dtau) + np.einsum("dqa,dq->a", grad, flux * W)
        np.add.at(b, g, be)
    return b


def _cells_around(mesh, g):
    """Base nodes of the (at most 8) cells containing node g."""
    k = mesh.degree
    Nx, Ny, _ = mesh.nnodes
    idx = (g % Nx, (g // Nx) % Ny, g // (Nx * Ny))
    ranges = []
    for d in range(3):
        i = idx[d]
        lo = i // k - 1 if i % k == 0 else i // k
        hi = i // k
        ranges.append(range(max(lo, 0), min(hi, mesh.ncells[d] - 1) + 1))
    for cz in ranges[2]:
        for cy in ranges[1]:
            for cx in ranges[0]:
                yield k * cx + Nx * (k * cy + Ny * k * cz)


def reinit_rows(mesh, normal, eps: float, dtau: float, x, psi, rows):
    """Rows `rows` of A x, of diag(A) and of the right-hand side of the step (the
    same cell integrals as reinit_matrix / reinit_rhs, summed over the cells
    around each row's node only).  Returns (Ax, diag, b), each of len(rows)."""
    val, grad, W, off = _cell_tables(mesh)
    x = np.asarray(x, dtype=np.float64)
    psi = np.asarray(psi, dtype=np.float64)
    ax, dg, rb = (np.zeros(len(rows)) for _ in range(3))
    for r, g in enumerate(np.asarray(rows, dtype=np.int64)):
        for base in _cells_around(mesh, int(g)):
            gl = base + off
            a = int(np.nonzero(gl == g)[0][0])
            nqv = np.stack([val @ np.asarray(normal[d])[gl] for d in range(3)])
            dn = np.einsum("dq,dqa->qa", nqv, grad)
            Ke_row = (val[:, a] * (W / dtau)) @ val + eps * (dn[:, a] * W) @ dn
            ax[r] += Ke_row @ x[gl]
            dg[r] += Ke_row[a]
            pq = val @ psi[gl]
            flux = 0.5 * (1.0 - pq * pq) * nqv
            rb[r] += val[:, a] @ (W * pq / dtau) + np.einsum("dq,dq->", grad[:, :, a], flux * W)
    return ax, dg, rb
