"""Independent NumPy constructions used to pin the C oracle.

Nothing here calls the oracle.  Basis functions are numpy Polynomial objects
built from their roots, quadrature comes from numpy's Gauss-Legendre routine,
and 1D element integrals are exact polynomial integrals.  The dense global
matrix is a separate brute-force loop over cells, basis pairs and quadrature
points.
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial import Polynomial as Poly
from numpy.polynomial import legendre as npleg


def gll_closed_form(k: int) -> np.ndarray:
    """Gauss-Lobatto-Legendre points on [0,1]: ends plus roots of P_k' (numpy)."""
    c = np.zeros(k + 1)
    c[k] = 1.0
    inner = np.sort(npleg.legroots(npleg.legder(c)).real)
    return np.concatenate(([0.0], 0.5 * (inner + 1.0), [1.0]))


def gauss01(n: int):
    x, w = npleg.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def lagrange_polys(nodes):
    """Lagrange basis of the given nodes as numpy Polynomials."""
    out = []
    for a, xa in enumerate(nodes):
        others = [xb for b, xb in enumerate(nodes) if b != a]
        p = Poly.fromroots(others)
        out.append(p / p(xa))
    return out


def _lagrange_eval(nodes, a, x, deriv=False):
    """Lagrange polynomial a of `nodes` (or its derivative) at points x, by products."""
    x = np.asarray(x, dtype=np.float64)
    others = [b for b in range(len(nodes)) if b != a]
    if not deriv:
        return np.prod([(x - nodes[b]) / (nodes[a] - nodes[b]) for b in others], axis=0)
    tot = np.zeros_like(x)
    for m in others:
        term = np.full_like(x, 1.0 / (nodes[a] - nodes[m]))
        for b in others:
            if b != m:
                term = term * (x - nodes[b]) / (nodes[a] - nodes[b])
        tot += term
    return tot


def element_1d(k: int):
    """1D mass and stiffness matrices of the GLL Lagrange basis on [0,1], integrated
    exactly by numpy's Gauss-Legendre rule with k+2 points (degree 2k+3 >= 2k)."""
    nodes = gll_closed_form(k)
    x, w = gauss01(k + 2)
    n = k + 1
    V = np.array([_lagrange_eval(nodes, a, x) for a in range(n)])
    D = np.array([_lagrange_eval(nodes, a, x, deriv=True) for a in range(n)])
    M = (V * w) @ V.T
    K = (D * w) @ D.T
    return M, K


def global_1d(k: int, n: int, h: float):
    """Assembled 1D mass/stiffness on n uniform cells of size h."""
    Me, Ke = element_1d(k)
    N = k * n + 1
    M = np.zeros((N, N))
    K = np.zeros((N, N))
    for c in range(n):
        s = slice(k * c, k * c + k + 1)
        M[s, s] += Me * h
        K[s, s] += Ke / h
    return M, K


def dense_operator(mesh, coef_at, constrained=True, mass=0.0):
    """Brute-force dense matrix: sum over cells and Gauss points of c W grad N_a . grad N_b
    + mass W N_a N_b for every basis pair (a,b) of the cell (outer products of the
    gradient and value tables).

    coef_at(cell_index, q_tuple, x_q) -> coefficient value at that Gauss point."""
    k = mesh.degree
    n1 = k + 1
    nodes = gll_closed_form(k)
    L = lagrange_polys(nodes)
    dL = [p.deriv() for p in L]
    gx, gw = gauss01(n1)
    nx, ny, nz = mesh.ncells
    Nx, Ny, Nz = mesh.nnodes
    h = mesh.h
    A = np.zeros((mesh.ndofs, mesh.ndofs))
    for cz in range(nz):
        for cy in range(ny):
            for cx in range(nx):
                cell = cx + nx * (cy + ny * cz)
                loc = []
                for a2 in range(n1):
                    for a1 in range(n1):
                        for a0 in range(n1):
                            g = (k * cx + a0) + Nx * ((k * cy + a1) + Ny * (k * cz + a2))
                            loc.append((g, a0, a1, a2))
                for q2 in range(n1):
                    for q1 in range(n1):
                        for q0 in range(n1):
                            xq = (mesh.origin[0] + (cx + gx[q0]) * h[0],
                                  mesh.origin[1] + (cy + gx[q1]) * h[1],
                                  mesh.origin[2] + (cz + gx[q2]) * h[2])
                            W = gw[q0] * gw[q1] * gw[q2] * h[0] * h[1] * h[2]
                            c = coef_at(cell, (q0, q1, q2), xq)
                            grads = []
                            vals = np.array([L[a0](gx[q0]) * L[a1](gx[q1]) * L[a2](gx[q2])
                                             for (g, a0, a1, a2) in loc])
                            for (g, a0, a1, a2) in loc:
                                grads.append(np.array([
                                    dL[a0](gx[q0]) * L[a1](gx[q1]) * L[a2](gx[q2]) / h[0],
                                    L[a0](gx[q0]) * dL[a1](gx[q1]) * L[a2](gx[q2]) / h[1],
                                    L[a0](gx[q0]) * L[a1](gx[q1]) * dL[a2](gx[q2]) / h[2]]))
                            G = np.array(grads)                  # (k+1)^3 x 3
                            idx = np.array([g for (g, *_) in loc])
                            A[np.ix_(idx, idx)] += c * W * (G @ G.T) + mass * W * np.outer(vals, vals)
    if constrained:
        mask = mesh.boundary_mask()
        A[mask, :] = 0.0
        A[:, mask] = 0.0
        A[mask, mask] = 1.0
    return A


def fe_values_at(mesh, u, cell, xi):
    """Value of the FE function u at reference point xi (3-tuple) of a cell."""
    k = mesh.degree
    n1 = k + 1
    L = lagrange_polys(gll_closed_form(k))
    nx, ny, _ = mesh.ncells
    Nx, Ny, _ = mesh.nnodes
    cx, cy, cz = cell % nx, (cell // nx) % ny, cell // (nx * ny)
    s = 0.0
    for a2 in range(n1):
        for a1 in range(n1):
            for a0 in range(n1):
                g = (k * cx + a0) + Nx * ((k * cy + a1) + Ny * (k * cz + a2))
                s += L[a0](xi[0]) * L[a1](xi[1]) * L[a2](xi[2]) * u[g]
    return s


def heaviside_closed(phi, linear=True):
    """H written in phi without eps: linear (phi+1)/2, or the sine ramp in a = artanh(phi)."""
    phi = np.clip(np.asarray(phi, dtype=np.float64), -1.0, 1.0)
    if linear:
        return 0.5 * (phi + 1.0)
    out = np.where(phi > 0, 1.0, 0.0)
    inside = np.abs(phi) < math.tanh(1.5)
    a = np.arctanh(np.where(inside, phi, 0.0))
    val = 0.5 + a / 3.0 + np.sin(2.0 * math.pi * a / 3.0) / (2.0 * math.pi)
    return np.where(inside, val, out)
