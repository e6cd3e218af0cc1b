"""Pressure operator on a once-refined hexahedral mesh with hanging nodes
(oracle).

TEST INFRASTRUCTURE ONLY, like the rest of this package.  It shares no code
with the HIP library.

The mesh: a uniform box of coarse cells, a chosen set of which is refined once
(each split into 2 x 2 x 2 cells), the adaptive refinement of Sec. "Numerical
framework" restricted to one level.  Where a refined cell meets an unrefined
one (a face, or only an edge or a vertex), the fine cells' nodes on the
unrefined cell's boundary are not unknowns: continuity of the Q_k space makes
them the coarse cell's Q_k interpolant there (hanging nodes; where a fine node
coincides with a coarse node, a copy).

Unknowns live on two lattices, held in one vector: the coarse lattice
(k n_d + 1 nodes per direction) first, then the fine lattice over the whole
box (2 k n_d + 1 per direction).  Free unknowns are the coarse nodes of
unrefined cells and the fine nodes of refined cells that lie on no unrefined
cell.  The operator is the plain definition
    A = C^T A_cells C,
A_cells the sum over the active cells (unrefined coarse cells on the coarse
lattice, fine cells of refined cells on the fine lattice) of their element
matrices K_e[a,b] = sum_q c_q W_q grad N_a . grad N_b by full quadrature
((k+1)^3 Gauss points, basis gradients by the product formula), C the
constraint matrix (identity on free unknowns, interpolation weights on
constrained fine nodes, zero elsewhere).  Every entry that is not a free
unknown, and every free unknown on a Dirichlet face, gets an identity row and
column, as A_D does on the uniform mesh.  The coefficient of a cell comes from
the nodal phi of its own lattice (Eq. rhoEff, clamp of reading R3).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import gauss_rule, gll_points, heaviside, lagrange


def lattices(mesh):
    """(coarse node counts, fine node counts, Nc, Nf)."""
    k = mesh.degree
    nc = [k * n + 1 for n in mesh.ncells]
    nf = [2 * k * n + 1 for n in mesh.ncells]
    return nc, nf, int(np.prod(nc)), int(np.prod(nf))


def num_dofs(mesh) -> int:
    _, _, Nc, Nf = lattices(mesh)
    return Nc + Nf


def _tables(k):
    """1D values V[q][a] and derivatives D[q][a] of the GLL Lagrange basis at the
    (k+1)-point Gauss points, and the Gauss weights, all on [0, 1]."""
    nodes = gll_points(k)
    gx, gw = gauss_rule(k + 1)
    V = np.array([[lagrange(k, nodes, a, x) for a in range(k + 1)] for x in gx])
    D = np.array([[lagrange(k, nodes, a, x, deriv=True) for a in range(k + 1)] for x in gx])
    return nodes, gx, gw, V, D


def _reference_basis(k, h):
    """Values (nq, nb) and physical gradients (3, nq, nb) of the cell basis at the
    Gauss points of a cell with edge lengths h, and the weights W_q (nq,),
    by the product formula; local index a0 + (k+1)(a1 + (k+1) a2)."""
    _, _, gw, V, D = _tables(k)
    n1 = k + 1
    nq = nb = n1 ** 3
    val = np.zeros((nq, nb))
    grad = np.zeros((3, nq, nb))
    W = np.zeros(nq)
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
    return val, grad, W


def _cell_nodes(k, n_nodes, cell):
    """Lattice indices of the (k+1)^3 nodes of lattice cell (cx, cy, cz)."""
    n1 = k + 1
    cx, cy, cz = cell
    a = np.arange(n1)
    i = k * cx + a[None, None, :]
    j = k * cy + a[None, :, None]
    l = k * cz + a[:, None, None]
    return (i + n_nodes[0] * (j + n_nodes[1] * l)).ravel()


def _coefficient(mesh, phq):
    """c of Eq. rhoEff at interpolated level-set values (clamped to [-1, 1])."""
    ph = np.clip(phq, -1.0, 1.0)
    if mesh.heaviside:
        H = np.array([heaviside(mesh, v) for v in ph])
    else:
        H = 0.5 * (ph + 1.0)
    return H / mesh.rho_l + (1.0 - H) / mesh.rho_g


def classify(mesh, refined):
    """Node sets of the two-lattice vector.

    refined: coarse-cell mask (cx fastest).  Returns a dict of boolean masks
    over the N = Nc + Nf entries ('free', 'constrained', 'dirichlet') and the
    constraint matrix C (N x N, CSR)."""
    k = mesh.degree
    ncel = list(mesh.ncells)
    refined = np.asarray(refined, dtype=bool).reshape(ncel[2], ncel[1], ncel[0])
    ncn, nfn, Nc, Nf = lattices(mesh)
    N = Nc + Nf
    # coarse nodes of unrefined cells
    c_active = np.zeros(Nc, dtype=bool)
    for cz in range(ncel[2]):
        for cy in range(ncel[1]):
            for cx in range(ncel[0]):
                if not refined[cz, cy, cx]:
                    c_active[_cell_nodes(k, ncn, (cx, cy, cz))] = True
    # fine nodes of refined cells
    f_in = np.zeros(Nf, dtype=bool)
    for fz in range(2 * ncel[2]):
        for fy in range(2 * ncel[1]):
            for fx in range(2 * ncel[0]):
                if refined[fz // 2, fy // 2, fx // 2]:
                    f_in[_cell_nodes(k, nfn, (fx, fy, fz))] = True
    nodes = gll_points(k)
    free = np.zeros(N, dtype=bool)
    free[:Nc] = c_active
    constrained = np.zeros(N, dtype=bool)
    rows, cols, vals = [], [], []
    for g in np.flatnonzero(c_active):
        rows.append(g), cols.append(g), vals.append(1.0)
    two_k = 2 * k
    for gf in np.flatnonzero(f_in):
        I = gf % nfn[0]
        J = (gf // nfn[0]) % nfn[1]
        L = gf // (nfn[0] * nfn[1])
        # unrefined coarse cells whose closure holds the node, lowest index first
        rng = []
        for v, n in zip((I, J, L), ncel):
            c = v // two_k
            rng.append([c - 1, c] if v % two_k == 0 else [c])
        owner = None
        for cz in rng[2]:
            for cy in rng[1]:
                for cx in rng[0]:
                    if owner is None and 0 <= cx < ncel[0] and 0 <= cy < ncel[1] and 0 <= cz < ncel[2] \
                            and not refined[cz, cy, cx]:
                        owner = (cx, cy, cz)
        g = Nc + gf
        if owner is None:
            free[g] = True
            rows.append(g), cols.append(g), vals.append(1.0)
            continue
        constrained[g] = True
        # position in coarse-cell units: fine cell v // k, its GLL point v % k, halved
        xi = [(v // k + nodes[v % k]) / 2.0 - c for v, c in zip((I, J, L), owner)]
        cn = _cell_nodes(k, ncn, owner)
        n1 = k + 1
        for a2 in range(n1):
            for a1 in range(n1):
                for a0 in range(n1):
                    w = (lagrange(k, nodes, a0, xi[0]) * lagrange(k, nodes, a1, xi[1])
                         * lagrange(k, nodes, a2, xi[2]))
                    if w != 0.0:
                        rows.append(g), cols.append(int(cn[a0 + n1 * (a1 + n1 * a2)])), vals.append(w)
    C = sp.csr_matrix((vals, (rows, cols)), shape=(N, N))
    # Dirichlet faces of the box, on either lattice
    dirichlet = np.zeros(N, dtype=bool)
    for lat, (off, nn) in enumerate(((0, ncn), (Nc, nfn))):
        n = int(np.prod(nn))
        idx = np.arange(n)
        ii, jj, ll = idx % nn[0], (idx // nn[0]) % nn[1], idx // (nn[0] * nn[1])
        m = np.zeros(n, dtype=bool)
        for f, (v, top) in enumerate(((ii, nn[0] - 1), (jj, nn[1] - 1), (ll, nn[2] - 1))):
            if mesh.bc[2 * f] == 0:
                m |= v == 0
            if mesh.bc[2 * f + 1] == 0:
                m |= v == top
        dirichlet[off:off + n] = m
    return {"free": free, "constrained": constrained, "dirichlet": dirichlet & free, "C": C,
            "refined": refined.ravel()}


def cell_matrices(mesh, refined, phi):
    """A_cells: the sum of the element matrices of the active cells over the
    two-lattice index space (no constraint applied)."""
    k = mesh.degree
    ncel = list(mesh.ncells)
    refined = np.asarray(refined, dtype=bool).reshape(ncel[2], ncel[1], ncel[0])
    ncn, nfn, Nc, Nf = lattices(mesh)
    phi = np.asarray(phi, dtype=np.float64)
    hc = [e / n for e, n in zip(mesh.extent, ncel)]
    hf = [v / 2.0 for v in hc]
    rows, cols, vals = [], [], []
    for lat in ("coarse", "fine"):
        h = hc if lat == "coarse" else hf
        val, grad, W = _reference_basis(k, h)
        nn, off = (ncn, 0) if lat == "coarse" else (nfn, Nc)
        mult = 1 if lat == "coarse" else 2
        for cz in range(mult * ncel[2]):
            for cy in range(mult * ncel[1]):
                for cx in range(mult * ncel[0]):
                    parent = refined[cz // mult, cy // mult, cx // mult]
                    if (lat == "coarse") == bool(parent):
                        continue
                    g = off + _cell_nodes(k, nn, (cx, cy, cz))
                    c = _coefficient(mesh, val @ phi[g])
                    Ke = np.einsum("q,dqa,dqb->ab", c * W, grad, grad)
                    rows.append(np.repeat(g, g.size))
                    cols.append(np.tile(g, g.size))
                    vals.append(Ke.ravel())
    N = Nc + Nf
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))


def operator(mesh, refined, phi):
    """The two-lattice operator: C^T A_cells C on the free unknowns, identity on
    every other entry (constrained, unused and Dirichlet ones)."""
    cls = classify(mesh, refined)
    C = cls["C"]
    A = (C.T @ cell_matrices(mesh, refined, phi) @ C).tocsr()
    ident = ~cls["free"] | cls["dirichlet"]
    keep = sp.diags((~ident).astype(np.float64))
    A = (keep @ A @ keep + sp.diags(ident.astype(np.float64))).tocsr()
    A.eliminate_zeros()
    return A, cls


def node_coords(mesh):
    """Coordinates (x, y, z) of every entry of the two-lattice vector."""
    ncn, nfn, _, _ = lattices(mesh)
    out = []
    for nn, div in ((ncn, 1.0), (nfn, 2.0)):
        axes = []
        for d in range(3):
            h = mesh.extent[d] / mesh.ncells[d] / div
            nodes = gll_points(mesh.degree)
            cells = np.arange((nn[d] - 1) // mesh.degree)
            pts = (cells[:, None] + nodes[None, :-1]).ravel()
            pts = np.concatenate([pts, [len(cells)]])
            axes.append(mesh.origin[d] + pts * h)
        Z, Y, X = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
        out.append((X.ravel(), Y.ravel(), Z.ravel()))
    return tuple(np.concatenate([out[0][d], out[1][d]]) for d in range(3))


def load(mesh, refined, f):
    """C^T of the load sum_cells sum_q W_q f(x_q) N_a(x_q) over the active cells
    (f a function of x, y, z); zero on every entry that is not a free unknown."""
    k = mesh.degree
    ncel = list(mesh.ncells)
    ref = np.asarray(refined, dtype=bool).reshape(ncel[2], ncel[1], ncel[0])
    ncn, nfn, Nc, Nf = lattices(mesh)
    _, gx, _, _, _ = _tables(k)
    hc = [e / n for e, n in zip(mesh.extent, ncel)]
    ell = np.zeros(Nc + Nf)
    n1 = k + 1
    for lat in ("coarse", "fine"):
        mult = 1 if lat == "coarse" else 2
        h = [v / mult for v in hc]
        val, _, W = _reference_basis(k, h)
        nn, off = (ncn, 0) if lat == "coarse" else (nfn, Nc)
        for cz in range(mult * ncel[2]):
            for cy in range(mult * ncel[1]):
                for cx in range(mult * ncel[0]):
                    if (lat == "coarse") == bool(ref[cz // mult, cy // mult, cx // mult]):
                        continue
                    q0 = np.tile(np.arange(n1), n1 * n1)
                    q1 = np.tile(np.repeat(np.arange(n1), n1), n1)
                    q2 = np.repeat(np.arange(n1), n1 * n1)
                    xq = mesh.origin[0] + (cx + gx[q0]) * h[0]
                    yq = mesh.origin[1] + (cy + gx[q1]) * h[1]
                    zq = mesh.origin[2] + (cz + gx[q2]) * h[2]
                    g = off + _cell_nodes(k, nn, (cx, cy, cz))
                    np.add.at(ell, g, val.T @ (W * f(xq, yq, zq)))
    cls = classify(mesh, refined)
    b = cls["C"].T @ ell
    b[~cls["free"] | cls["dirichlet"]] = 0.0
    return b


def pcg(A, b, rtol=1e-12, max_iter=100000):
    """Textbook Jacobi-preconditioned CG from 0 (Krylov solver of Sec. "Numerical
    framework") with the stopping rule ||r|| < rtol ||r0|| of Table
    tab:solver_settings.  Returns (x, iterations)."""
    dinv = 1.0 / A.diagonal()
    x = np.zeros_like(b)
    r = b.copy()
    r0 = np.linalg.norm(r)
    z = dinv * r
    p = z.copy()
    rz = r @ z
    for it in range(1, max_iter + 1):
        q = A @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        if np.linalg.norm(r) < rtol * r0:
            return x, it
        z = dinv * r
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, max_iter


def band_mask(mesh, centre, radius, layers):
    """Coarse cells whose centre lies within `layers` cell sizes of the sphere
    |x - centre| = radius (the interface layers the paper refines)."""
    axes = [mesh.origin[d] + (np.arange(mesh.ncells[d]) + 0.5) * mesh.extent[d] / mesh.ncells[d] for d in range(3)]
    Z, Y, X = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    dist = np.abs(np.sqrt((X - centre[0]) ** 2 + (Y - centre[1]) ** 2 + (Z - centre[2]) ** 2) - radius)
    h = max(e / n for e, n in zip(mesh.extent, mesh.ncells))
    return (dist < layers * h).ravel()
