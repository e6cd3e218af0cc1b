"""Pins of the oracle's operator on a once-refined mesh with hanging nodes
(oracle/amr.py): without refinement it is the uniform oracle on the coarse
lattice, with every cell refined the uniform oracle on the fine one; the
hanging-node weights reproduce Q_k polynomials; the matrix is symmetric and
has the constant nullspace under pure Neumann faces; a function of the coarse
Q_k space has the same energy on the refined mesh as on the coarse one
(constant coefficient, exact quadrature); and the patch test: a Q_k solution
vanishing on the box is reproduced exactly across the hanging faces."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle
import workloads as W
from oracle import amr
from indep import gll_closed_form, lagrange_polys

NEU = (1,) * 6


def _mesh(nc, k, bc=(0,) * 6, rho_l=1000.0, rho_g=1.0, hv=W.H_LINEAR):
    m = W.Mesh(ncells=nc, degree=k, bc=bc, rho_l=rho_l, rho_g=rho_g, heaviside=hv)
    m.eps = 0.15
    return m


def _phi2(m, centre=(0.45, 0.52, 0.5), r=0.3):
    """Nodal droplet phi on both lattices (each node its own sample)."""
    x, y, z = amr.node_coords(m)
    d = r - np.sqrt((x - centre[0]) ** 2 + (y - centre[1]) ** 2 + (z - centre[2]) ** 2)
    return np.tanh(d / (2 * m.eps))


def _mask(nc, cells):
    r = np.zeros(nc[::-1], dtype=bool)
    for (cx, cy, cz) in cells:
        r[cz, cy, cx] = True
    return r.ravel()


MASKS = {
    "box": lambda nc: _mask(nc, [(x, y, z) for x in (1, 2) for y in (1, 2) for z in (1,)]),
    "L": lambda nc: _mask(nc, [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]),
    "edge": lambda nc: _mask(nc, [(0, 0, 0), (1, 1, 0), (2, 2, 1)]),   # cells meeting along edges only
}


@pytest.mark.parametrize("k", [2, 3])
def test_no_refinement_and_full_refinement(k):
    nc = (3, 2, 2)
    m = _mesh(nc, k, bc=(0, 1, 1, 0, 0, 1), hv=W.H_PAPER)
    phi = _phi2(m)
    _, _, Nc, Nf = amr.lattices(m)
    A, cls = amr.operator(m, np.zeros(np.prod(nc), dtype=bool), phi)
    ref = oracle.Operator(m, phi=phi[:Nc]).to_scipy()
    assert abs(A[:Nc, :Nc] - ref).max() < 1e-14 * abs(ref).max()
    assert abs(A[Nc:, Nc:] - np.eye(Nf)).max() == 0 and abs(A[:Nc, Nc:]).max() == 0
    A, cls = amr.operator(m, np.ones(np.prod(nc), dtype=bool), phi)
    mf = _mesh(tuple(2 * v for v in nc), k, bc=m.bc, hv=W.H_PAPER)
    ref = oracle.Operator(mf, phi=phi[Nc:]).to_scipy()
    assert abs(A[Nc:, Nc:] - ref).max() < 1e-14 * abs(ref).max()
    assert abs(A[:Nc, :Nc] - np.eye(Nc)).max() == 0


@pytest.mark.parametrize("k", [2, 3, 4])
@pytest.mark.parametrize("shape", ["box", "L", "edge"])
def test_hanging_weights_reproduce_polynomials(k, shape):
    """Each constrained row of C evaluates the coarse Q_k interpolant: applied to
    the coarse nodal values of a polynomial of degree <= k in each variable it
    gives the polynomial at the hanging node (numpy polynomials, independent of
    the oracle's basis code)."""
    nc = (3, 3, 2)
    m = _mesh(nc, k)
    cls = amr.classify(m, MASKS[shape](nc))
    x, y, z = amr.node_coords(m)
    rng = np.random.default_rng(k)
    coef = rng.uniform(-1, 1, (k + 1, k + 1, k + 1))
    P = lambda X, Y, Z: np.einsum("abc,...a,...b,...c->...", coef, np.stack([X ** i for i in range(k + 1)], -1),
                                  np.stack([Y ** i for i in range(k + 1)], -1), np.stack([Z ** i for i in range(k + 1)], -1))
    v = P(x, y, z)
    con = cls["constrained"]
    assert con.any()
    got = cls["C"][con] @ np.where(cls["free"], v, 0.0)
    np.testing.assert_allclose(got, v[con], rtol=0, atol=1e-12 * np.abs(v).max())
    # partition of unity
    np.testing.assert_allclose(np.asarray(cls["C"][con].sum(axis=1)).ravel(), 1.0, atol=1e-13)


@pytest.mark.parametrize("k", [2, 3])
@pytest.mark.parametrize("shape", ["box", "edge"])
def test_symmetry_and_neumann_nullspace(k, shape):
    nc = (3, 3, 2)
    m = _mesh(nc, k, bc=NEU)
    phi = _phi2(m)
    A, cls = amr.operator(m, MASKS[shape](nc), phi)
    assert abs(A - A.T).max() < 1e-14 * abs(A).max()
    one = cls["free"].astype(np.float64)
    r = A @ one
    assert np.abs(r[cls["free"]]).max() < 1e-12 * abs(A).max()
    # positive definite once Dirichlet faces are added
    m2 = _mesh(nc, k, bc=(0, 1, 1, 0, 0, 1))
    A2, _ = amr.operator(m2, MASKS[shape](nc), phi)
    assert np.linalg.eigvalsh(A2.toarray()).min() > 0


@pytest.mark.parametrize("k", [2, 3])
def test_coarse_function_energy(k):
    """u in the coarse Q_k space (nodal values on the coarse lattice, its
    interpolant, evaluated with numpy polynomials, at the free fine nodes):
    u^T A u on the refined mesh equals u_c^T A_c u_c on the uniform coarse mesh
    for a constant coefficient."""
    nc = (3, 3, 2)
    m = _mesh(nc, k, bc=NEU, rho_l=4.0, rho_g=4.0)
    mask = MASKS["L"](nc)
    _, _, Nc, _ = amr.lattices(m)
    A, cls = amr.operator(m, mask, np.zeros(amr.num_dofs(m)))
    uc = np.random.default_rng(7).uniform(-1, 1, Nc)
    L = lagrange_polys(gll_closed_form(k))
    x, y, z = amr.node_coords(m)
    h = [e / n for e, n in zip(m.extent, nc)]
    u = np.zeros(amr.num_dofs(m))
    u[:Nc] = np.where(cls["free"][:Nc], uc, 0.0)
    Nxc = k * nc[0] + 1
    Nyc = k * nc[1] + 1
    for g in np.flatnonzero(cls["free"][Nc:]) + Nc:
        X = (x[g] / h[0], y[g] / h[1], z[g] / h[2])
        cell = [min(int(v), n - 1) for v, n in zip(X, nc)]
        xi = [v - c for v, c in zip(X, cell)]
        s = 0.0
        for a2 in range(k + 1):
            for a1 in range(k + 1):
                for a0 in range(k + 1):
                    gc = (k * cell[0] + a0) + Nxc * ((k * cell[1] + a1) + Nyc * (k * cell[2] + a2))
                    s += L[a0](xi[0]) * L[a1](xi[1]) * L[a2](xi[2]) * uc[gc]
        u[g] = s
    e_ref = uc @ (oracle.Operator(m, phi=np.zeros(Nc)).to_scipy() @ uc)
    e = u @ (A @ u)
    assert abs(e - e_ref) < 1e-12 * abs(e_ref)


@pytest.mark.parametrize("k", [2, 3])
@pytest.mark.parametrize("shape", ["box", "L", "edge"])
def test_patch_across_hanging_faces(k, shape):
    """Constant coefficient, Dirichlet faces, p* of degree <= k in each variable
    vanishing on the box: the refined solution equals p* at every free node."""
    nc = (3, 3, 2)
    m = _mesh(nc, k, rho_l=1.0, rho_g=1.0)
    mask = MASKS[shape](nc)
    A, cls = amr.operator(m, mask, np.zeros(amr.num_dofs(m)))
    if k == 2:
        p = lambda x, y, z: x * (1 - x) * y * (1 - y) * z * (1 - z)
        f = lambda x, y, z: 2 * (y * (1 - y) * z * (1 - z) + x * (1 - x) * z * (1 - z) + x * (1 - x) * y * (1 - y))
    else:
        p = lambda x, y, z: x * (1 - x) * y * (1 - y) * z * (1 - z) * (x + y + z)
        f = lambda x, y, z: -((-2 * (x + y + z) + 2 * (1 - 2 * x)) * y * (1 - y) * z * (1 - z)
                              + (-2 * (x + y + z) + 2 * (1 - 2 * y)) * x * (1 - x) * z * (1 - z)
                              + (-2 * (x + y + z) + 2 * (1 - 2 * z)) * x * (1 - x) * y * (1 - y))
    b = amr.load(m, mask, f)
    sol = spla.spsolve(A.tocsc(), b)
    x, y, z = amr.node_coords(m)
    ex = p(x, y, z)
    fr = cls["free"] & ~cls["dirichlet"]
    assert np.abs(sol[fr] - ex[fr]).max() < 1e-12 * np.abs(ex).max()


def test_pcg_matches_direct_solve():
    """The AMR oracle's Jacobi PCG reaches the sparse direct solution."""
    nc = (3, 3, 2)
    m = _mesh(nc, 2)
    A, cls = amr.operator(m, MASKS["L"](nc), _phi2(m))
    b = amr.load(m, MASKS["L"](nc), lambda x, y, z: np.sin(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z))
    x, it = amr.pcg(A, b, rtol=1e-13)
    xd = spla.spsolve(A.tocsc(), b)
    assert it > 1 and np.linalg.norm(x - xd) < 1e-10 * np.linalg.norm(xd)
