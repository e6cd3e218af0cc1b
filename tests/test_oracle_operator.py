"""Pins of the oracle's assembled operator a(p,q) = sum W_q c(x_q) grad p . grad q.

Checks: Kronecker closed form of the constant-coefficient element matrix
(textbook 1D factors for Q2, exact polynomial integrals for Q3/Q4), a separate
brute-force dense assembly on 1-8 cells with a variable coefficient, symmetry,
the constant nullspace under pure Neumann, positive definiteness with
Dirichlet faces, linearity in the coefficient, and the patch test (Q_k
solutions are reproduced exactly).
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as W
from indep import dense_operator, element_1d, gauss01, gll_closed_form, lagrange_polys

GOLD = os.path.join(os.path.dirname(__file__), "golden")
NEU = (1, 1, 1, 1, 1, 1)


def one_cell(k, extent=(1.0, 1.0, 1.0), rho=4.0):
    m = W.Mesh(ncells=(1, 1, 1), degree=k, extent=extent, bc=NEU, rho_l=rho, rho_g=rho)
    return m


def test_q2_1d_factors_golden():
    g = json.load(open(os.path.join(GOLD, "q2_1d_element.json")))
    M, K = element_1d(2)
    np.testing.assert_allclose(M * 30, g["mass_times_30"], atol=1e-13)
    np.testing.assert_allclose(K * 3, g["stiffness_times_3"], atol=1e-13)


@pytest.mark.parametrize("k", [2, 3, 4])
def test_element_matrix_kronecker(k):
    ext = (0.5, 0.25, 2.0)
    m = one_cell(k, ext, rho=4.0)
    c = 1.0 / 4.0
    A = oracle.Operator(m, phi=np.zeros(m.ndofs), constrained=False).to_scipy().toarray()
    M, K = element_1d(k)
    if k == 2:
        g = json.load(open(os.path.join(GOLD, "q2_1d_element.json")))
        M = np.array(g["mass_times_30"]) / 30.0
        K = np.array(g["stiffness_times_3"]) / 3.0
    hx, hy, hz = ext
    Mx, My, Mz = M * hx, M * hy, M * hz
    Kx, Ky, Kz = K / hx, K / hy, K / hz
    ref = c * (np.kron(Mz, np.kron(My, Kx)) + np.kron(Mz, np.kron(Ky, Mx))
               + np.kron(Kz, np.kron(My, Mx)))
    np.testing.assert_allclose(A, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


def droplet_mesh(ncells, k, bc=(0,) * 6, rho_l=1000.0, rho_g=1.0, heaviside=W.H_LINEAR):
    m = W.Mesh(ncells=ncells, degree=k, bc=bc, rho_l=rho_l, rho_g=rho_g, heaviside=heaviside)
    m.eps = 0.15
    phi = W.droplet_phi(m, 0.3, m.eps, centre=(0.45, 0.55, 0.5))
    return m, phi


@pytest.mark.parametrize("ncells,k,bc,hv", [
    ((1, 1, 1), 2, NEU, W.H_LINEAR),
    ((2, 2, 2), 2, (0,) * 6, W.H_LINEAR),
    ((2, 1, 2), 2, (0, 1, 1, 0, 0, 1), W.H_PAPER),
    ((2, 1, 1), 3, (0, 1, 1, 1, 1, 1), W.H_LINEAR),
    ((1, 2, 1), 4, (1, 1, 0, 0, 1, 1), W.H_LINEAR),
])
def test_brute_force_dense(ncells, k, bc, hv):
    m, phi = droplet_mesh(ncells, k, bc, heaviside=hv)
    cq = oracle.coef_qp(m, phi)
    nq = (k + 1) ** 3
    # the coefficient values are an input here: the brute force takes the same c_q
    A_dense = dense_operator(m, lambda cell, q, x: cq[cell * nq + q[0] + (k + 1) * (q[1] + (k + 1) * q[2])])
    A = oracle.Operator(m, phi=phi, constrained=True).to_scipy().toarray()
    np.testing.assert_allclose(A, A_dense, rtol=0, atol=1e-14 * np.abs(A_dense).max())


def test_coef_qp_is_interpolated_phi():
    """c_q from the oracle equals the law applied to phi_h(x_q) computed independently."""
    k = 3
    m, phi = droplet_mesh((2, 1, 2), k)
    cq = oracle.coef_qp(m, phi)
    L = lagrange_polys(gll_closed_form(k))
    gx, _ = gauss01(k + 1)
    Nx, Ny, _ = m.nnodes
    n1 = k + 1
    rho_l, rho_g = m.rho_l, m.rho_g
    for cell in range(4):
        cx, cy, cz = cell % 2, 0, cell // 2
        for q in range(n1 ** 3):
            q0, q1, q2 = q % n1, (q // n1) % n1, q // (n1 * n1)
            s = 0.0
            for a2 in range(n1):
                for a1 in range(n1):
                    for a0 in range(n1):
                        g = (k * cx + a0) + Nx * ((k * cy + a1) + Ny * (k * cz + a2))
                        s += L[a0](gx[q0]) * L[a1](gx[q1]) * L[a2](gx[q2]) * phi[g]
            s = min(1.0, max(-1.0, s))
            H = 0.5 * (s + 1)
            assert abs(cq[cell * n1 ** 3 + q] - (H / rho_l + (1 - H) / rho_g)) < 5e-14


@pytest.mark.parametrize("k", [2, 3, 4])
def test_symmetry_nullspace_spd_linearity(k):
    n = {2: (3, 2, 2), 3: (2, 2, 2), 4: (2, 1, 2)}[k]
    m, phi = droplet_mesh(n, k, bc=NEU)
    A = oracle.Operator(m, phi=phi, constrained=False).to_scipy()
    assert abs(A - A.T).max() == 0.0
    ones = np.ones(m.ndofs)
    assert np.abs(A @ ones).max() < 1e-13 * abs(A).max()
    # Dirichlet faces: SPD
    md, _ = droplet_mesh(n, k, bc=(0,) * 6)
    Ad = oracle.Operator(md, phi=phi, constrained=True).to_scipy().toarray()
    assert np.linalg.eigvalsh(Ad).min() > 0
    # linearity in the coefficient: halving both densities doubles c and A
    m2, _ = droplet_mesh(n, k, bc=NEU, rho_l=500.0, rho_g=0.5)
    A2 = oracle.Operator(m2, phi=phi, constrained=False).to_scipy()
    assert abs(A2 - 2.0 * A).max() < 1e-14 * abs(A2).max()


def _poly_terms(k):
    """p* in Q_k vanishing on the cube faces, as separable terms (px, py, pz)."""
    from numpy.polynomial import Polynomial as P
    b = P([0.0, 1.0, -1.0])            # x(1-x)
    if k == 2:
        return [(b, b, b)]
    xb = b * P([0.0, 1.0])
    if k == 3:                        # x(1-x)y(1-y)z(1-z)(x+y+z)
        return [(xb, b, b), (b, xb, b), (b, b, xb)]
    x2b = b * P([0.0, 0.0, 1.0])      # (x+y+z)^2 expanded
    return [(x2b, b, b), (b, x2b, b), (b, b, x2b), (xb, xb, b), (xb, xb, b),
            (xb, b, xb), (xb, b, xb), (b, xb, xb), (b, xb, xb)]


@pytest.mark.parametrize("k,n", [(2, 3), (3, 2), (4, 2)])
def test_patch_exactness(k, n):
    """Constant c, p* in Q_k with zero boundary values: the FE solution is p* at the nodes."""
    m = W.unit_cube(n, k, 2.0, 2.0)      # c = 1/2
    c = 0.5
    terms = _poly_terms(k)
    x, y, z, _ = oracle.qp_coords(m)
    lap = np.zeros_like(x)
    for px, py, pz in terms:
        lap += (px.deriv(2)(x) * py(y) * pz(z) + px(x) * py.deriv(2)(y) * pz(z)
                + px(x) * py(y) * pz.deriv(2)(z))
    b = oracle.rhs_qp(m, -c * lap)
    b[m.boundary_mask()] = 0.0
    op = oracle.Operator(m, phi=np.zeros(m.ndofs))
    import scipy.sparse.linalg as spla
    p = spla.spsolve(op.to_scipy().tocsc(), b)
    X, Y, Z = m.node_grid()
    ref = sum(px(X) * py(Y) * pz(Z) for px, py, pz in terms).ravel()
    assert np.abs(p - ref).max() < 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("k,n,bc", [(2, (5, 4, 3), (0,) * 6), (3, (3, 2, 4), (0, 1, 0, 1, 1, 0)), (4, (2, 3, 2), NEU)])
def test_apply_rows_match_matrix(k, n, bc):
    m, phi = droplet_mesh(n, k, bc=bc)
    op = oracle.Operator(m, phi=phi)
    x = np.random.default_rng(9).uniform(-1, 1, m.ndofs)
    y = op.matvec(x)
    rows = np.arange(m.ndofs)
    np.testing.assert_allclose(oracle.apply_rows(m, phi, x, rows), y, rtol=0, atol=1e-13 * np.abs(y).max())


@pytest.mark.parametrize("ncells,k,bc,hv,mass", [
    ((2, 2, 2), 2, (0,) * 6, W.H_LINEAR, 0.0),
    ((2, 1, 2), 2, (0, 1, 1, 0, 0, 1), W.H_PAPER, 0.0),
    ((2, 1, 1), 3, (1,) * 6, W.H_LINEAR, 2.5),
    ((1, 2, 1), 4, (1, 1, 0, 0, 1, 1), W.H_LINEAR, 0.0),
])
def test_diagonal_brute_force(ncells, k, bc, hv, mass):
    """orc_diag returns the diagonal of the brute-force dense matrix (identity
    entries on Dirichlet rows), with and without the mass shift."""
    m, phi = droplet_mesh(ncells, k, bc, heaviside=hv)
    m.mass = mass
    cq = oracle.coef_qp(m, phi)
    nq = (k + 1) ** 3
    A_dense = dense_operator(m, lambda cell, q, x: cq[cell * nq + q[0] + (k + 1) * (q[1] + (k + 1) * q[2])],
                             mass=mass)
    d = oracle.Operator(m, phi=phi).diagonal()
    ref = np.diag(A_dense)
    np.testing.assert_allclose(d, ref, rtol=0, atol=1e-14 * np.abs(ref).max())
    assert np.all(d[m.boundary_mask()] == 1.0)
