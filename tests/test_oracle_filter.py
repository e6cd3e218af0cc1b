"""Pins of the oracle's mass-shifted operator mu M + K_c.

With mu = 1 and a constant coefficient c = eta h^2 this is the weak form of
the level-set filters (Eqs. normal_vector_regularized and
curvature_regularized: n - eta h^2 Lap n = n_bar with homogeneous Neumann
conditions).  Checks: the Kronecker closed form of the element matrix (1D
mass factors from the textbook Q2 element), a brute-force dense assembly with
a variable coefficient and Dirichlet faces, the total mass 1^T A 1 = mu |Omega|
under pure Neumann (K_c 1 = 0), and the filter applied to cos(pi x), an
eigenfunction of the Neumann Laplacian, against its closed-form solution
cos(pi x) / (1 + eta h^2 pi^2) at the rate O(h^(k+1)).
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle
import workloads as W
from indep import dense_operator, element_1d

GOLD = os.path.join(os.path.dirname(__file__), "golden")
NEU = (1, 1, 1, 1, 1, 1)


@pytest.mark.parametrize("k", [2, 3, 4])
def test_element_matrix_kronecker_with_mass(k):
    ext = (0.5, 0.25, 2.0)
    mu, rho = 3.0, 4.0
    m = W.Mesh(ncells=(1, 1, 1), degree=k, extent=ext, bc=NEU, rho_l=rho, rho_g=rho, mass=mu)
    A = oracle.Operator(m, phi=np.zeros(m.ndofs), constrained=False).to_scipy().toarray()
    M, K = element_1d(k)
    if k == 2:
        g = json.load(open(os.path.join(GOLD, "q2_1d_element.json")))
        M = np.array(g["mass_times_30"]) / 30.0
        K = np.array(g["stiffness_times_3"]) / 3.0
    hx, hy, hz = ext
    Mx, My, Mz = M * hx, M * hy, M * hz
    Kx, Ky, Kz = K / hx, K / hy, K / hz
    ref = (np.kron(Mz, np.kron(My, Kx)) + np.kron(Mz, np.kron(Ky, Mx)) + np.kron(Kz, np.kron(My, Mx))) / rho
    ref += mu * np.kron(Mz, np.kron(My, Mx))
    np.testing.assert_allclose(A, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("ncells,k,bc", [
    ((2, 2, 1), 2, (0, 1, 1, 1, 0, 1)),
    ((2, 1, 1), 3, NEU),
])
def test_brute_force_dense_with_mass(ncells, k, bc):
    m = W.Mesh(ncells=ncells, degree=k, bc=bc, rho_l=1000.0, rho_g=1.0, mass=0.7)
    m.eps = 0.15
    phi = W.droplet_phi(m, 0.3, m.eps, centre=(0.45, 0.55, 0.5))
    cq = oracle.coef_qp(m, phi)
    nq = (k + 1) ** 3
    A_dense = dense_operator(m, lambda cell, q, x: cq[cell * nq + q[0] + (k + 1) * (q[1] + (k + 1) * q[2])],
                             mass=0.7)
    A = oracle.Operator(m, phi=phi, constrained=True).to_scipy().toarray()
    np.testing.assert_allclose(A, A_dense, rtol=0, atol=1e-14 * np.abs(A_dense).max())


@pytest.mark.parametrize("k", [2, 3])
def test_total_mass_under_neumann(k):
    ext = (1.0, 0.5, 0.75)
    mu = 2.5
    m = W.Mesh(ncells=(3, 2, 2), degree=k, extent=ext, bc=NEU, rho_l=1000.0, rho_g=1.0, mass=mu)
    m.eps = 0.2
    phi = W.droplet_phi(m, 0.3, m.eps)
    A = oracle.Operator(m, phi=phi, constrained=False)
    one = np.ones(m.ndofs)
    np.testing.assert_allclose(one @ A.matvec(one), mu * np.prod(ext), rtol=1e-13)
    # the same operator without the shift annihilates constants
    m0 = W.Mesh(ncells=(3, 2, 2), degree=k, extent=ext, bc=NEU, rho_l=1000.0, rho_g=1.0, mass=0.0)
    A0 = oracle.Operator(m0, phi=phi, constrained=False)
    np.testing.assert_allclose(A0.matvec(one), 0.0, atol=1e-12)


@pytest.mark.parametrize("k", [2, 3])
def test_filter_of_cosine_converges(k):
    """(M + eta h^2 K) n = M-projection of cos(pi x), pure Neumann, constant eta h^2."""
    filt = 0.01                      # eta h^2, fixed while the mesh is refined
    errs = []
    for n in (3, 6):
        m = W.Mesh(ncells=(n, n, n), degree=k, bc=NEU, rho_l=1.0 / filt, rho_g=1.0 / filt, mass=1.0)
        op = oracle.Operator(m, phi=np.zeros(m.ndofs), constrained=False)
        x, _, _, _ = oracle.qp_coords(m)
        b = oracle.rhs_qp(m, np.cos(np.pi * x))
        u = spla.spsolve(op.to_scipy().tocsc(), b)
        xe, _, _, we = oracle.qp_coords(m, nq=k + 3)   # a finer rule for the error
        exact = np.cos(np.pi * xe) / (1.0 + filt * np.pi ** 2)
        errs.append(np.sqrt(np.sum(we * (oracle.eval_qp(m, u, nq=k + 3) - exact) ** 2)))
    rate = np.log2(errs[0] / errs[1])
    assert errs[1] < 1e-3
    assert rate > k + 0.7, (errs, rate)
