"""Pins of the oracle's reinitialization step (Eq. reinitialization, one
semi-implicit Euler step in pseudo-time; oracle/reinit.py).

Checks: with the constant normal e_x the matrix is the Kronecker form
M/dtau + eps K_x (x-stiffness only) with the golden 1D Q2 factors; the matrix
is symmetric and positive definite for a variable normal; and the planar
tanh profile psi = tanh((x - x0)/(2 eps)) with its exact normal, a steady
state of the continuous equation ((1 - psi^2)/2 = eps dpsi/dx), is kept by a
step up to the discretisation error, which falls at the interpolation order.
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle
import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")
NEU = (1,) * 6


def test_constant_normal_kronecker_q2():
    ext = (0.5, 0.25, 2.0)
    m = W.Mesh(ncells=(1, 1, 1), degree=2, extent=ext, bc=NEU)
    n = m.ndofs
    normal = [np.ones(n), np.zeros(n), np.zeros(n)]
    eps, dtau = 0.3, 0.05
    A = oracle.reinit_matrix(m, normal, eps, dtau).toarray()
    g = json.load(open(os.path.join(GOLD, "q2_1d_element.json")))
    M = np.array(g["mass_times_30"]) / 30.0
    K = np.array(g["stiffness_times_3"]) / 3.0
    hx, hy, hz = ext
    ref = np.kron(M * hz, np.kron(M * hy, M * hx)) / dtau + eps * np.kron(M * hz, np.kron(M * hy, K / hx))
    np.testing.assert_allclose(A, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


def test_symmetric_positive_definite():
    m = W.unit_cube(3, 2, 1.0, 1.0, bc=NEU)
    comps = W.normal_field(m, (0.4, 0.55, 0.5))
    A = oracle.reinit_matrix(m, comps, 0.1, 0.05).toarray()
    np.testing.assert_allclose(A, A.T, rtol=0, atol=1e-14 * np.abs(A).max())
    assert np.linalg.eigvalsh(A).min() > 0


@pytest.mark.parametrize("k", [2, 3])
def test_planar_profile_is_steady(k):
    errs = []
    for n in (4, 8):
        m = W.Mesh(ncells=(n, 1, 1), degree=k, bc=NEU)
        eps = 0.1
        psi = W.slab_phi(m, 0.5, eps) * -1.0         # tanh((x - 0.5)/(2 eps)), increasing in x
        ones, zeros = np.ones(m.ndofs), np.zeros(m.ndofs)
        normal = [ones, zeros, zeros]               # grad psi / |grad psi| = e_x
        dtau = eps
        A = oracle.reinit_matrix(m, normal, eps, dtau)
        b = oracle.reinit_rhs(m, psi, normal, dtau)
        new = spla.spsolve(A.tocsc(), b)
        errs.append(np.abs(new - psi).max())
    assert errs[1] < errs[0] / 2 ** (k - 0.5), errs


def test_rhs_exact_for_linear_profile_q2():
    """k = 2, psi = a + b x (a Q2 function) and n = e_x: the integrands of the
    right-hand side have degree <= 5, which the 3-point Gauss rule integrates
    exactly, so b = M psi / dtau + (f_x, v) equals the 1D closed forms (numpy
    polynomial integrals of (1 - psi^2)/2 against the basis derivatives, the 1D
    mass matrix) times the node integrals in y and z."""
    from numpy.polynomial import Polynomial as Poly
    from indep import gll_closed_form, global_1d, lagrange_polys
    ncells, ext = (3, 1, 2), (0.6, 0.25, 2.0)
    m = W.Mesh(ncells=ncells, degree=2, extent=ext, bc=NEU)
    a0, b0, dtau = -0.3, 0.9, 0.07
    X, _, _ = m.node_grid()
    psi = a0 + b0 * X.ravel()
    ones, zeros = np.ones(m.ndofs), np.zeros(m.ndofs)
    b = oracle.reinit_rhs(m, psi, [ones, zeros, zeros], dtau)
    h = m.h
    Mx, _ = global_1d(2, ncells[0], h[0])
    My, _ = global_1d(2, ncells[1], h[1])
    Mz, _ = global_1d(2, ncells[2], h[2])
    xs = np.linspace(0.0, ext[0], 2 * ncells[0] + 1)
    L = lagrange_polys(gll_closed_form(2))
    fx = np.zeros(xs.size)
    for c in range(ncells[0]):
        x0 = c * h[0]
        xpoly = Poly([x0, h[0]])                       # x(xi) on the cell
        f = (1.0 - (a0 + b0 * xpoly) ** 2) / 2.0
        for a in range(3):
            fx[2 * c + a] += (f * L[a].deriv()).integ()(1.0)   # dx = h dxi, d/dx = d/dxi / h
    my, mz = My.sum(axis=1), Mz.sum(axis=1)
    ref = np.kron(mz, np.kron(my, Mx @ (a0 + b0 * xs))) / dtau + np.kron(mz, np.kron(my, fx))
    np.testing.assert_allclose(b, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("k", [2, 3])
def test_rows_match_full_assembly(k):
    """reinit_rows (cells around each node only) gives the rows of A x, diag(A)
    and b of the full assembly, on every node of a small mesh."""
    m = W.Mesh(ncells=(3, 2, 2), degree=k, bc=NEU)
    comps = W.normal_field(m, (0.4, 0.55, 0.5))
    eps, dtau = 0.1, 0.05
    psi = W.droplet_phi(m, 0.3, 0.05, centre=(0.4, 0.55, 0.5))
    x = W.uniform_vectors(5, 1, m.ndofs)[0]
    A = oracle.reinit_matrix(m, comps, eps, dtau)
    b = oracle.reinit_rhs(m, psi, comps, dtau)
    rows = np.arange(m.ndofs)
    ax, dg, rb = oracle.reinit_rows(m, comps, eps, dtau, x, psi, rows)
    np.testing.assert_allclose(ax, A @ x, rtol=0, atol=1e-13 * np.abs(A @ x).max())
    np.testing.assert_allclose(dg, A.diagonal(), rtol=0, atol=1e-13 * np.abs(A.diagonal()).max())
    np.testing.assert_allclose(rb, b, rtol=0, atol=1e-13 * np.abs(b).max())
