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
