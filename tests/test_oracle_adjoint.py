"""Pins of the oracle's adjoint gradient (dJ/dc at Gauss points, dJ/dphi at nodes).

J = 1/2 ||p - p_t||^2 with A(c) p = b and b independent of phi.  Checked by
* central finite differences on individual coefficient values c_q and on nodal phi_j
  (re-assembling and re-solving exactly);
* the homogeneity identity sum_q c_q dJ/dc_q = -(p - p_t) . p, which holds because
  A(alpha c) = alpha A(c);
* the compliance sign: for J = b.p the gradient is -W_q |grad p|^2 <= 0.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle
import workloads as W


def setup(k=2, n=(2, 2, 2), heaviside=W.H_LINEAR):
    m = W.Mesh(ncells=n, degree=k, rho_l=20.0, rho_g=1.0, heaviside=heaviside)
    m.eps = 0.15
    phi = W.droplet_phi(m, 0.3, m.eps, centre=(0.45, 0.5, 0.55))
    phit = W.droplet_phi(m, 0.27, m.eps, centre=(0.45, 0.5, 0.55))
    b = oracle.sine_load(m)
    return m, phi, phit, b


def solve_phi(m, phi, b):
    A = oracle.Operator(m, phi=phi).to_scipy().tocsc()
    return spla.spsolve(A, b)


def solve_cq(m, cq, b):
    A = oracle.Operator(m, cq=cq).to_scipy().tocsc()
    return spla.spsolve(A, b)


def adjoint(m, phi, pt, b):
    A = oracle.Operator(m, phi=phi).to_scipy().tocsc()
    p = spla.spsolve(A, b)
    lam = spla.spsolve(A, p - pt)
    return p, lam, oracle.grad_coef(m, p, lam)


@pytest.mark.parametrize("k", [2, 3])
def test_grad_coef_finite_differences(k):
    m, phi, phit, b = setup(k, (2, 1, 2) if k == 3 else (2, 2, 2))
    pt = solve_phi(m, phit, b)
    p, lam, g = adjoint(m, phi, pt, b)
    cq = oracle.coef_qp(m, phi)
    J = lambda c: 0.5 * np.sum((solve_cq(m, c, b) - pt) ** 2)
    rng = np.random.default_rng(7)
    for q in rng.choice(cq.size, 6, replace=False):
        h = 1e-4 * cq[q]
        cp, cm = cq.copy(), cq.copy()
        cp[q] += h
        cm[q] -= h
        fd = (J(cp) - J(cm)) / (2 * h)
        assert abs(fd - g[q]) <= 1e-6 * max(abs(g).max(), 1e-30), (q, fd, g[q])


@pytest.mark.parametrize("heaviside", [W.H_LINEAR, W.H_PAPER])
def test_grad_phi_finite_differences(heaviside):
    m, phi, phit, b = setup(2, (2, 2, 2), heaviside)
    pt = solve_phi(m, phit, b)
    p, lam, g = adjoint(m, phi, pt, b)
    gphi = oracle.grad_phi(m, phi, g)
    J = lambda f: 0.5 * np.sum((solve_phi(m, f, b) - pt) ** 2)
    rng = np.random.default_rng(8)
    free = np.flatnonzero(~m.boundary_mask())
    for j in rng.choice(free, 6, replace=False):
        h = 1e-6
        fp, fm = phi.copy(), phi.copy()
        fp[j] += h
        fm[j] -= h
        fd = (J(fp) - J(fm)) / (2 * h)
        assert abs(fd - gphi[j]) <= 1e-5 * abs(gphi).max(), (j, fd, gphi[j])


def test_homogeneity_identity():
    m, phi, phit, b = setup(3, (2, 2, 1))
    pt = solve_phi(m, phit, b) * 0.7
    p, lam, g = adjoint(m, phi, pt, b)
    cq = oracle.coef_qp(m, phi)
    lhs = float(np.dot(cq, g))
    rhs = -float(np.dot(p - pt, p))
    assert abs(lhs - rhs) < 1e-11 * abs(rhs)


def test_compliance_sign():
    m, phi, _, b = setup(2)
    p = solve_phi(m, phi, b)
    g = oracle.grad_coef(m, p, p)           # J = b.p has lambda = p
    assert (g <= 0).all()
    # sum_q c_q g_q = -b.p (energy identity)
    cq = oracle.coef_qp(m, phi)
    assert abs(np.dot(cq, g) + np.dot(b, p)) < 1e-12 * abs(np.dot(b, p))
