"""Pins of the oracle's coefficient law: Eq. heaviside, Eq. distance, Eq. rhoEff.

The sine ramp is checked through properties the paper's construction fixes
(H(0)=1/2, the phase symmetry H(phi)+H(-phi)=1, plateaus beyond |d|=3eps, a
smooth C^1 join, unit total mass of dH/dd), independence from eps when written
in phi, and the eps-free closed form in a = artanh(phi).
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from indep import heaviside_closed


def mesh_h(heaviside, eps=0.05, rho_l=1000.0, rho_g=1.0):
    m = W.unit_cube(1, 2, rho_l, rho_g)
    m.heaviside = heaviside
    m.eps = eps
    return m


def test_linear_heaviside_and_reciprocal_density():
    m = mesh_h(W.H_LINEAR, rho_l=1000.0, rho_g=2.0)
    assert oracle.heaviside(m, -1.0) == 0.0
    assert oracle.heaviside(m, 1.0) == 1.0
    assert oracle.heaviside(m, 0.0) == 0.5
    # pure phases: c = 1/rho of that phase (phi > 0 is liquid)
    assert abs(oracle.coefficient(m, 1.0) - 1 / 1000.0) < 1e-18
    assert abs(oracle.coefficient(m, -1.0) - 1 / 2.0) < 1e-18
    # interface: the reciprocal mean, not the arithmetic one
    c0 = oracle.coefficient(m, 0.0)
    assert abs(c0 - 0.5 * (1 / 1000.0 + 1 / 2.0)) < 1e-18
    assert abs(1.0 / c0 - 0.5 * (1000.0 + 2.0)) > 100
    # clamp: overshoots of the interpolated phi take the pure-phase value
    assert oracle.coefficient(m, 1.7) == oracle.coefficient(m, 1.0)
    assert oracle.coefficient(m, -3.0) == oracle.coefficient(m, -1.0)


def test_sine_ramp_properties():
    eps = 0.05
    m = mesh_h(W.H_PAPER, eps)
    assert abs(oracle.heaviside(m, 0.0) - 0.5) < 1e-16
    rng = np.random.default_rng(3)
    for phi in rng.uniform(-1, 1, 50):
        assert abs(oracle.heaviside(m, phi) + oracle.heaviside(m, -phi) - 1.0) < 1e-15
    t = math.tanh(1.5)                      # |d| = 3 eps  <=>  |phi| = tanh(3/2)
    for phi in (t + 1e-9, 0.95, 0.999999, 1.0):
        assert oracle.heaviside(m, phi) == 1.0
        assert oracle.heaviside(m, -phi) == 0.0
    # continuity and a flat (C^1) join at the plateau
    assert abs(oracle.heaviside(m, t - 1e-9) - 1.0) < 1e-8
    assert oracle.heaviside(m, t - 1e-6, deriv=True) < 1e-6
    # dH/dd integrates to 1 over the ramp: integrate dH/dphi dphi with phi = tanh(d/2eps)
    d = np.linspace(-3 * eps, 3 * eps, 20001)
    phi = np.tanh(d / (2 * eps))
    dHdphi = np.array([oracle.heaviside(m, p, deriv=True) for p in phi])
    dphidd = (1 - phi ** 2) / (2 * eps)
    assert abs(np.trapezoid(dHdphi * dphidd, d) - 1.0) < 1e-6


@pytest.mark.parametrize("eps", [0.5, 0.05, 1e-3])
def test_sine_ramp_eps_free_in_phi(eps):
    m = mesh_h(W.H_PAPER, eps)
    phis = np.linspace(-0.999, 0.999, 401)
    H = np.array([oracle.heaviside(m, p) for p in phis])
    np.testing.assert_allclose(H, heaviside_closed(phis, linear=False), rtol=0, atol=2e-15)


def test_sine_ramp_derivative_matches_difference_quotient():
    m = mesh_h(W.H_PAPER, 0.05)
    for phi in np.linspace(-0.89, 0.89, 37):
        h = 1e-6
        fd = (oracle.heaviside(m, phi + h) - oracle.heaviside(m, phi - h)) / (2 * h)
        assert abs(fd - oracle.heaviside(m, phi, deriv=True)) < 1e-7 * max(1.0, abs(fd))


def test_distance_inverse_of_profile():
    """H evaluated through d(phi) (Eq. distance) at phi = tanh(d/2eps) (Eq. initial_phi)
    equals the sine ramp written directly in d."""
    eps = 0.02
    m = mesh_h(W.H_PAPER, eps)
    for d in np.linspace(-2.9 * eps, 2.9 * eps, 29):
        phi = math.tanh(d / (2 * eps))
        direct = 0.5 + d / (6 * eps) + math.sin(math.pi * d / (3 * eps)) / (2 * math.pi)
        assert abs(oracle.heaviside(m, phi) - direct) < 1e-12


@pytest.mark.parametrize("paper", [False, True])
def test_arithmetic_mean_coefficient(paper):
    """coef_qp_arith: 1/(H rho_l + (1-H) rho_g) at the Gauss points.  By Jensen's
    inequality (1/x convex) it lies below the reciprocal mean of Eq. rhoEff
    wherever 0 < H < 1 and equals it where H is 0 or 1; at H = 1/2 it is
    2/(rho_l + rho_g); c rho = 1 with rho the arithmetic mean of the same H; and
    interpolated values beyond +-1 take the pure-phase value (clamp, R3)."""
    rl, rg = 1000.0, 2.0
    m = W.Mesh(ncells=(3, 2, 2), degree=2, rho_l=rl, rho_g=rg, heaviside=W.H_PAPER if paper else W.H_LINEAR)
    m.eps = 0.08
    phi = W.droplet_phi(m, 0.3, m.eps, centre=(0.45, 0.5, 0.55))
    ca = oracle.coef_qp_arith(m, phi, paper=paper)
    cr = oracle.coef_qp(m, phi)
    ph = np.clip(oracle.eval_qp(m, phi), -1, 1)
    H = heaviside_closed(ph, linear=not paper)
    inner = (H > 1e-12) & (H < 1 - 1e-12)
    assert inner.any() and (~inner).any() if paper else inner.all()
    assert np.all(ca[inner] < cr[inner])
    np.testing.assert_allclose(ca[~inner], cr[~inner], rtol=1e-14)
    # (the sine ramp's H here is the eps-free arctanh form, the oracle's the
    # logarithm of Eq. distance: equal up to the rounding of the two formulas)
    np.testing.assert_allclose(ca * (H * rl + (1 - H) * rg), 1.0, rtol=1e-12 if paper else 1e-14)
    # the value at H = 1/2 (phi_h = 0) and the clamp, through a constant nodal field
    for val, Hv in ((0.0, 0.5), (1.4, 1.0), (-2.0, 0.0)):
        c = oracle.coef_qp_arith(m, np.full(m.ndofs, val), paper=paper)
        np.testing.assert_allclose(c, 1.0 / (Hv * rl + (1 - Hv) * rg), rtol=1e-14)
