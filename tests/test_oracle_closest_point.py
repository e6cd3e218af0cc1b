"""Pins of the oracle's closest-point projection (appendix on closest point
projection, Eq. cpp; oracle/closest_point.py).

Checks: a planar interface on a node plane, where phi_h depends on x only and
vanishes exactly on the plane, so the closest point of (x, y, z) is (x0, y, z);
a sphere at a fixed interface thickness, where the projected points approach
the sphere at the interpolation order O(h^(k+1)) and their directions approach
the radial ones; and at every converged point the two defining properties,
phi_h(y) = 0 and x - y parallel to the normal at y.  The FE evaluation is
pinned against nodal values and against a tensor-product polynomial that the
Q_k space reproduces exactly.
"""
import numpy as np
import pytest

import oracle
from oracle.closest_point import evaluate
import workloads as W


@pytest.mark.parametrize("k", [2, 3, 4])
def test_evaluate_reproduces_q_k_polynomials(k):
    m = W.Mesh(ncells=(3, 2, 4), degree=k, extent=(1.0, 0.7, 1.3), bc=(1,) * 6)
    X, Y, Z = m.node_grid()
    f = lambda x, y, z: (x ** k - 2 * x) * (1 + y ** k) * (z ** (k - 1) + 0.5)
    phi = f(X, Y, Z).ravel()
    rng = np.random.default_rng(5)
    pts = rng.uniform([0, 0, 0], [1.0, 0.7, 1.3], size=(200, 3))
    val, grad = evaluate(m, phi, pts)
    x, y, z = pts.T
    np.testing.assert_allclose(val, f(x, y, z), rtol=1e-12, atol=1e-12)
    gx = (k * x ** (k - 1) - 2) * (1 + y ** k) * (z ** (k - 1) + 0.5)
    gy = (x ** k - 2 * x) * (k * y ** (k - 1)) * (z ** (k - 1) + 0.5)
    gz = (x ** k - 2 * x) * (1 + y ** k) * ((k - 1) * z ** (k - 2))
    np.testing.assert_allclose(grad, np.stack([gx, gy, gz], 1), rtol=1e-11, atol=1e-11)
    # at the nodes the interpolant takes the nodal values
    idx = np.arange(0, m.ndofs, 7)
    v, _ = evaluate(m, phi, oracle.node_coords(m, idx))
    np.testing.assert_allclose(v, phi[idx], rtol=0, atol=1e-13)


@pytest.mark.parametrize("k", [2, 3])
def test_plane_interface_exact(k):
    n = 8
    m = W.unit_cube(n, k, 1000.0, 1.0, bc=(1,) * 6)
    eps = 0.1
    phi = W.slab_phi(m, 0.5, eps)              # interface on the node plane x = 1/2
    idx = oracle.band_nodes(m, phi, 0.95)
    x = oracle.node_coords(m, idx)
    y, steps, done = oracle.closest_points(m, phi, x, eps, tol=1e-13)
    assert done.all() and steps.max() <= 3
    ref = x.copy()
    ref[:, 0] = 0.5
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-12)


def _sphere(n, k, eps=0.05, radius=0.3):
    m = W.unit_cube(n, k, 1000.0, 1.0, bc=(1,) * 6)
    phi = W.droplet_phi(m, radius, eps)
    idx = oracle.band_nodes(m, phi, 0.6)
    x = oracle.node_coords(m, idx)
    y, steps, done = oracle.closest_points(m, phi, x, eps, max_iter=50, tol=1e-11)
    return m, phi, x, y, done


@pytest.mark.parametrize("k", [2, 3])
def test_sphere_converges_at_interpolation_order(k):
    errs, derr = [], []
    for n in (8, 16):
        m, phi, x, y, done = _sphere(n, k)
        # points whose closest point sits near a cell face, where the C0 normal
        # jumps, may cycle between the two cells and stop at max_iter
        assert done.mean() > 0.8
        r = np.linalg.norm(y[done] - 0.5, axis=1)
        errs.append(np.abs(r - 0.3).max())
        u = (y[done] - 0.5) / r[:, None]
        ue = (x[done] - 0.5) / np.linalg.norm(x[done] - 0.5, axis=1)[:, None]
        derr.append(np.linalg.norm(u - ue, axis=1).max())
    assert np.log2(errs[0] / errs[1]) > k + 0.3, errs     # radius: O(h^(k+1))
    assert np.log2(derr[0] / derr[1]) > 1.0, derr         # direction: set by the C0 normal


def test_converged_points_satisfy_the_definition():
    m, phi, x, y, done = _sphere(12, 2)
    val, grad = evaluate(m, phi, y[done])
    assert np.abs(val).max() < 1e-10
    nrm = grad / np.linalg.norm(grad, axis=1)[:, None]
    d = x[done] - y[done]
    cross = np.linalg.norm(np.cross(d, nrm), axis=1)
    assert (cross < 1e-9 + 1e-9 * np.linalg.norm(d, axis=1)).all()


# ---------------------------------------------------------------------------
# The normal taken from a nodal normal field (n_Gamma of Eq. cpp is the
# filtered normal of Eq. normal_vector_regularized).

@pytest.mark.parametrize("k", [2, 3])
def test_plane_with_a_constant_normal_field(k):
    """phi(x) only, normal field a positive multiple of grad phi's direction
    (-e_x): the closest point of (x, y, z) is (x0, y, z), whatever the scale."""
    m = W.unit_cube(8, k, 1000.0, 1.0, bc=(1,) * 6)
    eps = 0.1
    phi = W.slab_phi(m, 0.5, eps)
    idx = oracle.band_nodes(m, phi, 0.95)
    x = oracle.node_coords(m, idx)
    nf = [np.full(m.ndofs, -2.5), np.zeros(m.ndofs), np.zeros(m.ndofs)]
    y, steps, done = oracle.closest_points(m, phi, x, eps, tol=1e-13, normal=nf)
    assert done.all() and steps.max() <= 3
    ref = x.copy()
    ref[:, 0] = 0.5
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-12)


def _filtered_normal(m, phi, eta=2.0):
    """The three solutions of (M + eta h^2 K) n = (grad phi_h/|grad phi_h|, v),
    pure Neumann, by the oracle's assembly and PCG."""
    n = m.ncells[0]
    filt = eta / n ** 2
    mf = W.Mesh(ncells=m.ncells, degree=m.degree, bc=(1,) * 6, rho_l=1 / filt, rho_g=1 / filt, mass=1.0)
    op = oracle.Operator(mf, phi=np.zeros(mf.ndofs), constrained=False)
    xq, yq, zq, _ = oracle.qp_coords(m)
    _, g = evaluate(m, phi, np.stack([xq, yq, zq], 1))
    nb = g / np.linalg.norm(g, axis=1)[:, None]
    return [op.pcg(oracle.rhs_qp(m, nb[:, d]), rtol=1e-12)[0] for d in range(3)]


def test_sphere_with_the_filtered_normal():
    """Droplet at 12^3 Q2: with the continuous filtered normal more points
    converge than with the C0 gradient, and every converged point satisfies
    the definition with that normal: phi_h(y) = 0 and x - y parallel to n_h(y)."""
    eps = 0.05
    m = W.unit_cube(12, 2, 1000.0, 1.0, bc=(1,) * 6)
    phi = W.droplet_phi(m, 0.3, eps)
    nf = _filtered_normal(m, phi)
    idx = oracle.band_nodes(m, phi, 0.6)
    x = oracle.node_coords(m, idx)
    y, steps, done = oracle.closest_points(m, phi, x, eps, max_iter=50, tol=1e-11, normal=nf)
    _, _, done_g = oracle.closest_points(m, phi, x, eps, max_iter=50, tol=1e-11)
    assert done.mean() > done_g.mean() and done.mean() > 0.95, (done.mean(), done_g.mean())
    val, _ = evaluate(m, phi, y[done])
    assert np.abs(val).max() < 1e-10
    nv = np.stack([evaluate(m, nf[d], y[done])[0] for d in range(3)], 1)
    nv /= np.linalg.norm(nv, axis=1)[:, None]
    d = x[done] - y[done]
    cross = np.linalg.norm(np.cross(d, nv), axis=1)
    assert (cross < 1e-9 + 1e-9 * np.linalg.norm(d, axis=1)).all()
    # and the points lie on the sphere to the interpolation error of phi_h
    r = np.linalg.norm(y[done] - 0.5, axis=1)
    assert np.abs(r - 0.3).max() < 2e-3
