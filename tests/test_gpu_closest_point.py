"""GPU closest-point projection (vpp_closest_points, and
vpp_closest_points_normal with a nodal normal field) against the oracle's
(oracle/closest_point.py, the appendix's normal and tangential corrections),
on unit cubes for k = 2-4, an anisotropic box away from the origin, a planar
interface and the full 64^3 band.

Bar: the band selection is identical (integer); points that converge on both
sides agree within 1e-9 (both stop once a step is below tol = 1e-11, and the
iteration contracts); their step counts differ by at most one (the stopping
test on a difference of rounded iterates).  Points that do not converge on
one side (their closest point lies on a cell face, where the C0 normal jumps,
and the iterates cycle) are checked for validity instead: still within the
cycle's amplitude of the oracle's iterate and close to the interface."""
import numpy as np
import pytest
import torch

import oracle
from oracle.closest_point import evaluate
import workloads as W
from gpu_util import dev, say

pytestmark = pytest.mark.gpu

vpp = pytest.importorskip("paper_2401_07805_amd")


def _problem(m, phi):
    p = vpp.Problem.from_mesh(m)
    p.set_phi(dev(phi))
    return p


@pytest.mark.parametrize("n,k", [(12, 2), (7, 3), (5, 4)])
def test_band_of_a_sphere_matches_oracle(n, k):
    eps = 0.05
    m = W.unit_cube(n, k, 1000.0, 1.0, bc=(1,) * 6)
    phi = W.droplet_phi(m, 0.3, eps, centre=(0.48, 0.51, 0.5))
    prob = _problem(m, phi)
    say("closest points band", n, k)
    y, info = prob.closest_points(eps, phi_lim=0.6, tol=1e-11, max_iter=50)
    y, info = y.cpu().numpy(), info.cpu().numpy()
    idx = oracle.band_nodes(m, phi, 0.6)
    out = np.setdiff1d(np.arange(m.ndofs), idx)
    assert (info[out] == -1).all() and (info[idx] >= 0).all()
    # outside the band y is the support point itself (GLL coordinates to rounding)
    np.testing.assert_allclose(y[out], oracle.node_coords(m, out), rtol=0, atol=1e-15)
    x = oracle.node_coords(m, idx)
    yo, so, do = oracle.closest_points(m, phi, x, eps, max_iter=50, tol=1e-11)
    yg, ig = y[idx], info[idx]
    both = do & (ig > 0)
    print(n, k, len(idx), "converged oracle", do.mean(), "gpu", (ig > 0).mean(), "both", both.mean())
    assert both.mean() > 0.75
    d = np.linalg.norm(yg[both] - yo[both], axis=1)
    assert d.max() < 1e-9, d.max()
    assert np.abs(ig[both] - so[both]).max() <= 1
    rest = ~both
    if rest.any():
        dr = np.linalg.norm(yg[rest] - yo[rest], axis=1)
        val, _ = evaluate(m, phi, yg[rest])
        print("not converged on one side:", rest.sum(), "max distance", dr.max(), "max |phi_h|", np.abs(val).max())
        assert dr.max() < 5e-3
        assert np.abs(val).max() < 0.05


def test_points_mode_and_plane_interface():
    eps = 0.1
    m = W.unit_cube(8, 2, 1000.0, 1.0, bc=(1,) * 6)
    phi = W.slab_phi(m, 0.5, eps)              # interface on the node plane x = 1/2
    prob = _problem(m, phi)
    rng = np.random.default_rng(9)
    pts = rng.uniform([0.3, 0.0, 0.0], [0.7, 1.0, 1.0], size=(500, 3))
    say("closest points plane")
    y, info = prob.closest_points(eps, pts=dev(pts), tol=1e-13)
    y, info = y.cpu().numpy(), info.cpu().numpy()
    assert (info > 0).all() and info.max() <= 6
    ref = pts.copy()
    ref[:, 0] = 0.5
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-12)
    # an empty point set is a no-op
    y0, i0 = prob.closest_points(eps, pts=torch.zeros((0, 3), dtype=torch.float64, device="cuda"))
    assert y0.shape == (0, 3) and i0.shape == (0,)


def test_closest_points_argument_errors():
    m = W.unit_cube(4, 2, 1000.0, 1.0)
    prob = vpp.Problem.from_mesh(m)
    with pytest.raises(vpp.VppError) as e:
        prob.closest_points(0.1)                # phi not set
    assert e.value.status == 7
    prob.set_phi(dev(W.droplet_phi(m, 0.3, 0.1)))
    for kw in ({"eps": 0.0}, {"eps": 0.1, "tol": 0.0}, {"eps": 0.1, "phi_lim": 1.5},
               {"eps": 0.1, "max_iter": 0}, {"eps": 0.1, "normal_steps": -1}):
        with pytest.raises(vpp.VppError) as e:
            prob.closest_points(**kw)
        assert e.value.status == 1


def test_extension_from_closest_points():
    """Values at the closest points extended over the band: a field that is
    constant along the normals of the sphere is unchanged (up to its
    interpolation error), and every band value equals the oracle's FE
    evaluation of the field at the GPU's closest point."""
    eps = 0.05
    m = W.unit_cube(10, 2, 1000.0, 1.0, bc=(1,) * 6)
    phi = W.droplet_phi(m, 0.3, eps)
    prob = _problem(m, phi)
    X, Y, Z = m.node_grid()
    f = (np.cos(2 * X) * (1 + Y) + Z ** 2).ravel()
    y, info = prob.closest_points(eps, phi_lim=0.6)
    out = prob.extend(y, info, dev(f))
    y, info, out = y.cpu().numpy(), info.cpu().numpy(), out.cpu().numpy()
    band = info >= 0
    np.testing.assert_array_equal(out[~band], f[~band])
    ref, _ = evaluate(m, f, y[band])
    np.testing.assert_allclose(out[band], ref, rtol=0, atol=1e-13)
    # a field constant along the radial lines is reproduced at the band nodes
    R = np.sqrt((X - 0.5) ** 2 + (Y - 0.5) ** 2 + (Z - 0.5) ** 2).ravel()
    g = np.where(R > 0, (X.ravel() - 0.5) / np.where(R > 0, R, 1.0), 0.0)   # x-component of the radial unit vector
    ext = prob.extend(dev(y), dev(info, torch.int32), dev(g)).cpu().numpy()
    assert np.abs(ext[band & (info > 0)] - g[band & (info > 0)]).max() < 0.05


def test_full_size_band_sample():
    """The 64^3 Q2 droplet's narrow band (the bench workload): a sample of 2000
    band nodes against the oracle, converged points within 1e-9."""
    wl = W.droplet_at_scale(k=2, nvec=0)
    m = wl.mesh
    prob = _problem(m, wl.phi)
    say("full size band")
    y, info = prob.closest_points(m.eps)
    y, info = y.cpu().numpy(), info.cpu().numpy()
    idx = oracle.band_nodes(m, wl.phi, 0.9)
    assert (info[idx] >= 0).all() and (info >= 0).sum() == len(idx)
    rng = np.random.default_rng(17)
    s = np.sort(rng.choice(idx, 2000, replace=False))
    yo, so, do = oracle.closest_points(m, wl.phi, oracle.node_coords(m, s), m.eps, max_iter=50, tol=1e-11)
    both = do & (info[s] > 0)
    assert both.mean() > 0.9
    assert np.linalg.norm(y[s][both] - yo[both], axis=1).max() < 1e-9


def _oracle_filtered_normal(m, phi, eta=2.0):
    """Inputs for both sides: the three solutions of the oracle's normal filter
    (M + eta h^2 K) n = (grad phi_h/|grad phi_h|, v), pure Neumann."""
    filt = eta / m.ncells[0] ** 2
    mf = W.Mesh(ncells=m.ncells, degree=m.degree, bc=(1,) * 6, rho_l=1 / filt, rho_g=1 / filt, mass=1.0)
    op = oracle.Operator(mf, phi=np.zeros(mf.ndofs), constrained=False)
    xq, yq, zq, _ = oracle.qp_coords(m)
    _, g = evaluate(m, phi, np.stack([xq, yq, zq], 1))
    nb = g / np.linalg.norm(g, axis=1)[:, None]
    return [op.pcg(oracle.rhs_qp(m, nb[:, d]), rtol=1e-12)[0] for d in range(3)]


@pytest.mark.parametrize("n,k", [(12, 2), (7, 3), (5, 4)])
def test_band_with_the_filtered_normal_matches_oracle(n, k):
    """vpp_closest_points_normal against the oracle with the same nodal normal
    field; with the continuous normal nearly every point converges on both sides."""
    eps = 0.05
    m = W.unit_cube(n, k, 1000.0, 1.0, bc=(1,) * 6)
    phi = W.droplet_phi(m, 0.3, eps, centre=(0.48, 0.51, 0.5))
    nf = _oracle_filtered_normal(m, phi)
    prob = _problem(m, phi)
    say("closest points band, filtered normal", n, k)
    y, info = prob.closest_points(eps, phi_lim=0.6, tol=1e-11, max_iter=50, normal=[dev(c) for c in nf])
    y, info = y.cpu().numpy(), info.cpu().numpy()
    idx = oracle.band_nodes(m, phi, 0.6)
    out = np.setdiff1d(np.arange(m.ndofs), idx)
    assert (info[out] == -1).all() and (info[idx] >= 0).all()
    x = oracle.node_coords(m, idx)
    yo, so, do = oracle.closest_points(m, phi, x, eps, max_iter=50, tol=1e-11, normal=nf)
    yg, ig = y[idx], info[idx]
    both = do & (ig > 0)
    print(n, k, len(idx), "converged oracle", do.mean(), "gpu", (ig > 0).mean(), "both", both.mean())
    assert both.mean() > 0.95
    assert np.linalg.norm(yg[both] - yo[both], axis=1).max() < 1e-9
    assert np.abs(ig[both] - so[both]).max() <= 1
    rest = ~both
    if rest.any():
        assert np.linalg.norm(yg[rest] - yo[rest], axis=1).max() < 5e-3


def test_points_mode_with_a_normal_field_and_errors():
    """Caller's points with a constant normal field on a planar interface
    (closest point (x0, y, z)), and the argument checks of the normal entry point."""
    import ctypes
    from paper_2401_07805_amd import _lib as L
    m = W.unit_cube(6, 2, 1000.0, 1.0, bc=(1,) * 6)
    eps = 0.1
    phi = W.slab_phi(m, 0.5, eps)
    prob = _problem(m, phi)
    rng = np.random.default_rng(3)
    pts = rng.uniform([0.3, 0.0, 0.0], [0.7, 1.0, 1.0], size=(500, 3))
    nf = [dev(np.full(m.ndofs, -1.0)), dev(np.zeros(m.ndofs)), dev(np.zeros(m.ndofs))]
    y, info = prob.closest_points(eps, pts=dev(pts), tol=1e-13, normal=nf)
    y, info = y.cpu().numpy(), info.cpu().numpy()
    ref = pts.copy()
    ref[:, 0] = 0.5
    assert (info > 0).all()
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-12)
    with pytest.raises(ValueError):
        prob.closest_points(eps, normal=nf[:2])
    o = L.CpOpts(eps, 0.9, 1e-11, 50, 3)
    yb = torch.empty((m.ndofs, 3), dtype=torch.float64, device="cuda")
    ib = torch.empty(m.ndofs, dtype=torch.int32, device="cuda")
    st = L.load().vpp_closest_points_normal(prob._h, None, 0, ctypes.c_void_p(nf[0].data_ptr()), None,
                                            ctypes.c_void_p(nf[2].data_ptr()), ctypes.byref(o),
                                            ctypes.c_void_p(yb.data_ptr()), ctypes.c_void_p(ib.data_ptr()), None)
    assert st == 1 and b"normal" in L.load().vpp_last_error()


def test_full_size_band_with_a_continuous_normal():
    """The 64^3 Q2 droplet's band with the droplet's exact (continuous) normal
    field as the nodal normal: a sample of 2000 band nodes against the oracle."""
    wl = W.droplet_at_scale(k=2, nvec=0)
    m = wl.mesh
    nf = W.normal_field(m)
    prob = _problem(m, wl.phi)
    say("full size band, continuous normal")
    y, info = prob.closest_points(m.eps, normal=[dev(c) for c in nf])
    y, info = y.cpu().numpy(), info.cpu().numpy()
    idx = oracle.band_nodes(m, wl.phi, 0.9)
    assert (info[idx] >= 0).all() and (info >= 0).sum() == len(idx)
    print("converged", (info[idx] > 0).mean())
    assert (info[idx] > 0).mean() > 0.99
    rng = np.random.default_rng(18)
    s = np.sort(rng.choice(idx, 2000, replace=False))
    yo, so, do = oracle.closest_points(m, wl.phi, oracle.node_coords(m, s), m.eps, max_iter=50, tol=1e-11,
                                       normal=nf)
    both = do & (info[s] > 0)
    assert both.mean() > 0.98
    assert np.linalg.norm(y[s][both] - yo[both], axis=1).max() < 1e-9


@pytest.mark.parametrize("use_normal", [False, True])
def test_anisotropic_offset_box_matches_oracle(use_normal):
    """Cells of different widths per direction and a box not at the origin
    (the 1/h_d of the gradient, the cell search from the origin, the clip to
    the box), with the gradient of phi_h and with a filtered normal field."""
    import dataclasses
    eps = 0.05
    m = W.Mesh(ncells=(10, 7, 9), degree=2, origin=(-0.1, 0.05, 0.0), extent=(1.2, 0.9, 1.0), bc=(1,) * 6)
    phi = W.droplet_phi(m, 0.3, eps, centre=(0.5, 0.5, 0.5))
    nf = None
    if use_normal:
        filt = 2.0 * max(m.h) ** 2
        mf = dataclasses.replace(m, rho_l=1 / filt, rho_g=1 / filt, mass=1.0)
        op = oracle.Operator(mf, phi=np.zeros(mf.ndofs), constrained=False)
        xq, yq, zq, _ = oracle.qp_coords(m)
        _, g = evaluate(m, phi, np.stack([xq, yq, zq], 1))
        nb = g / np.linalg.norm(g, axis=1)[:, None]
        nf = [op.pcg(oracle.rhs_qp(m, nb[:, d]), rtol=1e-12)[0] for d in range(3)]
    prob = _problem(m, phi)
    say("closest points anisotropic box, normal field" if use_normal else "closest points anisotropic box")
    y, info = prob.closest_points(eps, phi_lim=0.6, tol=1e-11, max_iter=50,
                                  normal=None if nf is None else [dev(c) for c in nf])
    y, info = y.cpu().numpy(), info.cpu().numpy()
    idx = oracle.band_nodes(m, phi, 0.6)
    assert (info[idx] >= 0).all() and (info >= 0).sum() == len(idx)
    x = oracle.node_coords(m, idx)
    yo, so, do = oracle.closest_points(m, phi, x, eps, max_iter=50, tol=1e-11, normal=nf)
    yg, ig = y[idx], info[idx]
    both = do & (ig > 0)
    print("converged oracle", do.mean(), "gpu", (ig > 0).mean(), "both", both.mean())
    assert both.mean() > (0.95 if use_normal else 0.75)
    assert np.linalg.norm(yg[both] - yo[both], axis=1).max() < 1e-9
    assert np.abs(ig[both] - so[both]).max() <= 1
