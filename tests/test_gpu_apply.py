"""GPU parity of the matrix-free apply and diagonal against the FP64 oracle.

Bar: FP64 apply within 1e-12 relative (2-norm over all N entries, max-norm
reported too); FP32 apply within the rounding of an FP32 evaluation (stated
bound 2e-6 relative); every kernel configuration gives the same result.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import dev, host, rel, rel_max, say

pytestmark = pytest.mark.gpu

vpp = pytest.importorskip("paper_2401_07805_amd")


def setup_problem(mesh, phi):
    p = vpp.Problem.from_mesh(mesh)
    p.set_phi(dev(phi))
    return p


def test_c0_apply_fp64_all_configs():
    wl = W.small_droplet(n=8, k=2, seed=0)
    m = wl.mesh
    op = oracle.Operator(m, phi=wl.phi)
    yref = op.matvec(wl.vectors[0])
    prob = setup_problem(m, wl.phi)
    for cfg in vpp.config_candidates(2):
        say("c0 apply", cfg)
        prob.set_config(cfg["variant"], cfg["tile"])
        y = host(prob.apply(dev(wl.vectors[0])))
        assert rel(y, yref) < 1e-12, (cfg, rel(y, yref))
        assert rel_max(y, yref) < 1e-12, (cfg, rel_max(y, yref))


CASES = [
    # (ncells, k, bc, heaviside, extent)
    ((5, 4, 3), 2, (0,) * 6, W.H_LINEAR, (1.0, 1.0, 1.0)),
    ((9, 5, 7), 2, (0, 1, 1, 0, 0, 1), W.H_PAPER, (1.0, 0.6, 0.9)),
    ((1, 1, 1), 2, (0,) * 6, W.H_LINEAR, (1.0, 1.0, 1.0)),
    ((1, 1, 1), 2, (1,) * 6, W.H_LINEAR, (1.0, 1.0, 1.0)),
    # several complete tiles of every instantiated shape, mixed boundary conditions
    ((16, 8, 12), 2, (0, 1, 1, 0, 0, 1), W.H_PAPER, (1.0, 0.8, 1.1)),
    ((8, 16, 4), 2, (1, 0, 0, 1, 1, 0), W.H_LINEAR, (0.7, 1.0, 1.0)),
    ((6, 3, 5), 3, (0,) * 6, W.H_LINEAR, (1.0, 1.0, 1.0)),
    ((3, 4, 2), 3, (1, 0, 1, 1, 0, 1), W.H_PAPER, (0.5, 1.0, 0.7)),
    ((1, 1, 1), 3, (0,) * 6, W.H_LINEAR, (1.0, 1.0, 1.0)),
    ((4, 3, 5), 4, (0,) * 6, W.H_LINEAR, (1.0, 1.0, 1.0)),
    ((2, 3, 1), 4, (1, 1, 0, 0, 1, 1), W.H_PAPER, (1.0, 1.2, 0.8)),
    ((1, 1, 1), 4, (0,) * 6, W.H_LINEAR, (1.0, 1.0, 1.0)),
]


@pytest.mark.parametrize("ncells,k,bc,hv,ext", CASES)
def test_apply_degrees_shapes_bcs(ncells, k, bc, hv, ext):
    m = W.Mesh(ncells=ncells, degree=k, bc=bc, heaviside=hv, extent=ext, rho_l=1000.0, rho_g=1.0)
    m.eps = 0.1
    phi = W.droplet_phi(m, 0.3, m.eps, centre=(0.45, 0.5, 0.55))
    x = W.uniform_vectors(11, 1, m.ndofs)[0]
    yref = oracle.Operator(m, phi=phi).matvec(x)
    prob = setup_problem(m, phi)
    for cfg in vpp.config_candidates(k):
        say("apply", ncells, k, bc, hv, cfg)
        prob.set_config(cfg["variant"], cfg["tile"])
        y = host(prob.apply(dev(x)))
        assert rel(y, yref) < 1e-12, (cfg, rel(y, yref))
        assert rel_max(y, yref) < 1e-12, (cfg, rel_max(y, yref))


@pytest.mark.parametrize("k,n", [(2, 8), (3, 6), (4, 4)])
def test_apply_fp32_error(k, n):
    m = W.unit_cube(n, k, 1000.0, 1.0)
    m.eps = 2.0 / n
    phi = W.droplet_phi(m, 0.25, m.eps)
    x = W.uniform_vectors(0, 1, m.ndofs)[0]
    yref = oracle.Operator(m, phi=phi).matvec(x)
    prob = setup_problem(m, phi)
    for cfg in vpp.config_candidates(k):
        say("fp32 apply", k, n, cfg)
        prob.set_config(cfg["variant"], cfg["tile"])
        y = host(prob.apply(dev(x, dtype=__import__("torch").float32)))
        err = rel(y, yref)
        print(f"fp32 apply k={k} n={n} {cfg}: rel err {err:.3e}")
        assert err < 2e-6, cfg


@pytest.mark.parametrize("k,n,bc", [(2, (6, 5, 4), (0,) * 6), (3, (3, 4, 2), (1, 0, 1, 0, 1, 0)),
                                    (4, (2, 2, 3), (0,) * 6)])
def test_diagonal(k, n, bc):
    m = W.Mesh(ncells=n, degree=k, bc=bc, rho_l=1000.0, rho_g=1.0)
    m.eps = 0.12
    phi = W.droplet_phi(m, 0.3, m.eps)
    dref = oracle.Operator(m, phi=phi).diagonal()
    prob = setup_problem(m, phi)
    say("diag", k, n, bc)
    d = host(prob.diagonal())
    assert rel_max(d, dref) < 1e-13


def test_unit_vectors_reproduce_columns():
    """The GPU apply to every unit vector gives the oracle's matrix column."""
    m = W.Mesh(ncells=(2, 2, 1), degree=2, bc=(0, 1, 1, 1, 1, 0), rho_l=50.0, rho_g=1.0)
    m.eps = 0.2
    phi = W.droplet_phi(m, 0.3, m.eps)
    A = oracle.Operator(m, phi=phi).to_scipy().toarray()
    prob = setup_problem(m, phi)
    say("unit vectors")
    import torch
    E = torch.eye(m.ndofs, dtype=torch.float64, device="cuda")
    cols = np.stack([host(prob.apply(E[i].contiguous())) for i in range(m.ndofs)], axis=1)
    assert np.abs(cols - A).max() < 1e-13 * np.abs(A).max()


def test_full_size_sampled_rows_q2():
    """64^3 Q2 (2.15M DoFs), droplet r=0.25, eps=2h, seed-1 vector: sampled rows
    against the oracle's row-by-row evaluation, plus symmetry x.Ay = y.Ax."""
    wl = W.droplet_at_scale(k=2, nvec=2, seed=1)
    m = wl.mesh
    prob = setup_problem(m, wl.phi)
    prob.tune()
    say("full size q2", prob.config)
    x, z = wl.vectors[0], wl.vectors[1]
    y = host(prob.apply(dev(x)))
    rng = np.random.default_rng(123)
    rows = np.unique(np.concatenate([rng.choice(m.ndofs, 3000, replace=False),
                                     np.arange(0, m.ndofs, 4099)]))
    yr = oracle.apply_rows(m, wl.phi, x, rows)
    assert rel(y[rows], yr) < 1e-12
    assert rel_max(y[rows], yr) < 1e-12
    w = host(prob.apply(dev(z)))
    assert abs(np.dot(z, y) - np.dot(x, w)) < 1e-12 * np.linalg.norm(y) * np.linalg.norm(z)


@pytest.mark.parametrize("k", [3, 4])
def test_full_size_sampled_rows_q3_q4(k):
    wl = W.droplet_at_scale(k=k, nvec=1, seed=1)
    m = wl.mesh
    prob = setup_problem(m, wl.phi)
    say("full size", k, prob.config)
    x = wl.vectors[0]
    y = host(prob.apply(dev(x)))
    rng = np.random.default_rng(7)
    rows = rng.choice(m.ndofs, 1500, replace=False)
    yr = oracle.apply_rows(m, wl.phi, x, rows)
    assert rel(y[rows], yr) < 1e-12



def test_misaligned_vectors_are_rejected_before_any_launch():
    """Caller vectors not aligned to their element size return
    VPP_ERR_INVALID_ARG from the C ABI.  Every buffer holds one spare element,
    so even a launch on the shifted pointer would stay inside it; an aligned
    call afterwards still gives the same result as before."""
    import ctypes
    import torch
    import paper_2401_07805_amd as vpp
    from paper_2401_07805_amd import _lib as L
    lib = L.load()
    m = W.unit_cube(4, 2, 1000.0, 1.0)
    m.eps = 0.5
    n = m.ndofs
    prob = vpp.Problem.from_mesh(m)
    phi = W.droplet_phi(m, 0.3, m.eps)
    prob.set_phi(dev(phi))
    x = dev(W.uniform_vectors(0, 1, n)[0])
    y_ref = host(prob.apply(x))
    buf = torch.zeros(n + 1, dtype=torch.float64, device="cuda")
    out = torch.zeros(n + 1, dtype=torch.float64, device="cuda")
    b32 = torch.zeros(n + 1, dtype=torch.float32, device="cuda")
    o32 = torch.zeros(n + 1, dtype=torch.float32, device="cuda")
    y3 = torch.zeros(3 * n + 1, dtype=torch.float64, device="cuda")
    inf = torch.zeros(n + 1, dtype=torch.int32, device="cuda")
    P = lambda t, off=0: ctypes.c_void_p(t.data_ptr() + off)
    say("misaligned pointers")
    h = prob._h
    assert lib.vpp_apply(h, 0, P(buf, 4), P(out), None) == 1
    assert b"aligned" in lib.vpp_last_error()
    assert lib.vpp_apply(h, 0, P(buf), P(out, 4), None) == 1
    assert lib.vpp_apply(h, 1, P(b32, 2), P(o32), None) == 1
    assert lib.vpp_set_phi(h, P(buf, 4), None) == 1
    assert lib.vpp_diagonal(h, P(out, 4), None) == 1
    o = L.CgOpts(1e-8, 0.0, 10, 0, 1e-3, 100, 8)
    ci = L.CgInfo()
    assert lib.vpp_cg_solve(h, P(buf, 4), P(out), ctypes.byref(o), ctypes.byref(ci), None) == 1
    co = L.CpOpts(m.eps, 0.9, 1e-11, 50, 3)
    assert lib.vpp_closest_points(h, None, 0, ctypes.byref(co), P(y3, 4), P(inf), None) == 1
    assert lib.vpp_closest_points(h, None, 0, ctypes.byref(co), P(y3), P(inf, 2), None) == 1
    assert lib.vpp_extend(h, P(y3), P(inf, 2), P(buf), P(out), None) == 1
    torch.cuda.synchronize()
    # nothing above ran: the problem still applies as before
    assert rel(host(prob.apply(x)), y_ref) < 1e-14
