"""GPU adjoint: dJ/dc at Gauss points and dJ/dphi at nodes.

Checked against the oracle's assembled-matrix gradient on 8^3 Q2 (same p and
lambda), the homogeneity identity sum_q c_q g_q = -(p - p_t).p, and central
finite differences of J through the autograd Function.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

import oracle
import workloads as W
from gpu_util import dev, host, rel, rel_max, say

pytestmark = pytest.mark.gpu

vpp = pytest.importorskip("paper_2401_07805_amd")


@pytest.mark.parametrize("k,hv", [(2, W.H_LINEAR), (2, W.H_PAPER), (3, W.H_LINEAR), (4, W.H_LINEAR)])
def test_gradients_match_oracle(k, hv):
    n = {2: 8, 3: 4, 4: 3}[k]
    m, phi, phit = W.adjoint_case(n=n, k=k)
    m.heaviside = hv
    A = oracle.Operator(m, phi=phi).to_scipy().tocsc()
    At = oracle.Operator(m, phi=phit).to_scipy().tocsc()
    b = oracle.sine_load(m)
    p = spla.spsolve(A, b)
    pt = spla.spsolve(At, b)
    lam = spla.spsolve(A, p - pt)
    gref = oracle.grad_coef(m, p, lam)
    gphi_ref = oracle.grad_phi(m, phi, gref)
    prob = vpp.Problem.from_mesh(m)
    prob.set_phi(dev(phi))
    say("grad", k, hv)
    g = host(prob.grad_coef(dev(p), dev(lam)))
    assert rel_max(g, gref) < 1e-12
    gphi = host(prob.grad_phi(dev(gref)))
    assert rel_max(gphi, gphi_ref) < 1e-12
    cq = oracle.coef_qp(m, phi)
    assert abs(np.dot(cq, g) + np.dot(p - pt, p)) < 1e-11 * abs(np.dot(p - pt, p))


def test_autograd_function_c4_small():
    """8^3 Q2, droplet r=0.3 vs target r=0.28: autograd gradient == oracle chain,
    and central differences (step 1e-6) at seeded interior nodes."""
    m, phi, phit = W.adjoint_case(n=8, k=2)
    b = oracle.sine_load(m)
    A = oracle.Operator(m, phi=phi).to_scipy().tocsc()
    At = oracle.Operator(m, phi=phit).to_scipy().tocsc()
    pt = spla.spsolve(At, b)
    prob = vpp.Problem.from_mesh(m)
    say("autograd small")
    opts = dict(rtol=1e-13)
    phi_t = dev(phi).requires_grad_(True)
    p = vpp.poisson_solve(phi_t, dev(b), prob, **opts)
    J = 0.5 * ((p - dev(pt)) ** 2).sum()
    J.backward()
    gphi = host(phi_t.grad)
    pr = spla.spsolve(A, b)
    lam = spla.spsolve(A, pr - pt)
    gref = oracle.grad_phi(m, phi, oracle.grad_coef(m, pr, lam))
    assert rel_max(gphi, gref) < 1e-8
    assert prob.last_grad_coef is not None and prob.last_grad_coef.numel() == prob.nq

    def Jof(f):
        prob.set_phi(dev(f))
        x, _ = prob.cg_solve(dev(b), rtol=1e-13)
        return 0.5 * float(((host(x) - pt) ** 2).sum())

    nodes = W.fd_nodes(m, count=8, seed=4)
    for j in nodes:
        h = 1e-6
        fp, fm = phi.copy(), phi.copy()
        fp[j] += h
        fm[j] -= h
        fd = (Jof(fp) - Jof(fm)) / (2 * h)
        assert abs(fd - gphi[j]) <= 1e-5 * np.abs(gphi).max() + 1e-7 * abs(fd), (j, fd, gphi[j])


def test_autograd_c4_full_size_fd_32_nodes():
    """48^3 Q2, droplet r=0.3 vs target r=0.28, ratio 1000: dJ/dphi from the
    autograd Function against central differences (step 1e-6) of J at the 32
    seeded nodes; the homogeneity identity at full size."""
    m, phi, phit = W.adjoint_case(n=48, k=2)
    b = dev(oracle.sine_load(m))
    prob = vpp.Problem.from_mesh(m)
    say("c4 48^3 target solve")
    prob.set_phi(dev(phit))
    pt, _ = prob.cg_solve(b, rtol=1e-13)
    phi_t = dev(phi).requires_grad_(True)
    say("c4 48^3 forward + adjoint")
    p = vpp.poisson_solve(phi_t, b, prob, rtol=1e-13)
    J = 0.5 * ((p - pt) ** 2).sum()
    J.backward()
    gphi = host(phi_t.grad)
    g = prob.last_grad_coef
    assert g is not None and g.numel() == prob.nq
    # sum_q c_q g_q = -(p - p_t) . p  (A(alpha c) = alpha A(c))
    cq = dev(oracle.coef_qp(m, phi))
    lhs = float((cq * g).sum())
    rhs = -float(((p - pt) * p).sum())
    assert abs(lhs - rhs) < 1e-9 * abs(rhs)

    def Jof(f):
        prob.set_phi(dev(f))
        x, _ = prob.cg_solve(b, rtol=1e-13)
        return 0.5 * float(((x - pt) ** 2).sum())

    nodes = W.fd_nodes(m, count=32, seed=4)
    say("c4 48^3 finite differences at 32 nodes")
    scale = np.abs(gphi).max()
    for j in nodes:
        h = 1e-6
        fp, fm = phi.copy(), phi.copy()
        fp[j] += h
        fm[j] -= h
        fd = (Jof(fp) - Jof(fm)) / (2 * h)
        assert abs(fd - gphi[j]) <= 1e-5 * scale + 1e-6 * abs(fd), (j, fd, gphi[j])
