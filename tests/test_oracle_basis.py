"""Pins of the oracle's 1D tables: Gauss rule, GLL support points, Lagrange basis.

Quadrature: (k+1) Gauss points per direction (Sec. "Numerical framework").
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads
from indep import gauss01, gll_closed_form, lagrange_polys

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_gauss3_closed_form():
    g = json.load(open(os.path.join(GOLD, "gauss3.json")))
    x, w = oracle.gauss_rule(3)
    ref_x = [eval(s, {"sqrt": math.sqrt}) for s in g["points"]]
    ref_w = [eval(s) for s in g["weights"]]
    np.testing.assert_allclose(x, ref_x, rtol=0, atol=1e-15)
    np.testing.assert_allclose(w, ref_w, rtol=0, atol=1e-15)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7])
def test_gauss_matches_library_and_is_exact(n):
    x, w = oracle.gauss_rule(n)
    rx, rw = gauss01(n)
    np.testing.assert_allclose(x, rx, rtol=0, atol=2e-15)
    np.testing.assert_allclose(w, rw, rtol=0, atol=2e-15)
    for p in range(2 * n):           # exact for degree <= 2n-1
        assert abs(np.sum(w * x ** p) - 1.0 / (p + 1)) < 1e-14
    assert abs(np.sum(w * x ** (2 * n)) - 1.0 / (2 * n + 1)) > 1e-12   # and not beyond


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_gll_points(k):
    xi = oracle.gll_points(k)
    np.testing.assert_allclose(xi, gll_closed_form(k), rtol=0, atol=2e-15)
    # the input generators place nodes at the same points
    np.testing.assert_allclose(xi, workloads.support_points(k), rtol=0, atol=2e-15)


def test_gll_closed_forms():
    np.testing.assert_allclose(oracle.gll_points(3)[1:3],
                               [0.5 - math.sqrt(5) / 10, 0.5 + math.sqrt(5) / 10], atol=1e-15)
    np.testing.assert_allclose(oracle.gll_points(4)[1:4],
                               [0.5 - math.sqrt(21) / 14, 0.5, 0.5 + math.sqrt(21) / 14], atol=1e-15)


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_lagrange_basis(k):
    nodes = oracle.gll_points(k)
    polys = lagrange_polys(nodes)
    rng = np.random.default_rng(11)
    xs = np.concatenate([nodes, rng.uniform(0, 1, 9)])
    for x in xs:
        vals = [oracle.lagrange(k, nodes, a, x) for a in range(k + 1)]
        ders = [oracle.lagrange(k, nodes, a, x, deriv=True) for a in range(k + 1)]
        assert abs(sum(vals) - 1.0) < 1e-14           # partition of unity
        assert abs(sum(ders)) < 1e-12                 # derivative of a constant
        for a in range(k + 1):
            assert abs(vals[a] - polys[a](x)) < 1e-13
            assert abs(ders[a] - polys[a].deriv()(x)) < 1e-12
    for a in range(k + 1):
        for b in range(k + 1):
            assert abs(oracle.lagrange(k, nodes, a, nodes[b]) - (a == b)) < 1e-15
