"""Pins for the general-kernel SBD with the multi-Dirichlet condition enforced
(Section 4.3): exact iterated Laplacians against hand-derived values, the enforced
kernel's Laplacian vanishing at r = 1 by finite differences, the general fit reducing
to the closed-form Laplace fit, and the two claims of the section's figures."""
import math

import numpy as np
import pytest
import scipy.special as sp

import oracle
from oracle import general as g


def test_laplacian_iterates_by_hand():
    G1 = g.TrigRadial(1.0, {(0, 1.0, "sin"): 1.0})                   # log r + sin r
    lam = g.laplacian_iterates_at_1(G1, 2)
    # -Delta sin r = sin r - cos r / r ; log r is harmonic
    assert lam[0] == pytest.approx(math.sin(1) - math.cos(1), rel=1e-14)
    c = 250.0
    G2 = g.TrigRadial(1.0, {(0, c, "sin"): 1.0})
    assert g.laplacian_iterates_at_1(G2, 1)[0] == pytest.approx(c * c * math.sin(c) - c * math.cos(c), rel=1e-12)
    Q = g.TrigRadial(0.0, {(2, 0.0, "cos"): 1.0})                   # r^2: Delta = 4
    assert np.allclose(g.laplacian_iterates_at_1(Q, 2), [-4.0, 0.0])


def test_enforced_kernel_has_vanishing_laplacian_at_the_circle():
    """(-Delta)(G - K) at r = 1 by a central-difference radial Laplacian of G - K."""
    G1 = g.TrigRadial(1.0, {(0, 1.0, "sin"): 1.0})
    lams = g.laplacian_iterates_at_1(G1, 3)
    om = g.choose_frequencies(lams, 1)
    mu = g.enforcement(lams, om)
    assert np.all(np.abs(sp.j1(om)) < 1e-13)                          # roots of J1
    H = lambda r: G1(r) - sp.j0(np.outer(np.atleast_1d(r), om)) @ mu
    h = 1e-3
    d2 = (H(1 + h) - 2 * H(1.0) + H(1 - h)) / h ** 2
    d1 = (H(1 + h) - H(1 - h)) / (2 * h)
    assert abs((d2 + d1)[0]) < 1e-5 and abs(lams[0]) > 0.1


def test_general_fit_reduces_to_the_laplace_fit():
    a, P = 0.05, 40
    fit = g.fit_general(g.TrigRadial(1.0, {}), a, P, 0)
    ref = oracle.fit_laplace(a, 1e-3, P=P)
    assert np.max(np.abs(fit.coef - ref.coef)) < 1e-10 * np.max(np.abs(ref.coef))
    assert abs(fit.const) < 1e-15


def test_enforcement_removes_the_stagnation_near_r_1():
    """Section 4.3 figure: log r + sin r with P = 10; at gamma = 3 the plain SBD
    stagnates while the enforced one keeps converging."""
    G1 = g.TrigRadial(1.0, {(0, 1.0, "sin"): 1.0})
    a = 0.3
    e0 = g.max_error(G1, g.fit_general(G1, a, 10, 0), a)
    e1 = g.max_error(G1, g.fit_general(G1, a, 10, 1), a)
    assert e1 < e0 / 5


def test_highly_oscillating_kernel_error_falls_with_n():
    """Section 4.3 figure: log x + sin(250 x) with 100 terms; the error stagnates without
    enforcement and falls with each enforced order n <= 3 (gamma = 6)."""
    G = g.TrigRadial(1.0, {(0, 250.0, "sin"): 1.0})
    a = 0.06
    e = [g.max_error(G, g.fit_general(G, a, 100, n), a) for n in range(4)]
    assert e[0] > 0.1
    assert e[0] > e[1] > e[2] > e[3]
    assert e[3] < 1e-5
