"""The library's host SBD fit (C++, compiled here with g++ on its own) against the
oracle's fit: the same order P (up to one), the same radial series to well within eps,
for Laplace, Helmholtz through kappa' rescaling, and Helmholtz in the Dini basis
(kappa below the first zero of Y0)."""
import json
import os
import subprocess
import time

import numpy as np
import pytest
import scipy.special as sp

from oracle import sbd_fit

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("hostfit") / "host_fit_driver")
    host = os.path.join(ROOT, "paper_1711_07877_amd", "csrc", "host")
    subprocess.run(["g++", "-O2", "-std=c++17", "-pthread", "-o", exe, os.path.join(ROOT, "tests", "host_fit_driver.cpp"),
                    os.path.join(host, "sbd_fit.cpp"), os.path.join(host, "bessel.cpp")], check=True)
    return exe


def _run(exe, kind, a, eps, kappa):
    out = subprocess.run([exe, str(kind), repr(a), repr(eps), repr(kappa)], check=True, capture_output=True, text=True)
    return json.loads(out.stdout)


@pytest.mark.parametrize("kind,a,eps,kappa", [
    (0, 0.05, 1e-3, 0.0), (0, 0.01, 1e-6, 0.0),
    (1, 0.05, 1e-4, 12.0),                      # kappa' rescaling
    (1, 0.05, 1e-4, 0.3), (1, 0.02, 1e-6, 0.05), (1, 0.05, 1e-3, 0.85),   # Dini basis
])
def test_host_fit_matches_oracle(driver, kind, a, eps, kappa):
    r = _run(driver, kind, a, eps, kappa)
    assert r["rc"] == 0
    if kind == 0:
        fit = sbd_fit.fit_laplace(a, eps)
        target = lambda s: np.log(s)
    else:
        fit = sbd_fit.fit_helmholtz(a, eps, kappa)
        target = lambda s: sp.y0(kappa * s)
        assert (r["robin_H"] > 0) == (kappa < sbd_fit.Y0_FIRST_ZERO)
        assert r["robin_H"] == pytest.approx(fit.robin_H, rel=1e-12, abs=0.0)
        assert r["lam"] == pytest.approx(fit.lam, rel=1e-14)
    assert abs(r["P"] - fit.P) <= 1
    n = min(r["P"], fit.P)
    assert np.allclose(np.array(r["radii"])[:n], fit.radii[:n], rtol=1e-12, atol=0)
    s = np.linspace(a, 1.0, 5001)
    lib_series = sp.j0(np.outer(s, r["radii"])) @ np.array(r["coef"])
    assert np.max(np.abs(lib_series - target(s))) <= 0.5 * eps
    assert np.max(np.abs(lib_series - sp.j0(np.outer(s, fit.radii)) @ fit.coef)) <= 0.5 * eps


def _run_general(exe, dmax, a, eps, c_log, enforce, terms):
    args = [exe, "general", repr(dmax), repr(a), repr(eps), repr(c_log), str(enforce)]
    args += [repr(float(v)) for t in terms for v in t]
    out = subprocess.run(args, check=True, capture_output=True, text=True)
    return json.loads(out.stdout)


GENERAL_CASES = [
    (1.0, 0.05, 1e-6, 1.0, 1, [(0, 1.0, 1.0, 0.0)]),                        # log r + sin r (Section 4.3)
    (1.0, 0.02, 1e-6, 1.0, 2, [(0, 250.0, 1.0, 0.0)]),                      # log r + sin(250 r)
    (1.4, 0.02, 1e-4, 0.5, 3, [(1, 7.0, 0.3, -0.2), (2, 3.0, 0.0, 1.0)]),    # mixed powers, delta_max != 1
    (2.0, 0.05, 1e-5, 0.0, 2, [(0, 4.0, 0.0, 1.0)]),                        # no log part
]


@pytest.mark.parametrize("dmax,a,eps,c_log,enforce,terms", GENERAL_CASES)
def test_host_general_fit(driver, dmax, a, eps, c_log, enforce, terms):
    """The general-kernel fit (Section 4.3): its series plus constant reproduces
    G(delta_max s) on [a, 1] within eps/2 (checked against the kernel's definition with
    scipy's Bessel functions), its enforced circles are the oracle's omega and mu, and at
    the same order it equals the oracle's fit."""
    from oracle import direct, general
    r = _run_general(driver, dmax, a, eps, c_log, enforce, terms)
    assert r["rc"] == 0 and r["n_enforced"] == enforce
    radii, coef = np.array(r["radii"]), np.array(r["coef"])
    s = np.linspace(a, 1.0, 20001)
    series = r["constant"] + sp.j0(np.outer(s, radii)) @ coef
    g = direct.general_kernel_values(dmax * s, c_log, terms)
    assert np.max(np.abs(series - g)) <= 0.55 * eps
    G = general.TrigRadial(c_log, {})
    for m, w, ca, cb in terms:
        G.terms[(m, w * dmax, "sin")] += ca * dmax ** m
        G.terms[(m, w * dmax, "cos")] += cb * dmax ** m
    lams = general.laplacian_iterates_at_1(G, max(enforce, 1) + 1)
    om = general.choose_frequencies(lams, enforce)
    mu = general.enforcement(lams, om)
    assert np.allclose(radii[len(radii) - enforce:], om, rtol=1e-12, atol=0)
    assert np.allclose(coef[len(coef) - enforce:], mu, rtol=1e-8, atol=0)
    # the same Galerkin system at the library's order, solved by the oracle with its own
    # quadrature of the right-hand side: the same series and coefficients
    fit = general.fit_general(G, a, r["P"] - enforce, enforce, nquad=8000)
    assert np.max(np.abs(series - (fit(s) + c_log * np.log(dmax)))) <= 1e-3 * eps
    nf = r["P"] - enforce
    assert np.max(np.abs(coef[:nf] - fit.coef)) <= 1e-7 * np.max(np.abs(fit.coef))


def test_host_general_enforcement_helps(driver):
    """Section 4.3: without the multi-Dirichlet condition the error of log r + sin(250 r)
    stagnates (the fit reports its floor at eps = 1e-6), while enforcing it to order 2
    reaches eps; for log r + sin r enforcement lowers the order P needed."""
    assert _run_general(driver, 1.0, 0.02, 1e-6, 1.0, 0, [(0, 250.0, 1.0, 0.0)])["rc"] == -4
    assert _run_general(driver, 1.0, 0.02, 1e-6, 1.0, 2, [(0, 250.0, 1.0, 0.0)])["rc"] == 0
    # a frequency the series cannot reach inside its conditioning range is refused at once
    t0 = time.perf_counter()
    assert _run_general(driver, 1.0, 0.02, 1e-3, 1.0, 2, [(0, 1e5, 1.0, 0.0)])["rc"] == -4
    assert time.perf_counter() - t0 < 2.0
    p0 = _run_general(driver, 1.0, 0.05, 1e-6, 1.0, 0, [(0, 1.0, 1.0, 0.0)])["P"]
    p1 = _run_general(driver, 1.0, 0.05, 1e-6, 1.0, 1, [(0, 1.0, 1.0, 0.0)])["P"] - 1
    assert p1 < 0.8 * p0
