"""SBD of a general radial kernel with the multi-Dirichlet condition enforced
(Section 4.3, "General kernel: enforcing the multi-Dirichlet condition").

TEST INFRASTRUCTURE ONLY (see the package docstring).

The error estimates of the Fourier-Bessel series (Section 2) need
(-Delta)^s G = 0 on the unit circle for s = 1..n.  For a kernel without this
property the SBD error stagnates near r = 1.  The paper subtracts
K(r) = sum_t mu_t J0(omega_t r), with omega_t roots of J1 near
omega' = sqrt(mean ratio of successive iterates (-Delta)^(s+1) G(1) / (-Delta)^s G(1)),
fits H = G - K by the SBD, and adds K back: every term is still a dilated J0,
so the circles of the far field simply gain n radii.

Readings taken:
* The conditions.  (-Delta)^s J0(omega r) = omega^(2s) J0(omega r), so
  (-Delta)^s (G - K)(1) = 0 for s = 1..n reads
  sum_t mu_t omega_t^(2s) J0(omega_t) = (-Delta)^s G(1).  The printed matrix M
  has entries (-1)^s omega_t^(2s) and no factor J0(omega_t): its sign pattern is
  that of Delta^s, and without J0(omega_t) the mu_t of the printed K would not
  satisfy the conditions; the condition itself is taken as the definition.
* The constant.  The Dirichlet basis vanishes at r = 1, so the fitted shape is
  H - H(1) and the constant H(1) is carried separately (for the far field it is
  the node xi = 0, as log delta_max is for Laplace).
* The right-hand side int_{A(a)} grad H . grad e_p has no closed form for a general
  kernel: Gauss-Legendre quadrature on [a, 1] with enough nodes for the
  oscillation of H.
* (-Delta)^s G(1) is computed exactly for kernels of the form
  c log r + sum_j r^m_j (A_j sin(w_j r) + B_j cos(w_j r)) by applying the radial
  Laplacian d2/dr2 + (1/r) d/dr term by term (Delta log r = 0 for r > 0).
"""
from __future__ import annotations

import math
from collections import defaultdict

import numpy as np
import scipy.special as sp

from .sbd_fit import bessel_basis, gram_matrix, fit_coefficients, check_grid


class TrigRadial:
    """f(r) = c_log log r + sum over terms (m, w, kind) -> coef of coef r^m sin/cos(w r)."""

    def __init__(self, c_log=0.0, terms=None):
        self.c_log = float(c_log)
        self.terms = defaultdict(float, terms or {})

    def d(self):
        out = defaultdict(float)
        for (m, w, kind), c in self.terms.items():
            if c == 0.0:
                continue
            if m != 0:
                out[(m - 1, w, kind)] += c * m
            if kind == "sin":
                out[(m, w, "cos")] += c * w
            else:
                out[(m, w, "sin")] -= c * w
        r = TrigRadial(0.0, out)
        if self.c_log:
            r.terms[(-1, 0.0, "cos")] += self.c_log       # d/dr log r = 1/r = r^-1 cos(0 r)
        return r

    def over_r(self):
        out = defaultdict(float)
        for (m, w, kind), c in self.terms.items():
            out[(m - 1, w, kind)] += c
        return TrigRadial(0.0, out)

    def laplacian(self):
        """Radial Laplacian f'' + f'/r (the log part is harmonic)."""
        d1 = self.d()
        d2 = d1.d()
        lap = TrigRadial(0.0, dict(d2.terms))
        for k, c in d1.over_r().terms.items():
            lap.terms[k] += c
        return lap

    def __call__(self, r):
        r = np.asarray(r, dtype=np.float64)
        v = self.c_log * np.log(r) if self.c_log else np.zeros_like(r)
        for (m, w, kind), c in self.terms.items():
            if c:
                v = v + c * r ** m * (np.sin(w * r) if kind == "sin" else np.cos(w * r))
        return v

    def derivative(self, r):
        return self.d()(r)


def laplacian_iterates_at_1(G: TrigRadial, n: int):
    """lambda_s = (-Delta)^s G at r = 1, s = 1..n."""
    out, f = [], G
    for _ in range(n):
        f = f.laplacian()
        f = TrigRadial(0.0, {k: -c for k, c in f.terms.items()})
        out.append(float(f(np.array([1.0]))[0]))
    return np.array(out)


def choose_frequencies(lams, n: int):
    """omega' from the mean ratio of successive iterates, then the n roots of J1
    closest to omega' (Section 4.3)."""
    if n == 0:
        return np.zeros(0)
    ratios = lams[1:] / lams[:-1] if len(lams) > 1 else np.array([abs(lams[0])])
    wp = math.sqrt(abs(float(np.mean(ratios))))
    z = sp.jn_zeros(1, int(wp / math.pi) + n + 4)
    return np.sort(z[np.argsort(np.abs(z - wp))[:n]])


def enforcement(lams, omegas):
    """mu with sum_t mu_t omega_t^(2s) J0(omega_t) = lambda_s, s = 1..n."""
    n = len(omegas)
    if n == 0:
        return np.zeros(0)
    M = np.array([[w ** (2 * s) * sp.j0(w) for w in omegas] for s in range(1, n + 1)])
    return np.linalg.solve(M, lams[:n])


class GeneralFit:
    def __init__(self, const, rho, coef, omegas, mu):
        self.const, self.rho, self.coef, self.omegas, self.mu = const, rho, coef, omegas, mu

    def __call__(self, s):
        s = np.asarray(s, dtype=np.float64)
        v = self.const + sp.j0(np.outer(s, self.rho)) @ self.coef
        if len(self.omegas):
            v = v + sp.j0(np.outer(s, self.omegas)) @ self.mu
        return v


def fit_general(G: TrigRadial, a: float, P: int, n: int, nquad: int = 4000):
    """SBD of order P of G on [a, 1] with the multi-Dirichlet condition enforced to order n."""
    lams = laplacian_iterates_at_1(G, max(n, 1) + 1)
    omegas = choose_frequencies(lams, n)
    mu = enforcement(lams, omegas)
    x, w = np.polynomial.legendre.leggauss(nquad)
    r = 0.5 * (1.0 - a) * x + 0.5 * (1.0 + a)
    w = 0.5 * (1.0 - a) * w
    dH = G.derivative(r)
    if n:
        dH = dH + (sp.j1(np.outer(r, omegas)) * omegas) @ mu          # -(d/dr) K
    rho, C = bessel_basis(P)
    de = -(C * rho)[:, None] * sp.j1(np.outer(rho, r))                  # e_p'(r)
    b = 2.0 * math.pi * de @ (r * w * dH)
    alpha = fit_coefficients(gram_matrix(rho, C, a), b)
    const = float(G(np.array([1.0]))[0]) - (float(sp.j0(omegas) @ mu) if n else 0.0)
    return GeneralFit(const, rho, alpha * C, omegas, mu)


def max_error(G: TrigRadial, fit: GeneralFit, a: float):
    s = np.concatenate([check_grid(a), np.linspace(a, 1.0, 20001)])
    return float(np.max(np.abs(fit(s) - G(s))))
