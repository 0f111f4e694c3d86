"""Sparse Bessel Decomposition fit, FP64 (Sections 2, 3, 4 and 5 of the paper).

Notation follows the paper: rho_p is the p-th positive zero of J0,
e_p(r) = C_p J0(rho_p r) with C_p = 1 / (sqrt(pi) rho_p |J1(rho_p)|)
(Section 2.1), a = delta_min / delta_max, gamma = P a.

The fit minimises Q^P (Section 3.1), the H^1 seminorm of the error on the
annulus A(a) = {a < |x| < 1}, by solving A^P alpha = b (Section 3.2) with
the explicit Gram matrix A^P.

Readings taken (each one also listed in the design notes):

* Off-diagonal sign of A^P.  Green's formula applied to two radial solutions
  u = J0(rho_i r), v = J0(rho_j r) of Bessel's equation gives
  int_a^1 r u' v' dr = rho_i rho_j [F_ji - F_ij]_a^1 / (rho_j^2 - rho_i^2)
  with F_ij(r) = rho_i r J0(rho_i r) J0'(rho_j r).  The printed Section 3.2
  formula has the bracket with the opposite sign; the derivation and a
  direct quadrature (see the tests) agree with the sign used here.
* Basis.  Eq. "LinearSystem" is written for the unnormalised J0 basis while
  A^P uses e_p; the normalised basis is used throughout and the coefficient
  of J0(rho_p s) is alpha_p C_p.
* Order search.  Section 1 asks for increasing P by dichotomy until the
  L-infinity error, monitored near delta_min, is below tolerance, without
  fixing a bracket or a grid.  Here: bisection on P in [ceil(1/a), ceil(6/a)]
  (Helmholtz: also P > kappa'/pi) for the smallest P whose maximum error on
  4096 points s_j = a (1/a)^((j/4095)^2) (clustered near a) is <= eps/2;
  monotonicity in P is assumed.  The upper end gamma = 6 sits just below the
  floor the Section 4.1 remark reports (error stagnating near 1e-10 from
  gamma ~ 6.7, A numerically indefinite near gamma ~ 7.5).
* Error budget.  eps/2 for the radial fit and eps/2 for the circular
  quadrature (Section 6.1: SBD to eps/2, then eq. "temp1").
* Circle sizes.  Eq. "temp1" asks |J0(rho_p|x|) - quadrature| <= eps /
  (2 P |alpha_p| C_p); Proposition "suboptCirc" gives a sufficient M_p with an
  unknown constant K.  Instead M_p is the smallest even M > x_p with
  2 (|J_M(x_p)| + |J_2M(x_p)|) <= eps / (2 P |alpha_p C_p|), which bounds the
  exact aliasing identity of Section 5 (J0 minus the M-point rule equals
  -sum_{k != 0} e^{i M k phi} J_{Mk}) for every |x| <= delta_max because
  |J_M(x_p t)| <= |J_M(x_p)| for t <= 1 < M / x_p.  Even M_p keeps the node
  set symmetric under x -> -x, so the Laplace G_approx is real.
* Helmholtz (Section 4.2).  kappa = k delta_max; kappa' is the smallest zero
  of Y0 that is >= kappa and lambda = kappa / kappa'.  h(t) = Y0(kappa' t) is
  fitted on [lambda a, 1] (Dirichlet at t = 1 at every order); then
  Y0(kappa s) = h(lambda s) ~ sum_p beta_p C_p J0(rho_p lambda s).  The J0 part
  of H0 is one exact circle of radius k.  The right-hand side b_p uses the
  same Green's formula with Y0(kappa' r) in place of one J0 (Section 3.2 notes
  the formulas hold for any value of rho).
* Helmholtz with kappa below the first zero y_{0,1} of Y0 (Section 4.2, third
  case; Robin conditions and Dini series, Section 2.3).  Rescaling to kappa'
  would shrink the fitted annulus to lambda a with lambda = kappa / y_{0,1}
  small, and lengthen the series.  Instead Y0(kappa s) is fitted on [a, 1]
  directly in the Dini basis e_p = C_p J0(rho_p s), rho_p the positive roots of
  r J0'(r) + H J0(r) = 0 with H = -kappa Y0'(kappa) / Y0(kappa) > 0, which
  Y0(kappa s) satisfies at every order since (-Delta)^n Y0(kappa s) =
  kappa^(2n) Y0(kappa s).  C_p normalises e_p in
  a_H(u, v) = int_B grad u . grad v + H int_C u v.  The quadratic form Q^P
  becomes the same a_H restricted to the annulus (the seminorm of Section 3.1
  plus H times the squared error on the unit circle, which pins the constant
  that the seminorm alone leaves free when e_p(1) != 0).  Its Gram matrix is
  the Section 3.2 formula (valid for any rho) plus 2 pi H e_i(1) e_j(1).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math
import numpy as np
import scipy.special as sp
from scipy.linalg import cho_factor, cho_solve
from scipy.optimize import brentq

NCHECK = 4096


def bessel_basis(P: int):
    """rho_p (first P zeros of J0) and C_p = 1/(sqrt(pi) rho_p |J1(rho_p)|) (Section 2.1)."""
    rho = sp.jn_zeros(0, P)
    C = 1.0 / (math.sqrt(math.pi) * rho * np.abs(sp.j1(rho)))
    return rho, C


def _F(rho_i, rho_j, r):
    """F_ij(r) = rho_i r J0(rho_i r) J0'(rho_j r), with J0' = -J1 (Section 3.2)."""
    return rho_i[:, None] * r * sp.j0(rho_i[:, None] * r) * (-sp.j1(rho_j[None, :] * r))


def _F_diag(rho, r):
    """F_i(r) = rho_i^2 r^2 [J0^2/2 + J0'^2/2] + rho_i r J0 J0' at argument rho_i r (Section 3.2)."""
    j0 = sp.j0(rho * r)
    j0p = -sp.j1(rho * r)
    return rho ** 2 * r ** 2 * (0.5 * j0 ** 2 + 0.5 * j0p ** 2) + rho * r * j0 * j0p


def gram_matrix(rho, C, a: float):
    """A^P_ij = int_{A(a)} grad e_i . grad e_j (Section 3.2), sign-corrected off the diagonal."""
    F1 = _F(rho, rho, 1.0)
    Fa = _F(rho, rho, a)
    ri = rho[:, None]
    rj = rho[None, :]
    P = len(rho)
    with np.errstate(divide="ignore", invalid="ignore"):
        A = (2.0 * math.pi * C[:, None] * C[None, :] * ri * rj / (rj ** 2 - ri ** 2)
             * ((F1.T - F1) - (Fa.T - Fa)))
    A[np.diag_indices(P)] = 2.0 * math.pi * C ** 2 * (_F_diag(rho, 1.0) - _F_diag(rho, a))
    return A


def rhs_laplace(rho, C, a: float):
    """b_p = int_{A(a)} grad(log|x|) . grad e_p = -2 pi C_p (J0(rho_p a) - J0(rho_p)); J0(rho_p) = 0."""
    return -2.0 * math.pi * C * sp.j0(rho * a)


def rhs_helmholtz(rho, C, a: float, kp: float):
    """b_p = int_{A(a)} grad Y0(kp|x|) . grad e_p via Green's formula (Section 3.2 pattern).

    With u = Y0(kp r), v = J0(rho_p r):
    int_a^1 r u' v' dr = [r (kp^2 u v' - rho_p^2 u' v)]_a^1 / (kp^2 - rho_p^2).
    """
    def g(r):
        u = sp.y0(kp * r)
        up = -kp * sp.y1(kp * r)
        v = sp.j0(rho * r)
        vp = -rho * sp.j1(rho * r)
        return r * (kp ** 2 * u * vp - rho ** 2 * up * v)
    return 2.0 * math.pi * C * (g(1.0) - g(a)) / (kp ** 2 - rho ** 2)


Y0_FIRST_ZERO = float(sp.yn_zeros(0, 1)[0])


def robin_constant(kappa: float) -> float:
    """H = -kappa Y0'(kappa) / Y0(kappa) = kappa Y1(kappa) / Y0(kappa) (Section 4.2); > 0 for kappa < y_{0,1}."""
    return float(kappa * sp.y1(kappa) / sp.y0(kappa))


def dini_roots(H: float, P: int):
    """First P positive roots of r J0'(r) + H J0(r) = H J0(r) - r J1(r) (Section 2.3 Theorem, H > 0).

    The function is H > 0 at 0 and equals -j J1(j) at each zero j of J0, whose sign
    alternates, so there is one root in (0, j_{0,1}) and one in each (j_{0,p-1}, j_{0,p})."""
    j = sp.jn_zeros(0, P)
    lo = np.concatenate([[0.0], j[:-1]])
    g = lambda r: H * sp.j0(r) - r * sp.j1(r)
    return np.array([brentq(g, l, h, xtol=1e-15, rtol=1e-15, maxiter=300) for l, h in zip(lo, j)])


def dini_basis(H: float, P: int):
    """rho_p (Dini roots) and C_p with a_H(e_p, e_p) = 1 on the unit disk B:
    a_H(e, e) = 2 pi C^2 [rho^2 int_0^1 r J1(rho r)^2 dr + H J0(rho)^2] and
    int_0^1 r J1(rho r)^2 dr = (J1(rho)^2 - J0(rho) J2(rho)) / 2 (Lommel)."""
    rho = dini_roots(H, P)
    q = rho ** 2 * 0.5 * (sp.j1(rho) ** 2 - sp.j0(rho) * sp.jv(2, rho)) + H * sp.j0(rho) ** 2
    C = 1.0 / np.sqrt(2.0 * math.pi * q)
    return rho, C


def gram_robin(rho, C, a: float, H: float):
    """int_{A(a)} grad e_i . grad e_j + 2 pi H e_i(1) e_j(1)."""
    e1 = C * sp.j0(rho)
    return gram_matrix(rho, C, a) + 2.0 * math.pi * H * np.outer(e1, e1)


def rhs_helmholtz_robin(rho, C, a: float, kappa: float, H: float):
    """int_{A(a)} grad Y0(kappa|x|) . grad e_p + 2 pi H Y0(kappa) e_p(1)."""
    return rhs_helmholtz(rho, C, a, kappa) + 2.0 * math.pi * H * sp.y0(kappa) * C * sp.j0(rho)


def fit_coefficients(A, b):
    """Solve A alpha = b by Cholesky (A is symmetric positive definite)."""
    return cho_solve(cho_factor(A), b)


def check_grid(a: float, n: int = NCHECK):
    """s_j = a (1/a)^((j/(n-1))^2), clustered near a where the error peaks (Section 1, Section 4.1 remark)."""
    return a * (1.0 / a) ** (np.linspace(0.0, 1.0, n) ** 2)


@dataclass
class SBDFit:
    kind: str                 # "laplace" or "helmholtz"
    a: float                  # annulus inner radius of the fitted shape
    P: int
    rho: np.ndarray           # J0 zeros rho_p
    C: np.ndarray
    alpha: np.ndarray         # coefficients on e_p
    lam: float = 1.0          # dilation of the J0 arguments (Helmholtz lambda)
    kappa: float = 0.0
    kappa_p: float = 0.0
    err: float = 0.0          # max error on the check grid
    M: np.ndarray = field(default=None)
    robin_H: float = 0.0      # > 0: Dini basis of the Robin condition with this H

    @property
    def coef(self):
        """Coefficient of J0(rho_p lam s): alpha_p C_p."""
        return self.alpha * self.C

    @property
    def radii(self):
        """Circle radii in unit-scaled frequency: rho_p lam."""
        return self.rho * self.lam


def _target(kind, t, kp):
    return np.log(t) if kind == "laplace" else sp.y0(kp * t)


def _fit_order(kind, P, a_fit, kp, H=None):
    if H is not None:  # Dini basis (Helmholtz, kappa below the first zero of Y0)
        rho, C = dini_basis(H, P)
        alpha = fit_coefficients(gram_robin(rho, C, a_fit, H), rhs_helmholtz_robin(rho, C, a_fit, kp, H))
        return rho, C, alpha
    rho, C = bessel_basis(P)
    A = gram_matrix(rho, C, a_fit)
    b = rhs_laplace(rho, C, a_fit) if kind == "laplace" else rhs_helmholtz(rho, C, a_fit, kp)
    alpha = fit_coefficients(A, b)
    return rho, C, alpha


def _max_error(kind, P, a_fit, kp, H=None):
    rho, C, alpha = _fit_order(kind, P, a_fit, kp, H)
    s = check_grid(a_fit)
    e = _target(kind, s, kp) - sp.j0(np.outer(s, rho)) @ (alpha * C)
    return float(np.max(np.abs(e)))


def choose_order(kind, a_fit, eps, kp=0.0, P=None, H=None):
    """Smallest P in the bracket with max check-grid error <= eps/2 (bisection)."""
    if P is not None:
        return int(P), _max_error(kind, int(P), a_fit, kp, H)
    lo = int(math.ceil(1.0 / a_fit))
    if kind == "helmholtz":
        lo = max(lo, int(math.ceil(kp / math.pi)) + 1)
    hi = max(lo, int(math.ceil(6.0 / a_fit)))
    ehi = _max_error(kind, hi, a_fit, kp, H)
    if ehi > eps / 2:
        raise ValueError(f"tolerance {eps} below the reachable SBD floor (error {ehi:.3e} at P={hi})")
    while lo < hi:
        mid = (lo + hi) // 2
        if _max_error(kind, mid, a_fit, kp, H) <= eps / 2:
            hi = mid
        else:
            lo = mid + 1
    return lo, _max_error(kind, lo, a_fit, kp, H)


def circle_sizes(x, coef, eps, P):
    """M_p: smallest even M > x_p with 2(|J_M(x_p)| + |J_2M(x_p)|) <= eps/(2 P |coef_p|) (Section 5, eq. temp1)."""
    out = np.empty(len(x), dtype=np.int64)
    for p, (xp, cp) in enumerate(zip(x, coef)):
        eta = eps / (2.0 * P * abs(cp)) if cp != 0 else np.inf
        M = int(math.floor(xp)) + 1
        M += M % 2
        while 2.0 * (abs(sp.jv(M, xp)) + abs(sp.jv(2 * M, xp))) > eta:
            M += 2
        out[p] = M
    return out


def fit_laplace(a: float, eps: float, P=None) -> SBDFit:
    """SBD of log s on [a, 1] (Section 4.1) plus circle sizes."""
    P, err = choose_order("laplace", a, eps, P=P)
    rho, C, alpha = _fit_order("laplace", P, a, 0.0)
    fit = SBDFit("laplace", a, P, rho, C, alpha, err=err)
    fit.M = circle_sizes(fit.radii, fit.coef, eps, P)
    return fit


def fit_helmholtz(a: float, eps: float, kappa: float, P=None, basis: str = "auto") -> SBDFit:
    """SBD of Y0(kappa s) on [a, 1] (Section 4.2): for kappa >= y_{0,1} (or basis
    "rescale") through h(t) = Y0(kappa' t) on [lambda a, 1]; for kappa < y_{0,1} (or
    basis "dini") directly in the Dini basis of the Robin condition H = -kappa Y0'/Y0."""
    if basis == "dini" or (basis == "auto" and kappa < Y0_FIRST_ZERO):
        H = robin_constant(kappa)
        if not H > 0:
            raise ValueError("the Dini basis needs kappa below the first zero of Y0")
        P, err = choose_order("helmholtz", a, eps, kp=kappa, P=P, H=H)
        rho, C, alpha = _fit_order("helmholtz", P, a, kappa, H)
        fit = SBDFit("helmholtz", a, P, rho, C, alpha, lam=1.0, kappa=kappa, kappa_p=kappa, err=err, robin_H=H)
        fit.M = circle_sizes(fit.radii, fit.coef, eps, P)
        return fit
    nz = int(kappa / math.pi) + 3
    yz = sp.yn_zeros(0, nz)
    kp = float(yz[np.searchsorted(yz, kappa)])
    lam = kappa / kp
    a_fit = lam * a
    P, err = choose_order("helmholtz", a_fit, eps, kp=kp, P=P)
    rho, C, alpha = _fit_order("helmholtz", P, a_fit, kp)
    fit = SBDFit("helmholtz", a_fit, P, rho, C, alpha, lam=lam, kappa=kappa, kappa_p=kp, err=err)
    fit.M = circle_sizes(fit.radii, fit.coef, eps, P)
    return fit
