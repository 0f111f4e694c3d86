"""Fixed-radius pair set and close-correction values (Section 1, eq. "defD").

P = {(k, l) : |z_k - z_l| <= delta_min}, diagonal included.  The predicate is
evaluated exactly as d2 = (x_k - x_l)*(x_k - x_l) + (y_k - y_l)*(y_k - y_l) in
FP64 (two products, one sum, no fused multiply-add) against
delta_min * delta_min, so that the GPU index build can be compared bit for
bit.

Reading taken for D: eq. "defD" subtracts the NUFFT quadrature G_approx; here
D_kl = G(z_k - z_l) - G_SBD(|z_k - z_l|) with G_SBD the radial Bessel series
(the quadrature's limit), summed term by term.  Their difference on pairs
closer than delta_min is the circular-quadrature error, which the circle
sizes keep far below eps.  D_kk = -G_SBD(0) removes the self term that the
far field includes.
"""
import numpy as np
import scipy.special as sp
from scipy.spatial import cKDTree

from .kernels import laplace_kernel, helmholtz_kernel


def near_pairs(z, delta_min: float, brute: bool = False):
    """All (k, l) with d2 <= delta_min^2, diagonal included, sorted by (k, l)."""
    z = np.asarray(z, dtype=np.float64)
    n = len(z)
    d2max = delta_min * delta_min
    if brute:
        dx = z[:, 0][:, None] - z[:, 0][None, :]
        dy = z[:, 1][:, None] - z[:, 1][None, :]
        d2 = dx * dx + dy * dy
        k, l = np.nonzero(d2 <= d2max)
        return k, l
    tree = cKDTree(z)
    pr = tree.query_pairs(delta_min * (1.0 + 1e-9), output_type="ndarray")
    if len(pr):
        k = np.concatenate([pr[:, 0], pr[:, 1]])
        l = np.concatenate([pr[:, 1], pr[:, 0]])
        dx = z[k, 0] - z[l, 0]
        dy = z[k, 1] - z[l, 1]
        keep = (dx * dx + dy * dy) <= d2max
        k, l = k[keep], l[keep]
    else:
        k = l = np.zeros(0, dtype=np.int64)
    k = np.concatenate([k, np.arange(n)])
    l = np.concatenate([l, np.arange(n)])
    order = np.lexsort((l, k))
    return k[order], l[order]


def g_sbd(r, fit, delta_max, kind, wavenumber=0.0):
    """Radial SBD series G_SBD(r) (Section 1 sparse-spectrum step, un-scaled)."""
    r = np.asarray(r, dtype=np.float64)
    s = r / delta_max
    series = sp.j0(np.outer(s, fit.radii)) @ fit.coef
    if kind == "laplace":
        return -(1.0 / (2.0 * np.pi)) * (np.log(delta_max) + series)
    return -0.25 * series + 0.25j * sp.j0(wavenumber * r)


def near_values(z, rows, cols, fit, delta_max, kind, wavenumber=0.0):
    """D values on the pair list (rows, cols)."""
    z = np.asarray(z, dtype=np.float64)
    dx = z[rows, 0] - z[cols, 0]
    dy = z[rows, 1] - z[cols, 1]
    d2 = dx * dx + dy * dy
    diag = rows == cols
    d2s = np.where(diag, 1.0, d2)
    g = laplace_kernel(d2s) if kind == "laplace" else helmholtz_kernel(d2s, wavenumber)
    g = np.where(diag, 0.0, g)
    return g - g_sbd(np.sqrt(d2), fit, delta_max, kind, wavenumber)


def near_values_nufft(z, rows, cols, xi, w, w0, kind, wavenumber=0.0, block=4096):
    """D values on the pair list by the Section 1 assembly (eq. "defD"): for each pair
    the difference y = z_k - z_l, G(y) minus the sparse-spectrum sum
    sum_nu omega_hat_nu exp(i y . xi_nu) (+ omega_hat_0), written as the plain
    exponential sum over every circle node (the NUFFT_+ of the pair differences).
    xi, w, w0 as returned by the oracle's ``frequencies``.  Cost #pairs * N_xi."""
    z = np.asarray(z, dtype=np.float64)
    dx = z[rows, 0] - z[cols, 0]
    dy = z[rows, 1] - z[cols, 1]
    d2 = dx * dx + dy * dy
    diag = rows == cols
    d2s = np.where(diag, 1.0, d2)
    g = laplace_kernel(d2s) if kind == "laplace" else helmholtz_kernel(d2s, wavenumber)
    g = np.where(diag, 0.0, g).astype(np.complex128)
    yv = np.stack([dx, dy], axis=1)
    s = np.full(len(rows), w0, dtype=np.complex128)
    for b in range(0, len(xi), block):
        s += np.exp(1j * (yv @ xi[b:b + block].T)) @ w[b:b + block]
    return g - s


def near_pairs_targets(x, y, delta_min: float, brute: bool = False):
    """All (target k, source l) with d2 <= delta_min^2 (same predicate), sorted by (k, l)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    d2max = delta_min * delta_min
    if brute:
        dx = x[:, 0][:, None] - y[:, 0][None, :]
        dy = x[:, 1][:, None] - y[:, 1][None, :]
        return np.nonzero(dx * dx + dy * dy <= d2max)
    lists = cKDTree(x).query_ball_tree(cKDTree(y), delta_min * (1.0 + 1e-9))
    k = np.repeat(np.arange(len(x)), [len(li) for li in lists])
    l = np.concatenate([np.asarray(li, dtype=np.int64) for li in lists]) if len(k) else np.zeros(0, dtype=np.int64)
    dx = x[k, 0] - y[l, 0]
    dy = x[k, 1] - y[l, 1]
    keep = (dx * dx + dy * dy) <= d2max
    k, l = k[keep], l[keep]
    order = np.lexsort((l, k))
    return k[order], l[order]


def near_values_targets(x, y, rows, cols, fit, delta_max, kind, wavenumber=0.0):
    """D values G(x_k - y_l) - G_SBD(|x_k - y_l|) on a two-set pair list."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    dx = x[rows, 0] - y[cols, 0]
    dy = x[rows, 1] - y[cols, 1]
    d2 = dx * dx + dy * dy
    g = laplace_kernel(d2) if kind == "laplace" else helmholtz_kernel(d2, wavenumber)
    return g - g_sbd(np.sqrt(d2), fit, delta_max, kind, wavenumber)
