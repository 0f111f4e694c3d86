"""The SBD algorithm of Section 1 with exact exponential sums for the NUFFTs.

Off-line part (Section 1): geometry, sparse spectrum sampling (SBD fit, then
circular quadrature), pair set and D.  On-line part: f_hat = NUFFT_-(f),
g_hat = omega_hat * f_hat, q_far = NUFFT_+(g_hat) (eq. "far convolution",
Section 6.2 steps (i)-(iii)), q_close = D f, q = q_far + q_close.

Here each NUFFT is the plain sum it stands for:
  f_hat_nu = sum_l exp(-i (z_l - c) . xi_nu) f_l,
  q_far_k  = sum_nu exp(+i (z_k - c) . xi_nu) omega_hat_nu f_hat_nu + omega_hat_0 sum_l f_l,
cost N * N_xi, so it is meant for N up to about 1e5.

Readings taken:
* Geometry: c is the bounding-box centre and delta_max = 2 max |z_k - c|
  (an upper bound of the diameter that Section 6.1 uses; deterministic).
* Scaling: the paper's "J0(delta_max rho_p r)" is read as J0(rho_p r/delta_max),
  and G(delta_max) becomes a node at xi = 0 with weight -(1/2 pi) log delta_max.
* Normalisation: Laplace G = -(1/2 pi) log r, so the circle weights are
  -(1/2 pi) alpha_p C_p / M_p; Helmholtz G = (i/4) H0^(1)(k r): the Y0 circles
  carry -(1/4) beta_p C_p / M_p and the J0 circle of radius k carries (i/4)/M_0.
* Nodes xi_{p,m} = (rho_p lam / delta_max)(cos 2 pi m/M_p, sin 2 pi m/M_p), no
  angular offset (eq. "defXimp").
* delta_min: the "ten" rule uses delta_min^2 = 10 area / (pi N) (about ten
  neighbours for area-uniform points); the "curve" rule is Theorem 1's
  a = |log eps|^(2/3) / N^(2/3) (alpha = 0, natural log) for points on curves.
"""
from __future__ import annotations

import math
import numpy as np

from .sbd_fit import fit_laplace, fit_helmholtz, circle_sizes
from .nearfield import near_pairs, near_values


def geometry(z):
    z = np.asarray(z, dtype=np.float64)
    lo = z.min(axis=0)
    hi = z.max(axis=0)
    c = 0.5 * (lo + hi)
    dmax = 2.0 * float(np.max(np.hypot(z[:, 0] - c[0], z[:, 1] - c[1])))
    return c, dmax


def default_delta_min(z, rule, eps, area=None):
    n = len(z)
    if rule == "ten":
        return math.sqrt(10.0 * area / (math.pi * n))
    if rule == "curve":
        _, dmax = geometry(z)
        return abs(math.log(eps)) ** (2.0 / 3.0) / n ** (2.0 / 3.0) * dmax
    return float(rule)


def frequencies(fit, delta_max, kind, eps, wavenumber=0.0):
    """Concentric-circle nodes xi [N_xi, 2] and weights omega_hat [N_xi]; plus omega_hat_0."""
    xs, ws = [], []
    cg = -1.0 / (2.0 * math.pi) if kind == "laplace" else -0.25
    for R, c, M in zip(fit.radii, fit.coef, fit.M):
        th = 2.0 * math.pi * np.arange(M) / M
        xs.append(np.stack([np.cos(th), np.sin(th)], axis=1) * (R / delta_max))
        ws.append(np.full(M, cg * c / M, dtype=np.complex128))
    w0 = 0.0
    if kind == "laplace":
        w0 = -math.log(delta_max) / (2.0 * math.pi)
    else:
        kap = wavenumber * delta_max
        M0 = int(circle_sizes(np.array([kap]), np.array([1.0]), eps, fit.P)[0])
        th = 2.0 * math.pi * np.arange(M0) / M0
        xs.append(np.stack([np.cos(th), np.sin(th)], axis=1) * wavenumber)
        ws.append(np.full(M0, 0.25j / M0))
    return np.concatenate(xs), np.concatenate(ws), w0


def far_exact(z, f, c, xi, w, w0, block=2048):
    """NUFFT_+(omega_hat * NUFFT_-(f)) by exact sums, blocked over frequencies."""
    zc = np.asarray(z, dtype=np.float64) - c
    q = np.zeros(f.shape, dtype=np.complex128)
    for s in range(0, len(xi), block):
        ph = zc @ xi[s:s + block].T                      # [N, B]
        E = np.exp(1j * ph)
        fh = f @ np.conj(E)                              # [nrhs, B]   (NUFFT_-)
        q += (fh * w[s:s + block][None, :]) @ E.T        # [nrhs, N]   (NUFFT_+)
    q += w0 * np.sum(f, axis=1, keepdims=True)
    return q


def sbd_oracle(z, f, kind="laplace", eps=1e-3, delta_min=None, wavenumber=0.0, P=None,
               return_parts=False):
    """q = q_far + D f for every row; f is [N] or [nrhs, N]."""
    z = np.asarray(z, dtype=np.float64)
    f = np.asarray(f)
    squeeze = f.ndim == 1
    f2 = (f[None, :] if squeeze else f).astype(np.complex128)
    c, dmax = geometry(z)
    a = delta_min / dmax
    if not (0.0 < a < 1.0):
        raise ValueError("need 0 < delta_min < delta_max")
    if kind == "laplace":
        fit = fit_laplace(a, eps, P=P)
    else:
        fit = fit_helmholtz(a, eps, wavenumber * dmax, P=P)
    xi, w, w0 = frequencies(fit, dmax, kind, eps, wavenumber)
    q_far = far_exact(z, f2, c, xi, w, w0)
    rows, cols = near_pairs(z, delta_min)
    vals = near_values(z, rows, cols, fit, dmax, kind, wavenumber)
    q_close = np.zeros_like(q_far)
    for r in range(f2.shape[0]):
        q_close[r] = np.bincount(rows, weights=(vals * f2[r, cols]).real, minlength=len(z)) + \
            1j * np.bincount(rows, weights=(vals * f2[r, cols]).imag, minlength=len(z))
    q = q_far + q_close
    if kind == "laplace" and not np.iscomplexobj(f):
        q, q_far, q_close = q.real, q_far.real, q_close.real
    if squeeze:
        q, q_far, q_close = q[0], q_far[0], q_close[0]
    if return_parts:
        return dict(q=q, q_far=q_far, q_close=q_close, fit=fit, xi=xi, w=w, w0=w0, c=c,
                    delta_max=dmax, delta_min=delta_min, nnz=len(rows))
    return q
