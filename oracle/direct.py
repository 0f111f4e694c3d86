"""O(N^2) direct sum: the exact definition (Introduction, eq. "discreteConv").

q_k = sum_{l != k} G(z_k - z_l) f_l, and its two-set form
q_k = sum_l G(x_k - y_l) f_l with targets x and sources y (the setting of the
numerical experiments, Section 7), where no term is omitted.

Reading taken: the paper's sum includes l = k, where G is singular; the term
l = k is omitted (G(0) := 0).  Distinct coincident points are rejected.

Squared distances are formed as dx*dx + dy*dy in FP64 and each row is summed
with numpy's pairwise summation.
"""
import numpy as np

from .kernels import laplace_kernel, helmholtz_kernel


def _row_block(z, f, rows, kind, k):
    """Return q for the given row indices (all N sources)."""
    out = np.zeros((f.shape[0], len(rows)), dtype=np.complex128 if (kind == "helmholtz" or np.iscomplexobj(f)) else np.float64)
    x, y = z[:, 0], z[:, 1]
    for i, r in enumerate(rows):
        dx = x[r] - x
        dy = y[r] - y
        d2 = dx * dx + dy * dy
        d2[r] = 1.0
        if np.count_nonzero(d2 == 0.0):
            raise ValueError("coincident distinct points")
        g = laplace_kernel(d2) if kind == "laplace" else helmholtz_kernel(d2, k)
        g[r] = 0.0
        out[:, i] = np.sum(g[None, :] * f, axis=1)
    return out


def direct_sum(z, f, kind="laplace", wavenumber=0.0, rows=None):
    """Direct FP64 sum.

    z: [N, 2] FP64 points; f: [N] or [nrhs, N]; rows: optional row indices
    (all rows if None).  Returns q with the same leading shape as f,
    restricted to ``rows``.
    """
    z = np.asarray(z, dtype=np.float64)
    f = np.asarray(f)
    squeeze = f.ndim == 1
    f2 = f[None, :] if squeeze else f
    n = z.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    q = _row_block(z, f2, rows, kind, wavenumber)
    return q[0] if squeeze else q


def direct_sum_targets(x, y, f, kind="laplace", wavenumber=0.0, rows=None):
    """Direct FP64 two-set sum q_k = sum_l G(x_k - y_l) f_l.

    x: [M, 2] targets; y: [N, 2] sources; f: [N] or [nrhs, N]; rows: optional
    target indices.  A target that coincides with a source is rejected.
    """
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    f = np.asarray(f)
    squeeze = f.ndim == 1
    f2 = f[None, :] if squeeze else f
    rows = np.arange(len(x)) if rows is None else np.asarray(rows)
    cplx = kind == "helmholtz" or np.iscomplexobj(f2)
    out = np.zeros((f2.shape[0], len(rows)), dtype=np.complex128 if cplx else np.float64)
    for i, r in enumerate(rows):
        dx = x[r, 0] - y[:, 0]
        dy = x[r, 1] - y[:, 1]
        d2 = dx * dx + dy * dy
        if np.count_nonzero(d2 == 0.0):
            raise ValueError("a target coincides with a source")
        g = laplace_kernel(d2) if kind == "laplace" else helmholtz_kernel(d2, wavenumber)
        out[:, i] = np.sum(g[None, :] * f2, axis=1)
    return out[0] if squeeze else out


def general_kernel_values(r, c_log=0.0, terms=()):
    """G(r) = c_log log r + sum_j r^m_j (a_j sin(w_j r) + b_j cos(w_j r)) for r > 0 (the
    radial kernels of Section 4.3, e.g. log r + sin r), terms = [(m, w, a, b), ...]."""
    r = np.asarray(r, dtype=np.float64)
    v = c_log * np.log(r) if c_log else np.zeros_like(r)
    for m, w, a, b in terms:
        v = v + r ** m * (a * np.sin(w * r) + b * np.cos(w * r))
    return v


def direct_sum_general(z, f, c_log=0.0, terms=(), rows=None):
    """Direct FP64 sum q_k = sum_{l != k} G(|z_k - z_l|) f_l for a general radial kernel."""
    z = np.asarray(z, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    rows = np.arange(len(z)) if rows is None else np.asarray(rows)
    out = np.zeros(len(rows))
    for i, k in enumerate(rows):
        d = np.hypot(z[k, 0] - z[:, 0], z[k, 1] - z[:, 1])
        d[k] = 1.0                      # placeholder; the self term is dropped below
        g = general_kernel_values(d, c_log, terms)
        g[k] = 0.0
        out[i] = np.dot(g, f)
    return out
