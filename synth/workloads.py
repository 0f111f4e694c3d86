"""Seeded point clouds and vectors (no SBD arithmetic lives here)."""
from __future__ import annotations

import math
import numpy as np


def disk_points(n: int, seed: int) -> np.ndarray:
    """Area-uniform points in the unit disk: r = sqrt(U1), t = 2 pi U2."""
    rng = np.random.default_rng(seed)
    u = rng.random((n, 2))
    r = np.sqrt(u[:, 0])
    t = 2.0 * math.pi * u[:, 1]
    return np.stack([r * np.cos(t), r * np.sin(t)], axis=1)


def square_points(n: int, seed: int) -> np.ndarray:
    """Points uniform in the unit square [0, 1]^2."""
    rng = np.random.default_rng(seed)
    return rng.random((n, 2))


def _sample_closed_curve(curve, n: int, rng, jitter: float, fine: int = 1 << 16) -> np.ndarray:
    """Arclength-uniform samples of a closed parametric curve t in [0, 2 pi).

    The arclength is tabulated on ``fine`` parameter values (piecewise-linear
    chord lengths); sample positions are equispaced in arclength from a random
    origin, each moved by U[-jitter, jitter] times the spacing.
    """
    t = np.linspace(0.0, 2.0 * math.pi, fine + 1)
    xy = curve(t)
    seg = np.hypot(np.diff(xy[0]), np.diff(xy[1]))
    s = np.concatenate([[0.0], np.cumsum(seg)])
    length = s[-1]
    spacing = length / n
    origin = rng.random() * length
    targets = origin + spacing * (np.arange(n) + jitter * (2.0 * rng.random(n) - 1.0))
    targets = np.mod(targets, length)
    tt = np.interp(targets, s, t)
    p = curve(tt)
    return np.stack([p[0], p[1]], axis=1)


def _ellipse(cx, cy, a, b, rot):
    c, s = math.cos(rot), math.sin(rot)

    def curve(t):
        x = a * np.cos(t)
        y = b * np.sin(t)
        return np.array([cx + c * x - s * y, cy + s * x + c * y])
    return curve


def _ellipse_perimeter(a, b, m=4096):
    t = np.linspace(0, 2 * math.pi, m + 1)
    return float(np.sum(np.hypot(np.diff(a * np.cos(t)), np.diff(b * np.sin(t)))))


def _inside(poly, pts):
    """Even-odd point-in-polygon test for many points."""
    x, y = poly[:, 0], poly[:, 1]
    xn, yn = np.roll(x, -1), np.roll(y, -1)
    px = pts[:, 0][:, None]
    py = pts[:, 1][:, None]
    cond = ((y[None, :] > py) != (yn[None, :] > py))
    with np.errstate(divide="ignore", invalid="ignore"):
        xint = x[None, :] + (py - y[None, :]) * (xn - x)[None, :] / (yn - y)[None, :]
    cross = cond & (px < xint)
    return (np.sum(cross, axis=1) % 2) == 1


def _segments_cross(p, q) -> bool:
    """Any proper intersection between edges of closed polygons p and q."""
    a0, a1 = p, np.roll(p, -1, axis=0)
    b0, b1 = q, np.roll(q, -1, axis=0)

    def orient(o, u, v):
        return (u[..., 0] - o[..., 0]) * (v[..., 1] - o[..., 1]) - (u[..., 1] - o[..., 1]) * (v[..., 0] - o[..., 0])
    A0, A1 = a0[:, None, :], a1[:, None, :]
    B0, B1 = b0[None, :, :], b1[None, :, :]
    d1 = orient(A0, A1, B0)
    d2 = orient(A0, A1, B1)
    d3 = orient(B0, B1, A0)
    d4 = orient(B0, B1, A1)
    return bool(np.any((d1 * d2 < 0) & (d3 * d4 < 0)))


def ellipse_points(n: int, seed: int, count: int = 3, jitter: float = 0.01):
    """Points on ``count`` disjoint, non-nested ellipses in the unit square.

    Semi-axes U[0.1, 0.3], centres U(unit square), rotations U[0, pi).  Ellipse
    triples are redrawn until every pair is disjoint and non-nested (tested on
    512-gons, which is conservative enough at these sizes because rejection
    also requires a 2e-3 clearance).  Points are split in proportion to the
    perimeters and placed uniformly in arclength with a tangential jitter of
    U[-jitter, jitter] times the local spacing.
    """
    rng = np.random.default_rng(seed)
    while True:
        params = []
        for _ in range(count):
            a, b = rng.uniform(0.1, 0.3, size=2)
            cx, cy = rng.random(2)
            rot = rng.uniform(0.0, math.pi)
            params.append((cx, cy, a, b, rot))
        polys = []
        for (cx, cy, a, b, rot) in params:
            t = np.linspace(0, 2 * math.pi, 512, endpoint=False)
            polys.append(_ellipse(cx, cy, a * 1.01, b * 1.01, rot)(t).T)
        ok = True
        for i in range(count):
            for j in range(i + 1, count):
                if _segments_cross(polys[i], polys[j]):
                    ok = False
                elif _inside(polys[i], polys[j][:1]).any() or _inside(polys[j], polys[i][:1]).any():
                    ok = False
        if ok:
            break
    per = np.array([_ellipse_perimeter(p[2], p[3]) for p in params])
    counts = np.floor(n * per / per.sum()).astype(int)
    counts[: n - counts.sum()] += 1
    pts = [_sample_closed_curve(_ellipse(*p), int(m), rng, jitter) for p, m in zip(params, counts)]
    return np.concatenate(pts, axis=0), params


def star_points(n: int, seed: int, r0: float = 0.5, modes: int = 5, amp=0.02,
                relative: bool = False, jitter: float = 0.0):
    """Closed star-shaped curve sampled uniformly in arclength.

    r(t) = r0 + sum_{m=1..modes} A_m cos(m t + p_m) with p_m ~ U[0, 2 pi).
    If ``relative`` the amplitudes multiply r0 and A_m ~ U[0, amp] (serving
    stream curves), otherwise A_m = amp (perturbed-circle Helmholtz case).
    """
    rng = np.random.default_rng(seed)
    ph = rng.uniform(0.0, 2 * math.pi, size=modes)
    if relative:
        am = r0 * rng.uniform(0.0, amp, size=modes)
    else:
        am = np.full(modes, amp)

    def curve(t):
        t = np.asarray(t)
        r = r0 + sum(am[m] * np.cos((m + 1) * t + ph[m]) for m in range(modes))
        return np.array([r * np.cos(t), r * np.sin(t)])
    return _sample_closed_curve(curve, n, rng, jitter)


def serving_curve(n: int, seed: int) -> np.ndarray:
    """Serving-stream geometry: r(t) = 0.5 (1 + sum_{m<=4} a_m cos(m t + p_m)), a_m ~ U[0, 0.1]."""
    return star_points(n, seed, r0=0.5, modes=4, amp=0.1, relative=True)


def curve_weights(z: np.ndarray) -> np.ndarray:
    """Arclength quadrature weights of a closed polyline given in curve order:
    w_k = (|z_{k+1} - z_k| + |z_k - z_{k-1}|) / 2."""
    seg = np.hypot(*(np.roll(z, -1, axis=0) - z).T)
    return 0.5 * (seg + np.roll(seg, 1))


def real_rhs(n: int, seed: int, nrhs: int = 1) -> np.ndarray:
    """f ~ N(0, 1), shape [nrhs, n] (FP64)."""
    rng = np.random.default_rng(seed + 1000)
    return rng.standard_normal((nrhs, n))


def complex_rhs(n: int, seed: int, nrhs: int = 1) -> np.ndarray:
    """Complex f with independent N(0, 1) real and imaginary parts, shape [nrhs, n]."""
    rng = np.random.default_rng(seed + 2000)
    return rng.standard_normal((nrhs, n)) + 1j * rng.standard_normal((nrhs, n))


def request_stream(count: int, seed: int, nmin: float = 1e3, nmax: float = 1e6):
    """Serving stream: log-uniform N, star curve, eps in {1e-3, 1e-6}, apply or GMRES.

    Returns a list of dicts with keys: n, curve_seed, eps, kind ("apply"|"gmres"),
    gap (exponential inter-arrival draw with unit mean, to be scaled by the rate).
    """
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(round(10 ** rng.uniform(math.log10(nmin), math.log10(nmax))))
        out.append(dict(n=n, curve_seed=int(rng.integers(1 << 30)),
                        eps=float(rng.choice([1e-3, 1e-6])),
                        kind=str(rng.choice(["apply", "gmres"])),
                        gap=float(rng.exponential(1.0))))
    return out


# Named workloads (size, generator, tolerance).  delta_min: "ten" means
# delta_min^2 = 10 * area / (pi N) (about ten neighbours per point for
# area-uniform sets); "curve" means the curve rule of Theorem 1 with alpha = 0.
WORKLOADS = {
    "disk4k":      dict(n=4000, seed=1, gen="disk", eps=1e-3, kernel="laplace", delta_min="ten", area=math.pi),
    "ellipses1m":  dict(n=1_000_000, seed=2, gen="ellipses", eps=1e-6, kernel="laplace", delta_min="curve"),
    "square10m":   dict(n=10_000_000, seed=3, gen="square", eps=1e-3, kernel="laplace", delta_min="ten", area=1.0),
    "helmholtz200k": dict(n=200_000, seed=4, gen="star", eps=1e-4, kernel="helmholtz",
                          wavenumber=2 * math.pi * 50, nrhs=16, delta_min="curve"),
}


def make_workload(name: str, n: int | None = None, nrhs: int | None = None):
    """Return (points [n,2] FP64, f [nrhs,n], spec) for a named workload, optionally resized."""
    spec = dict(WORKLOADS[name])
    if n is not None:
        spec["n"] = n
    if nrhs is not None:
        spec["nrhs"] = nrhs
    n = spec["n"]
    seed = spec["seed"]
    gen = spec["gen"]
    if gen == "disk":
        z = disk_points(n, seed)
    elif gen == "square":
        z = square_points(n, seed)
    elif gen == "ellipses":
        z, _ = ellipse_points(n, seed)
    elif gen == "star":
        z = star_points(n, seed)
    else:
        raise ValueError(gen)
    k = spec.get("nrhs", 1)
    if spec["kernel"] == "helmholtz":
        f = complex_rhs(n, seed, k)
    else:
        f = real_rhs(n, seed, k)
    return z, f, spec
