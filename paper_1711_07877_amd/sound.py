"""Sound cancelling with SBD matvecs (Section 7, "Sound canceling").

N point sources z_l emit at one frequency with unit amplitude and phases phi_l.
The intensity at x is Pi(x, phi) = |sum_l H0(k |x - z_l|) exp(i phi_l)|^2, and the
phases are chosen to minimise its mean over Q quadrature points x_q of a silence
zone:

  J(phi) = (1/Q) |A u|^2,   A_ql = H0(k |x_q - z_l|),   u_l = exp(i phi_l).

The gradient is dJ/dphi_l = (2/Q) Re(conj(w_l) i u_l) with w = A^H (A u).  Both
products are two-set Helmholtz applies of the far part only (the zone is far from
the sources, so no pair is closer than delta_min and D is empty):

  A u       = -4i * apply[targets x, sources z](u)            (G = (i/4) H0)
  A^H v     = conj(-4i * apply[targets z, sources x](conj v))  (H0 is symmetric)

The optimiser is L-BFGS (scipy), stopped after a fixed number of objective and
gradient evaluations, as in the paper's experiment.

Readings (the paper fixes N = 100, sources at random spots on a half circle of
radius 0.5, k about 90, Q = 2.5e5 and 500 evaluations, and leaves the rest open):
the half circle is the upper one centred at the origin; the silence zone is the
disk of radius 0.2 centred at (0, -1); its quadrature points are area-uniform
random; the initial phases are uniform random.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np


@dataclass
class Scene:
    sources: np.ndarray        # [N, 2]
    zone: np.ndarray           # [Q, 2] quadrature points of the silence zone
    wavenumber: float
    zone_center: tuple
    zone_radius: float


def make_scene(n_sources: int = 100, q_points: int = 250_000, wavenumber: float = 90.0, seed: int = 7,
               zone_center=(0.0, -1.0), zone_radius: float = 0.2) -> Scene:
    rng = np.random.default_rng(seed)
    th = np.sort(rng.uniform(0.0, math.pi, n_sources))
    z = 0.5 * np.stack([np.cos(th), np.sin(th)], axis=1)
    r = zone_radius * np.sqrt(rng.uniform(0.0, 1.0, q_points))
    a = rng.uniform(0.0, 2.0 * math.pi, q_points)
    x = np.stack([zone_center[0] + r * np.cos(a), zone_center[1] + r * np.sin(a)], axis=1)
    return Scene(z, x, float(wavenumber), tuple(zone_center), float(zone_radius))


def objective_and_gradient(forward, adjoint, phi: np.ndarray):
    """J(phi) and dJ/dphi given forward(u) = A u and adjoint(v) = A^H v (host arrays)."""
    u = np.exp(1j * phi)
    v = forward(u)
    q = v.shape[0]
    J = float(np.vdot(v, v).real) / q
    w = adjoint(v)
    grad = (2.0 / q) * np.real(np.conj(w) * 1j * u)
    return J, grad


class SoundProblem:
    """The two far-only two-set plans of a scene (FP64 far field)."""

    def __init__(self, scene: Scene, eps: float = 1e-6, precision: int = 1):
        import torch
        import paper_1711_07877_amd as sbd
        self.sbd, self.torch = sbd, torch
        self.scene = scene
        dev = torch.device("cuda:0")
        self.dev = dev
        z, x = scene.sources, scene.zone
        # closest source-to-zone distance, from the zone's disk
        dist = np.hypot(z[:, 0] - scene.zone_center[0], z[:, 1] - scene.zone_center[1]) - scene.zone_radius
        if dist.min() <= 0:
            raise ValueError("the silence zone must not contain a source")
        # any delta_min below the gap leaves D empty; at most one wavelength keeps the fit
        # order P >= k delta_max / pi (needed to resolve the oscillation) inside the
        # well-conditioned range P <= 6 / a of the Fourier-Bessel basis on [a, 1]
        self.delta_min = min(0.5 * float(dist.min()), 2.0 * math.pi / scene.wavenumber)
        zt = torch.tensor(z, device=dev)
        xt = torch.tensor(x, device=dev)
        k = scene.wavenumber
        t0 = time.perf_counter()
        self.fwd = sbd.sbd_plan_targets(xt, zt, kind=sbd.SBD_HELMHOLTZ, wavenumber=k, eps=eps,
                                        delta_min=self.delta_min, precision=precision)
        self.adj = sbd.sbd_plan_targets(zt, xt, kind=sbd.SBD_HELMHOLTZ, wavenumber=k, eps=eps,
                                        delta_min=self.delta_min, precision=precision)
        torch.cuda.synchronize()
        self.plan_seconds = time.perf_counter() - t0
        if self.fwd.info()["nnz"] or self.adj.info()["nnz"]:
            raise ValueError("a source-zone pair is closer than delta_min")
        self.evaluations = 0

    def _apply(self, plan, f: np.ndarray) -> np.ndarray:
        torch = self.torch
        ft = torch.tensor(f.astype(np.complex128)[None, :], device=self.dev)
        q = plan.apply(ft, parts=self.sbd.SBD_PART_FAR)
        return q[0].cpu().numpy()

    def forward(self, u: np.ndarray) -> np.ndarray:
        return -4j * self._apply(self.fwd, u)

    def adjoint(self, v: np.ndarray) -> np.ndarray:
        return np.conj(-4j * self._apply(self.adj, np.conj(v)))

    def objective_and_gradient(self, phi: np.ndarray):
        self.evaluations += 1
        return objective_and_gradient(self.forward, self.adjoint, phi)

    def optimise(self, phi0: np.ndarray, max_evaluations: int = 500):
        from scipy.optimize import minimize
        J0 = self.objective_and_gradient(phi0)[0]
        t0 = time.perf_counter()
        res = minimize(self.objective_and_gradient, phi0, jac=True, method="L-BFGS-B",
                       options={"maxfun": max_evaluations, "maxiter": max_evaluations})
        secs = time.perf_counter() - t0
        return res.x, J0, float(res.fun), secs, int(res.nfev)

    def free(self):
        self.fwd.free()
        self.adj.free()


def run(sources: int = 100, q: int = 250_000, k: float = 90.0, evaluations: int = 500, grid: int = 4472,
        seed: int = 7) -> dict:
    """The experiment: optimise the phases, then evaluate the resulting field on a
    grid x grid image (4472^2 = 2e7 points, the paper's image size).  Returns the
    intensity in the zone before and after (dB), evaluations and times."""
    import torch
    import paper_1711_07877_amd as sbd
    scene = make_scene(sources, q, k, seed)
    prob = SoundProblem(scene)
    phi0 = np.random.default_rng(seed + 1).uniform(0.0, 2.0 * math.pi, sources)
    phi, J0, J1, secs, nfev = prob.optimise(phi0, evaluations)
    out = {"sources": sources, "zone_points": q, "wavenumber": k, "max_evaluations": evaluations,
           "plan_seconds": round(prob.plan_seconds, 3), "evaluations": nfev, "optimise_seconds": round(secs, 3),
           "ms_per_evaluation": round(1e3 * secs / max(1, nfev), 3),
           "zone_intensity_before": J0, "zone_intensity_after": J1,
           "reduction_db": round(10.0 * math.log10(J0 / J1), 2)}
    prob.free()
    # the resulting field on a square grid around sources and zone: every grid point is a
    # target, and grid points next to a source (closer than delta_min) are corrected by D
    if grid > 0:
        g = np.linspace(-1.5, 1.5, grid)
        gx, gy = np.meshgrid(g, g)
        pts = torch.tensor(np.stack([gx.ravel(), gy.ravel()], axis=1), device="cuda:0")
        zt = torch.tensor(scene.sources, device="cuda:0")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan = sbd.sbd_plan_targets(pts, zt, kind=sbd.SBD_HELMHOLTZ, wavenumber=k, eps=1e-4,
                                    delta_min=2.0 * 3.0 / grid)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        u = torch.tensor(np.exp(1j * phi)[None, :], device="cuda:0")
        field = plan.apply(u)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        inside = torch.tensor(((gx.ravel() - scene.zone_center[0]) ** 2 + (gy.ravel() - scene.zone_center[1]) ** 2
                               <= scene.zone_radius ** 2), device="cuda:0")
        level = (4.0 * field[0].abs()) ** 2
        out["field_points"] = int(pts.shape[0])
        out["field_plan_seconds"] = round(t1 - t0, 3)
        out["field_apply_ms"] = round(1e3 * (t2 - t1), 3)
        out["field_mean_db_inside_zone"] = round(10.0 * math.log10(float(level[inside].mean())), 2)
        out["field_median_db_outside_zone"] = round(10.0 * math.log10(float(level[~inside].median())), 2)
        plan.free()
        del pts, u, field, inside, level
        torch.cuda.empty_cache()
    return out


def main(argv=None):
    """Run the experiment and print one JSON line."""
    import argparse
    import json
    ap = argparse.ArgumentParser()
    ap.add_argument("--sources", type=int, default=100)
    ap.add_argument("--q", type=int, default=250_000)
    ap.add_argument("--k", type=float, default=90.0)
    ap.add_argument("--evaluations", type=int, default=500)
    ap.add_argument("--grid", type=int, default=4472, help="field image: grid x grid points (4472^2 = 2e7)")
    ap.add_argument("--seed", type=int, default=7)
    args = ap.parse_args(argv)
    print(json.dumps(run(args.sources, args.q, args.k, args.evaluations, args.grid, args.seed)), flush=True)


if __name__ == "__main__":
    main()
