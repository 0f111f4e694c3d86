"""GMRES on the SBD operator (single-layer system on a closed curve) against the
FP64 direct sum: the returned x must solve the exact dense system to the
solver tolerance plus the SBD error bound."""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_util import device, lib

pytestmark = pytest.mark.gpu


def _system(n, seed):
    z = synth.serving_curve(n, seed)
    w = synth.curve_weights(z)
    # self panel: integral of -(1/2 pi) log|s| over |s| <= w/2
    d = -w / (2 * math.pi) * (np.log(w / 2) - 1.0)
    b = -np.log(np.hypot(z[:, 0] - 2.0, z[:, 1] - 2.0)) / (2 * math.pi)
    return z, w, d, b


def _exact_residual(z, w, d, b, x):
    ax = oracle.direct_sum(z, w * x) + d * x
    return np.linalg.norm(ax - b) / np.linalg.norm(b)


@pytest.mark.parametrize("eps,precision", [(1e-6, 1), (1e-3, 0)])
def test_gmres_solves_exact_system(eps, precision):
    import torch
    pkg = lib()
    dev = device()
    z, w, d, b = _system(3000, 11)
    print(f"gmres n=3000 eps={eps} precision={precision}", flush=True)
    plan = pkg.sbd_plan(torch.tensor(z, device=dev), eps=eps, precision=precision)
    bt, wt, dt = (torch.tensor(v, device=dev) for v in (b, w, d))
    rtol = 1e-6 if precision else 1e-5
    x, its, rel = plan.gmres(bt, weights=wt, diag=dt, rtol=rtol)
    x = x.cpu().numpy()
    assert rel <= rtol and 0 < its <= 60
    # |A_exact x - A_sbd x|_k <= 1.1 eps/(2 pi) sum |w x| per row (off-diagonal part only)
    model = 1.1 * eps / (2 * math.pi) * np.abs(w * x).sum() * math.sqrt(len(x)) / np.linalg.norm(b)
    assert _exact_residual(z, w, d, b, x) <= rtol * 1.01 + model
    plan.free()


def test_gmres_restart_and_initial_guess():
    import torch
    pkg = lib()
    dev = device()
    z, w, d, b = _system(2000, 12)
    print("gmres restart n=2000", flush=True)
    plan = pkg.sbd_plan(torch.tensor(z, device=dev), eps=1e-6, precision=1)
    bt, wt, dt = (torch.tensor(v, device=dev) for v in (b, w, d))
    x1, its1, rel1 = plan.gmres(bt, weights=wt, diag=dt, restart=4, max_restarts=50, rtol=1e-8)
    x2, its2, rel2 = plan.gmres(bt, weights=wt, diag=dt, restart=30, rtol=1e-8)
    assert rel1 <= 1e-8 and rel2 <= 1e-8 and its1 >= its2
    x1 = x1.cpu().numpy()
    x2h = x2.cpu().numpy()
    assert np.linalg.norm(x1 - x2h) <= 1e-5 * np.linalg.norm(x2h)
    # starting from the solution: converged at the first residual check
    x3, its3, rel3 = plan.gmres(bt, x=x2.clone(), weights=wt, diag=dt, rtol=2e-8)
    assert its3 == 0 and rel3 <= 2e-8
    # a cycle cap below what is needed reports SBD_ENOCONV
    with pytest.raises(pkg.SbdError):
        plan.gmres(bt, weights=wt, diag=dt, restart=1, max_restarts=1, rtol=1e-12)
    plan.free()


def test_gmres_rejects_helmholtz():
    import torch
    pkg = lib()
    dev = device()
    z = synth.serving_curve(500, 3)
    plan = pkg.sbd_plan(torch.tensor(z, device=dev), kind=pkg.SBD_HELMHOLTZ, wavenumber=20.0, eps=1e-4)
    b = torch.ones(500, dtype=torch.float64, device=dev)
    with pytest.raises(pkg.SbdError):
        plan.gmres(b)
    plan.free()


def test_gmres_general_kernel():
    """GMRES through a general-kernel plan (Section 4.3): single-layer log plus a smooth
    oscillating part, against the exact dense residual of the same kernel."""
    import torch
    pkg = lib()
    dev = device()
    z, w, d, b = _system(2500, 13)
    c_log, terms = -1.0 / (2 * math.pi), [(0, 3.0, 0.05, 0.0)]       # -(1/2 pi) log r + 0.05 sin 3r
    eps = 1e-6
    print("gmres general kernel n=2500", flush=True)
    plan = pkg.sbd_plan(torch.tensor(z, device=dev), kind=pkg.SBD_GENERAL, eps=eps, precision=1,
                        general=pkg.general_kernel(c_log, terms, 1))
    bt, wt, dt = (torch.tensor(v, device=dev) for v in (b, w, d))
    x, its, rel = plan.gmres(bt, weights=wt, diag=dt, rtol=1e-7)
    plan.free()
    x = x.cpu().numpy()
    assert rel <= 1e-7 and its > 0
    ax = oracle.direct_sum_general(z, w * x, c_log, terms) + d * x
    model = 1.1 * eps * np.abs(w * x).sum() * math.sqrt(len(x)) / np.linalg.norm(b)
    assert np.linalg.norm(ax - b) / np.linalg.norm(b) <= 1e-7 * 1.01 + model
