"""The three close-part traversals of the interpolation kernel (flat runs of CSR
entries, the default; 16-lane row groups, pipelined; 16-lane row groups, plain) give
the same close correction to rounding, and each matches the oracle's D f, for short
rows (uniform points), long rows (a dense cluster) and complex data (Helmholtz)."""
import math
import os

import numpy as np
import pytest

import oracle
import synth
from gpu_util import device, lib, rel_l2

pytestmark = pytest.mark.gpu


def _near(plan, f, mode):
    import torch
    os.environ["SBD_NEAR_MODE"] = str(mode)
    try:
        ft = torch.tensor(np.atleast_2d(f), device=device())
        q = plan.apply(ft, parts=2)
        torch.cuda.synchronize()
    finally:
        del os.environ["SBD_NEAR_MODE"]
    return q.cpu().numpy()[0]


def _cases():
    rng = np.random.default_rng(401)
    r = 2e-3 * np.sqrt(rng.uniform(0, 1, 800))
    a = rng.uniform(0, 2 * math.pi, 800)
    cluster = np.concatenate([np.stack([0.4 + r * np.cos(a), 0.6 + r * np.sin(a)], axis=1),
                              rng.uniform(0, 1, (3000, 2))])
    return {
        "uniform": (synth.square_points(8000, 402), 0, 0.0, math.sqrt(10.0 / (math.pi * 8000)), 1e-4),
        "cluster": (cluster, 0, 0.0, 0.02, 1e-3),
        "helmholtz": (synth.star_points(4000, 403), 1, 40.0, 0.0, 1e-4),
    }


@pytest.mark.parametrize("name", ["uniform", "cluster", "helmholtz"])
@pytest.mark.parametrize("precision", [0, 1])
def test_close_part_traversals_agree(name, precision):
    import torch
    z, kind, k, dmin, eps = _cases()[name]
    n = len(z)
    f = synth.complex_rhs(n, 404)[0] if kind == 1 else synth.real_rhs(n, 404)[0]
    print(f"near modes {name} precision={precision}", flush=True)
    plan = lib().sbd_plan(torch.tensor(z, device=device()), kind=kind, wavenumber=k, eps=eps, delta_min=dmin,
                          precision=precision)
    outs = [_near(plan, f, m) for m in (2, 1, 0)]
    tol = 1e-6 if precision == 0 else 1e-13
    for o in outs[1:]:
        assert rel_l2(o, outs[0]) < tol
    # against the oracle's D f (pair set and D values with the plan's fit order)
    info = plan.info()
    a_ratio = info["delta_min"] / info["delta_max"]
    if kind == 0:
        fit = oracle.fit_laplace(a_ratio, eps, P=info["P"])
    else:
        fit = oracle.fit_helmholtz(a_ratio, eps, k * info["delta_max"], P=info["P"])
    rows, cols = oracle.near_pairs(z, info["delta_min"])
    vals = oracle.near_values(z, rows, cols, fit, info["delta_max"], "helmholtz" if kind else "laplace", k)
    prod = vals * f[cols]
    ref = np.bincount(rows, weights=prod.real, minlength=n) + 1j * np.bincount(rows, weights=prod.imag, minlength=n)
    if kind == 0:
        ref = ref.real
    assert rel_l2(outs[0], ref) < (1e-5 if precision == 0 else 1e-10)
    plan.free()
