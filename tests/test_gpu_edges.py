"""Edge cases of plan and apply on the GPU: the smallest inputs, ragged sizes,
degenerate geometry (collinear points; a dense cluster whose tile is split into
several work units and whose close rows take the long-row path), and every
documented error path (coincident points, non-finite coordinates, bad arguments),
each checked against the FP64 direct sum or the documented status."""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_util import device, lib, rel_l2

pytestmark = pytest.mark.gpu

SBD_EINVAL, SBD_EDUP = -1, -3


def _t(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=device())


def _apply(plan, f, parts=3):
    import torch
    ft = torch.tensor(np.atleast_2d(f), device=device())
    q = plan.apply(ft, parts=parts)
    torch.cuda.synchronize()
    return q.cpu().numpy()


def _laplace_bound(f, eps):
    return 1.1 * eps / (2 * math.pi) * np.abs(f).sum()


@pytest.mark.parametrize("n", [2, 3, 7])
@pytest.mark.parametrize("precision", [0, 1])
def test_tiny_point_sets(n, precision):
    rng = np.random.default_rng(100 + n)
    z = rng.uniform(0, 1, (n, 2))
    f = rng.standard_normal(n)
    eps = 1e-3
    print(f"tiny n={n} precision={precision}", flush=True)
    plan = lib().sbd_plan(_t(z), eps=eps, delta_min=0.02, precision=precision)
    q = _apply(plan, f)[0]
    qd = oracle.direct_sum(z, f)
    assert np.max(np.abs(q - qd)) <= _laplace_bound(f, eps)
    plan.free()


def test_one_target_one_source():
    x = np.array([[0.25, 0.75]])
    y = np.array([[0.6, 0.1]])
    f = np.array([1.7])
    plan = lib().sbd_plan_targets(_t(x), _t(y), eps=1e-5, delta_min=0.02, precision=1)
    q = _apply(plan, f)[0]
    exact = -math.log(math.hypot(0.25 - 0.6, 0.75 - 0.1)) / (2 * math.pi) * 1.7
    assert abs(q[0] - exact) <= 1.1e-5 / (2 * math.pi) * 1.7
    plan.free()


@pytest.mark.parametrize("n", [1023, 4097])
@pytest.mark.parametrize("precision", [0, 1])
def test_ragged_sizes(n, precision):
    z = synth.square_points(n, 200 + n)
    f = synth.real_rhs(n, 200 + n)[0]
    eps = 1e-3
    dmin = math.sqrt(10.0 / (math.pi * n))
    print(f"ragged n={n} precision={precision}", flush=True)
    plan = lib().sbd_plan(_t(z), eps=eps, delta_min=dmin, precision=precision)
    q = _apply(plan, f)[0]
    qd = oracle.direct_sum(z, f)
    assert rel_l2(q, qd) < eps and np.max(np.abs(q - qd)) <= _laplace_bound(f, eps)
    plan.free()


def test_collinear_points():
    """All points on one horizontal segment: a bounding box of zero height (one tile row)."""
    rng = np.random.default_rng(301)
    x = np.sort(rng.uniform(0, 1, 3000))
    z = np.stack([x, np.full_like(x, 0.3)], axis=1)
    f = rng.standard_normal(3000)
    eps = 1e-4
    plan = lib().sbd_plan(_t(z), eps=eps)
    assert plan.info()["nty"] == 1
    q = _apply(plan, f)[0]
    qd = oracle.direct_sum(z, f)
    assert np.max(np.abs(q - qd)) <= _laplace_bound(f, eps)
    plan.free()


@pytest.mark.parametrize("precision", [0, 1])
def test_dense_cluster(precision):
    """6000 points within 1e-3 of one spot plus 4000 spread ones: the cluster's tile holds
    more points than one work unit and its close rows (thousands of entries) take the
    long-row path of the interpolation kernel."""
    rng = np.random.default_rng(302)
    r = 1e-3 * np.sqrt(rng.uniform(0, 1, 6000))
    a = rng.uniform(0, 2 * math.pi, 6000)
    cl = np.stack([0.3 + r * np.cos(a), 0.3 + r * np.sin(a)], axis=1)
    z = np.concatenate([cl, rng.uniform(0, 1, (4000, 2))])
    f = rng.standard_normal(len(z))
    eps = 1e-3
    print(f"dense cluster precision={precision}", flush=True)
    plan = lib().sbd_plan(_t(z), eps=eps, delta_min=0.01, precision=precision)
    info = plan.info()
    assert info["nnz"] > 6000 * 6000
    q = _apply(plan, f)[0]
    qd = oracle.direct_sum(z, f)
    assert rel_l2(q, qd) < eps and np.max(np.abs(q - qd)) <= _laplace_bound(f, eps)
    plan.free()


def _status(fn):
    pkg = lib()
    with pytest.raises(pkg.SbdError) as e:
        fn()
    return e.value.status


def test_plan_error_paths():
    pkg = lib()
    z = synth.square_points(500, 303)
    # two distinct points at the same place
    zd = z.copy()
    zd[17] = zd[311]
    assert _status(lambda: pkg.sbd_plan(_t(zd), eps=1e-3, delta_min=0.05)) == SBD_EDUP
    # a target on a source
    assert _status(lambda: pkg.sbd_plan_targets(_t(z[:3]), _t(z), eps=1e-3, delta_min=0.05)) == SBD_EDUP
    # every point at one place (delta_max = 0)
    assert _status(lambda: pkg.sbd_plan(_t(np.tile([[0.2, 0.4]], (5, 1))), eps=1e-3)) == SBD_EINVAL
    # a NaN coordinate
    zn = z.copy()
    zn[42, 1] = np.nan
    assert _status(lambda: pkg.sbd_plan(_t(zn), eps=1e-3, delta_min=0.05)) == SBD_EINVAL
    # one point, eps out of range, delta_min >= delta_max, no wavenumber for Helmholtz
    assert _status(lambda: pkg.sbd_plan(_t(z[:1]), eps=1e-3)) == SBD_EINVAL
    assert _status(lambda: pkg.sbd_plan(_t(z), eps=0.0)) == SBD_EINVAL
    assert _status(lambda: pkg.sbd_plan(_t(z), eps=1e-3, delta_min=10.0)) == SBD_EINVAL
    assert _status(lambda: pkg.sbd_plan(_t(z), kind=pkg.SBD_HELMHOLTZ, eps=1e-3, wavenumber=0.0)) == SBD_EINVAL


def test_apply_error_paths():
    import torch
    pkg = lib()
    z = synth.square_points(500, 304)
    plan = pkg.sbd_plan(_t(z), eps=1e-3, delta_min=0.05, max_rhs=2)
    f3 = torch.zeros((3, 500), dtype=torch.float64, device=device())
    assert _status(lambda: plan.apply(f3)) == SBD_EINVAL                       # nrhs > max_rhs
    f1 = torch.zeros((1, 500), dtype=torch.float64, device=device())
    assert _status(lambda: plan.apply(f1, parts=0)) == SBD_EINVAL              # no part selected
    ws = torch.empty(16, dtype=torch.uint8, device=device())
    assert _status(lambda: plan.apply(f1, workspace=ws)) == SBD_EINVAL         # workspace too small
    plan.free()
    h = pkg.sbd_plan(_t(z), kind=pkg.SBD_HELMHOLTZ, wavenumber=20.0, eps=1e-3, delta_min=0.05)
    assert _status(lambda: h.apply(f1)) == SBD_EINVAL                          # Helmholtz needs complex data
    h.free()
