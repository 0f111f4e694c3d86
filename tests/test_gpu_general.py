"""General radial kernels with the multi-Dirichlet condition enforced (Section 4.3) on
the GPU, through the C ABI: q against the FP64 direct sum of the kernel's definition,
relative l2 error at most eps and |q_k - exact_k| <= 1.1 eps sum_l |f_l| (c_G = 1 for
SBD_GENERAL), in both precisions,
for one set and for targets/sources, and the argument checks of the kernel description."""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_util import device, direct_rows, lib, rel_l2

pytestmark = pytest.mark.gpu

SBD_EINVAL = -1

KERNELS = {
    "log_plus_sin": (1.0, [(0, 1.0, 1.0, 0.0)], 1),                       # log r + sin r
    "log_plus_sin60": (1.0, [(0, 60.0, 1.0, 0.0)], 2),                    # oscillating
    "mixed": (0.5, [(1, 7.0, 0.3, -0.2), (2, 3.0, 0.0, 1.0)], 3),
    "log_only": (-1.0 / (2.0 * math.pi), [], 0),                            # the Laplace kernel
}


def _t(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=device())


def _apply(plan, f, precision):
    import torch
    ft = torch.tensor(np.atleast_2d(f), device=device(), dtype=torch.float64 if precision else torch.float32)
    q = plan.apply(ft)
    torch.cuda.synchronize()
    return q[0].double().cpu().numpy()


@pytest.mark.parametrize("name", sorted(KERNELS))
@pytest.mark.parametrize("precision,eps", [(1, 1e-6), (0, 1e-3)])
def test_general_kernel_matches_direct_sum(name, precision, eps):
    pkg = lib()
    c_log, terms, enforce = KERNELS[name]
    n = 3001
    z = synth.square_points(n, 410)
    f = synth.real_rhs(n, 410)[0]
    print(f"general {name} precision={precision} eps={eps} n={n}", flush=True)
    plan = pkg.sbd_plan(_t(z), kind=pkg.SBD_GENERAL, eps=eps, delta_min=0.03, precision=precision,
                        general=pkg.general_kernel(c_log, terms, enforce))
    info = plan.info()
    assert info["kind"] == pkg.SBD_GENERAL and info["nnz"] > 0
    q = _apply(plan, f, precision)
    plan.free()
    exact = oracle.direct_sum_general(z, f, c_log, terms)
    err = rel_l2(q, exact)
    print(f"  rel l2 {err:.3e}", flush=True)
    assert err <= eps
    assert np.max(np.abs(q - exact)) <= 1.1 * eps * np.abs(f).sum()


def test_general_kernel_targets():
    pkg = lib()
    c_log, terms, enforce = KERNELS["log_plus_sin60"]
    rng = np.random.default_rng(411)
    y = rng.uniform(0, 1, (2000, 2))
    x = rng.uniform(0.2, 1.2, (1500, 2))
    f = rng.standard_normal(2000)
    eps = 1e-6
    plan = pkg.sbd_plan_targets(_t(x), _t(y), kind=pkg.SBD_GENERAL, eps=eps, delta_min=0.03, precision=1,
                                general=pkg.general_kernel(c_log, terms, enforce))
    q = _apply(plan, f, 1)
    plan.free()
    d = np.hypot(x[:, None, 0] - y[None, :, 0], x[:, None, 1] - y[None, :, 1])
    exact = oracle.general_kernel_values(d, c_log, terms) @ f
    assert rel_l2(q, exact) <= eps
    assert np.max(np.abs(q - exact)) <= 1.1 * eps * np.abs(f).sum()


def test_general_kernel_argument_checks():
    pkg = lib()
    z = _t(synth.square_points(400, 412))

    def status(general):
        with pytest.raises(pkg.SbdError) as e:
            pkg.sbd_plan(z, kind=pkg.SBD_GENERAL, eps=1e-3, delta_min=0.05, general=general)
        return e.value.status

    assert status(pkg.general_kernel(1.0, [(0, 1.0, 1.0, 0.0)], 5)) == SBD_EINVAL          # enforce > 4
    assert status(pkg.general_kernel(1.0, [(1.5, 1.0, 1.0, 0.0)], 1)) == SBD_EINVAL        # m not an integer
    assert status(pkg.general_kernel(1.0, [(0, -2.0, 1.0, 0.0)], 1)) == SBD_EINVAL         # w < 0
    assert status(pkg.general_kernel(0.0, [], 0)) == SBD_EINVAL                            # G = 0
    assert status(pkg.general_kernel(1.0, [], 1)) == SBD_EINVAL                            # log r is harmonic
    assert status(pkg.general_kernel(1.0, [(0, 1.0, 1.0, 0.0)] * 9, 0)) == SBD_EINVAL      # > 8 terms


@pytest.mark.parametrize("precision,eps", [(0, 1e-3), (1, 1e-6)])
def test_general_kernel_full_size_sampled(precision, eps):
    """The bench leg's configuration (N = 1e6 uniform points, log r + sin 60r, order 2,
    two right-hand sides): sampled rows against the direct sum of the kernel's definition."""
    import torch
    pkg = lib()
    c_log, terms, enforce = KERNELS["log_plus_sin60"]
    n = 1_000_000
    z = synth.square_points(n, 413)
    f = np.stack([synth.real_rhs(n, 413)[0], synth.real_rhs(n, 414)[0]])
    print(f"general full size n={n} precision={precision}", flush=True)
    plan = pkg.sbd_plan(_t(z), kind=pkg.SBD_GENERAL, eps=eps, delta_min=math.sqrt(10.0 / (math.pi * n)),
                        precision=precision, max_rhs=2, general=pkg.general_kernel(c_log, terms, enforce))
    ft = torch.tensor(f, device=device(), dtype=torch.float64 if precision else torch.float32)
    q = plan.apply(ft)
    torch.cuda.synchronize()
    q = q.double().cpu().numpy()
    plan.free()
    rows = np.random.default_rng(415).integers(0, n, 1024)
    for j in range(2):
        exact = direct_rows(z, f[j], rows, general=(c_log, terms))
        err = rel_l2(q[j, rows], exact)
        print(f"  rhs {j}: rel l2 {err:.3e}", flush=True)
        assert err <= eps
        assert np.max(np.abs(q[j, rows] - exact)) <= 1.1 * eps * np.abs(f[j]).sum()
