"""Several right-hand sides in one apply (one pass over D for all of them, the sorted f copy
interleaved per point) give, right-hand side by right-hand side, the q of single applies
(real and complex data, FP32 and FP64 far field, two point sets); deterministic plans
repeat bit for bit."""
import math

import numpy as np
import pytest

import synth
from gpu_util import device, lib, rel_l2

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("case,nrhs", [("square_fp32", 4), ("square_fp64", 3), ("helmholtz_fp32", 5),
                                       ("two_sets_fp64", 2), ("curve_fp64_det", 8)])
def test_batched_rhs_match_single_applies(case, nrhs):
    import torch
    pkg = lib()
    print(f"multi rhs {case} nrhs={nrhs}", flush=True)
    n = 20000
    det = case.endswith("det")
    if case.startswith("helmholtz"):
        z = torch.tensor(synth.star_points(n, 971), device=device())
        plan = pkg.sbd_plan(z, kind=pkg.SBD_HELMHOLTZ, wavenumber=60.0, eps=1e-4, max_rhs=nrhs)
        f = torch.tensor(synth.complex_rhs(n, 972, nrhs=nrhs), device=device()).to(torch.complex64)
    elif case.startswith("two_sets"):
        z = torch.tensor(synth.square_points(n, 973), device=device())
        t = torch.tensor(synth.square_points(15000, 974), device=device())
        plan = pkg.sbd_plan_targets(t, z, eps=1e-6, precision=1, max_rhs=nrhs)
        f = torch.tensor(synth.real_rhs(n, 975, nrhs=nrhs), device=device())
    elif case.startswith("curve"):
        z = torch.tensor(synth.star_points(n, 976), device=device())
        plan = pkg.sbd_plan(z, eps=1e-6, precision=1, max_rhs=nrhs, deterministic=1)
        f = torch.tensor(synth.real_rhs(n, 977, nrhs=nrhs), device=device())
    else:
        z = torch.tensor(synth.square_points(n, 978), device=device())
        prec = 0 if case.endswith("fp32") else 1
        plan = pkg.sbd_plan(z, eps=1e-3 if prec == 0 else 1e-6, delta_min=math.sqrt(10.0 / (math.pi * n)),
                            precision=prec, max_rhs=nrhs)
        f = torch.tensor(synth.real_rhs(n, 979, nrhs=nrhs), device=device())
    qb = plan.apply(f).cpu().numpy()
    for r in range(nrhs):
        q1 = plan.apply(f[r:r + 1].contiguous()).cpu().numpy()[0]
        d = rel_l2(qb[r], q1)
        assert d < 1e-12, (r, d)
    if det:
        assert np.array_equal(plan.apply(f).cpu().numpy(), qb)
    torch.cuda.synchronize()
    plan.free()
