"""SBD_IO_SORTED: f read and q written in the plan's sorted order give the same q as the
user-order apply, permuted (single set and two sets, real and complex data, FP32 and FP64
far field); GMRES, which iterates in sorted order, is covered by test_gpu_gmres.py."""
import numpy as np
import pytest

import synth
from gpu_util import device, lib, rel_l2

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("case", ["square_fp32", "square_fp64", "helmholtz_fp32", "two_sets_fp64"])
def test_sorted_io_matches_user_order(case):
    import torch
    from paper_1711_07877_amd import SBD_ARR_PERM, SBD_ARR_TPERM
    pkg = lib()
    n = 30000
    print(f"sorted io {case}", flush=True)
    z = torch.tensor(synth.square_points(n, 951), device=device())
    if case == "helmholtz_fp32":
        z = torch.tensor(synth.star_points(n, 952), device=device())
        plan = pkg.sbd_plan(z, kind=pkg.SBD_HELMHOLTZ, wavenumber=50.0, eps=1e-4, max_rhs=2)
        f = synth.complex_rhs(n, 953, nrhs=2)
    elif case == "two_sets_fp64":
        t = torch.tensor(synth.square_points(20000, 954), device=device())
        plan = pkg.sbd_plan_targets(t, z, eps=1e-6, precision=1)
        f = synth.real_rhs(n, 955)
    else:
        plan = pkg.sbd_plan(z, eps=1e-6 if case.endswith("64") else 1e-3, precision=1 if case.endswith("64") else 0)
        f = synth.real_rhs(n, 956)
    perm = plan.export(SBD_ARR_PERM)
    tperm = plan.export(SBD_ARR_TPERM) if case == "two_sets_fp64" else perm
    ft = torch.tensor(np.atleast_2d(f), device=device())
    q_user = plan.apply(ft).cpu().numpy()
    fs = torch.tensor(np.atleast_2d(f)[:, perm].copy(), device=device())
    q_sorted = plan.apply(fs, sorted_io=True).cpu().numpy()
    torch.cuda.synchronize()
    d = rel_l2(q_sorted, q_user[:, tperm])
    print(f"  rel l2 (sorted vs user order, permuted) {d:.2e}", flush=True)
    assert d < 1e-12
    plan.free()
