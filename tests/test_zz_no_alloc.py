"""The allocation-free apply (sbd_apply_noalloc, static per-device scratch) against
sbd_apply with a caller workspace, through the C ABI: two calls in a row, the second on a
smaller plan, bit for bit on deterministic plans and to rounding on default ones; a plan
whose workspace exceeds the scratch is refused before any launch."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import device, lib, rel_l2

pytestmark = pytest.mark.gpu

SBD_ENOMEM = -2


def _t(a, dtype=None):
    import torch
    t = torch.tensor(np.ascontiguousarray(a), device=device())
    return t if dtype is None else t.to(dtype)


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_matches_workspace_apply(precision):
    import torch
    pkg = lib()
    results = []
    for n, seed, nrhs in ((30000, 71, 2), (9000, 72, 1)):          # the second call is smaller
        z = synth.square_points(n, seed)
        f = synth.real_rhs(n, seed, nrhs)
        print(f"noalloc precision={precision} n={n} nrhs={nrhs}", flush=True)
        plan = pkg.sbd_plan(_t(z), eps=1e-3 if precision == 0 else 1e-6, delta_min=(10 / (np.pi * n)) ** 0.5,
                            precision=precision, max_rhs=nrhs, deterministic=1)
        assert plan.workspace_bytes(nrhs) <= pkg._abi.SBD_NOALLOC_SCRATCH_BYTES
        ft = _t(f)
        ws = torch.empty(plan.workspace_bytes(nrhs), dtype=torch.uint8, device=device())
        q_ws = plan.apply(ft, workspace=ws)
        q_na = torch.empty_like(q_ws)
        pkg.sbd_apply_noalloc(plan, ft, q_na)
        torch.cuda.synchronize()
        a, b = q_ws.cpu().numpy(), q_na.cpu().numpy()
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8))
        rows = np.arange(0, n, max(1, n // 64))
        ref = oracle.direct_sum(z, f, rows=rows)
        assert rel_l2(b[:, rows], ref) < (1e-3 if precision == 0 else 1e-6)
        results.append(b)
        plan.free()
    assert results[0].shape != results[1].shape


def test_noalloc_default_plan_and_repeat():
    import torch
    pkg = lib()
    z = synth.star_points(30000, 73)
    f = synth.complex_rhs(30000, 73, 1)
    plan = pkg.sbd_plan(_t(z), eps=1e-4)
    ft = _t(f).to(torch.complex64)
    q_ws = plan.apply(ft)
    outs = []
    for _ in range(2):
        q = torch.empty_like(q_ws)
        pkg.sbd_apply_noalloc(plan, ft, q)
        outs.append(q)
    torch.cuda.synchronize()
    for q in outs:
        assert rel_l2(q.cpu().numpy(), q_ws.cpu().numpy()) < 1e-6
    plan.free()


def test_noalloc_refuses_workspace_beyond_scratch():
    import torch
    pkg = lib()
    n = 1_000_000
    z = synth.square_points(n, 74)
    plan = pkg.sbd_plan(_t(z), eps=1e-3, delta_min=(10 / (np.pi * n)) ** 0.5, max_rhs=2)
    assert plan.workspace_bytes(2) > pkg._abi.SBD_NOALLOC_SCRATCH_BYTES
    ft = _t(synth.real_rhs(n, 74, 2))
    q = torch.full_like(ft, 7.0)
    with pytest.raises(pkg.SbdError) as e:
        pkg.sbd_apply_noalloc(plan, ft, q)
    assert e.value.status == SBD_ENOMEM and "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert bool(torch.all(q == 7.0))                 # nothing was launched
    plan.free()
