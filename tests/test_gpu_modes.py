"""Plan options on the GPU, through the C ABI:

* close-correction entries in FP64 under the FP32 far field (the default; the FP32 NUFFT
  path with FP64 near-field entries of the headline workload) against D stored in FP32
  (near_fp32): the near part alone equals the oracle's D f to FP64 accuracy in the first and
  to FP32 rounding in the second, the FP32 plan releases the FP64 entries, and both meet the
  tolerance against the direct sum;
* deterministic plans return bit-identical q on repeated applies (FP32 and FP64, real and
  complex f) and agree with the default mode to rounding;
* a non-finite value in f makes q non-finite (documented propagation), in every spread;
* byte_cap refuses a plan whose memory exceeds it with SBD_ENOMEM."""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_util import device, lib, rel_l2

pytestmark = pytest.mark.gpu

SBD_ENOMEM = -2


def _t(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=device())


def _apply(plan, f, parts=3, dtype=None):
    import torch
    ft = torch.tensor(np.atleast_2d(f), device=device())
    if dtype is not None:
        ft = ft.to(dtype)
    q = plan.apply(ft, parts=parts)
    torch.cuda.synchronize()
    return q.cpu().numpy()


@pytest.fixture(scope="module")
def disk():
    z, f, spec = synth.make_workload("disk4k")
    dmin = oracle.default_delta_min(z, "ten", spec["eps"], area=math.pi)
    return z, f, dmin, spec["eps"]


def test_fp64_entries_under_fp32_far_field(disk):
    from paper_1711_07877_amd import SBD_ARR_VAL
    z, f, dmin, eps = disk
    pkg = lib()
    print("plan disk4k fp32 far field, FP64 and FP32 close entries", flush=True)
    p64 = pkg.sbd_plan(_t(z), eps=eps, delta_min=dmin)
    p32 = pkg.sbd_plan(_t(z), eps=eps, delta_min=dmin, near_fp32=1)
    i64, i32 = p64.info(), p32.info()
    assert i64["nnz"] == i32["nnz"] > 0
    # the FP32-entry plan keeps 4 bytes per entry instead of 8
    assert i64["plan_bytes"] - i32["plan_bytes"] == 4 * i64["nnz"]
    v64, v32 = p64.export(SBD_ARR_VAL), p32.export(SBD_ARR_VAL)
    assert np.array_equal(v32, v64.astype(np.float32).astype(np.float64))
    out = oracle.sbd_oracle(z, f[0], eps=eps, delta_min=dmin, P=i64["P"], return_parts=True)
    ref = out["q_close"]
    scale = np.abs(ref).max()
    n64 = _apply(p64, f[0], parts=2)[0]
    n32 = _apply(p32, f[0], parts=2)[0]
    # FP64 entries, FP64 row sums: only f's FP32 rounding in the sorted copy remains
    e64 = np.max(np.abs(n64 - ref)) / scale
    e32 = np.max(np.abs(n32 - ref)) / scale
    print(f"near part error: fp64 entries {e64:.2e}, fp32 entries {e32:.2e}", flush=True)
    assert e64 < 3e-7
    assert e32 < 3e-6
    qd = oracle.direct_sum(z, f[0])
    for p in (p64, p32):
        q = _apply(p, f[0])[0]
        assert rel_l2(q, qd) < eps
        assert np.max(np.abs(q - qd)) <= 1.1 * eps / (2 * math.pi) * np.abs(f[0]).sum()
    p64.free()
    p32.free()


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("cplx", [False, True])
def test_deterministic_repeats_bitwise(precision, cplx):
    import torch
    pkg = lib()
    # a dense curve: long close rows (many partial sums per row) and crowded spread tiles
    z = synth.star_points(20000, 31)
    f = synth.complex_rhs(20000, 31, 2) if cplx else synth.real_rhs(20000, 31, 2)
    eps = 1e-6 if precision else 1e-3
    print(f"deterministic precision={precision} complex={cplx}", flush=True)
    pd = pkg.sbd_plan(_t(z), eps=eps, precision=precision, max_rhs=2, deterministic=1)
    pn = pkg.sbd_plan(_t(z), eps=eps, precision=precision, max_rhs=2)
    assert pd.info()["nnz"] / len(z) > 30
    dt = torch.complex128 if cplx else torch.float64
    runs = [_apply(pd, f, dtype=dt) for _ in range(4)]
    for r in runs[1:]:
        assert np.array_equal(r.view(np.uint8), runs[0].view(np.uint8))
    qn = _apply(pn, f, dtype=dt)
    assert rel_l2(runs[0], qn) < (1e-12 if precision else 1e-6)
    rows = np.arange(0, len(z), 997)
    kind = "laplace"
    ref = oracle.direct_sum(z, f, kind, 0.0, rows=rows)
    assert rel_l2(runs[0][:, rows], ref) < eps
    pd.free()
    pn.free()


@pytest.mark.parametrize("precision,deterministic", [(0, 0), (1, 0), (1, 1)])
@pytest.mark.parametrize("bad", [float("nan"), float("inf")])
def test_non_finite_f_propagates(precision, deterministic, bad):
    pkg = lib()
    z = synth.square_points(3000, 33)
    f = synth.real_rhs(3000, 33)[0].copy()
    f[1234] = bad
    plan = pkg.sbd_plan(_t(z), eps=1e-3, delta_min=0.03, precision=precision, deterministic=deterministic)
    q = _apply(plan, f)[0]
    plan.free()
    assert not np.any(np.isfinite(q))


def test_byte_cap_refuses_large_plans():
    pkg = lib()
    z = synth.square_points(20000, 34)
    ok = pkg.sbd_plan(_t(z), eps=1e-3, delta_min=0.01)
    need = ok.plan_bytes() + ok.workspace_bytes(1)
    ok.free()
    with pytest.raises(pkg.SbdError) as e:
        pkg.sbd_plan(_t(z), eps=1e-3, delta_min=0.01, byte_cap=need // 2)
    assert e.value.status == SBD_ENOMEM
    fits = pkg.sbd_plan(_t(z), eps=1e-3, delta_min=0.01, byte_cap=need + 4096)
    fits.free()
