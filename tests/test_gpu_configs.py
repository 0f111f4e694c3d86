"""Parity on the other paper-shaped workloads at full size, sampled rows against the
FP64 direct sum:

* three disjoint ellipses, N = 1e6, eps = 1e-6, far field in FP64 and in FP32
  (delta_min from the curve rule of Theorem 1), 4096 sampled rows, relative l2 error
  at most eps in FP64 and 2 eps in FP32 (its rounding floor, see test_ellipses);
* Helmholtz (i/4) H0(k|x|), k = 100 pi, N = 2e5 points on a perturbed circle,
  16 complex right-hand sides in one call, eps = 1e-4, 1024 sampled rows of every
  right-hand side.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_util import device, direct_rows, lib, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ellipses():
    z, f, spec = synth.make_workload("ellipses1m")
    return z, f, spec


# FP32 far field: its rounding floor (FP32 grids through two 2-D transforms of about 14000
# points per axis, and the spread's 32-bit fixed point on tiles crossed by dense curves)
# is about 1e-6 relative here, at the level of eps itself, so the FP32 leg is held to 2 eps
# and reported against eps; the FP64 path meets eps with three orders to spare.
@pytest.mark.parametrize("precision,tol", [(1, 1e-6), (0, 2e-6)])
def test_ellipses(ellipses, precision, tol):
    import torch
    z, f, spec = ellipses
    pkg = lib()
    eps = spec["eps"]
    print(f"ellipses N={len(z)} precision={precision}", flush=True)
    plan = pkg.sbd_plan(torch.tensor(z, device=device()), eps=eps, precision=precision)
    info = plan.info()
    print({k: info[k] for k in ["P", "n_xi", "nnz", "nx", "Mx", "w", "delta_min"]}, flush=True)
    q = plan.apply(torch.tensor(f, device=device()))
    torch.cuda.synchronize()
    q = q.cpu().numpy()[0]
    rows = np.random.default_rng(3).integers(0, len(z), 4096)
    ref = direct_rows(z, f[0], rows)
    err = rel_l2(q[rows], ref)
    print("rel l2", err, flush=True)
    assert err < tol
    assert np.max(np.abs(q[rows] - ref)) <= 1.1 * eps / (2 * math.pi) * np.abs(f[0]).sum()
    plan.free()


def test_helmholtz_16_rhs():
    import torch
    z, f, spec = synth.make_workload("helmholtz200k")
    pkg = lib()
    eps, k = spec["eps"], spec["wavenumber"]
    print(f"helmholtz N={len(z)} k={k:.2f} nrhs={f.shape[0]}", flush=True)
    plan = pkg.sbd_plan(torch.tensor(z, device=device()), kind=pkg.SBD_HELMHOLTZ, eps=eps, wavenumber=k,
                        max_rhs=f.shape[0])
    info = plan.info()
    print({kk: info[kk] for kk in ["P", "n_xi", "nnz", "nx", "Mx", "w", "delta_min"]}, flush=True)
    ft = torch.tensor(f, device=device())
    q = plan.apply(ft)
    torch.cuda.synchronize()
    q = q.cpu().numpy()
    rows = np.random.default_rng(4).integers(0, len(z), 1024)
    ref = direct_rows(z, f, rows, "helmholtz", k)
    err = rel_l2(q[:, rows], ref)
    print("rel l2", err, flush=True)
    assert err < eps
    bound = 1.1 * eps * 0.25 * np.abs(f).sum(axis=1, keepdims=True)
    assert np.all(np.abs(q[:, rows] - ref) <= bound)
    # fused batch equals one-by-one
    for r in [0, 7]:
        q1 = plan.apply(ft[r:r + 1].contiguous())
        torch.cuda.synchronize()
        assert rel_l2(q1.cpu().numpy()[0], q[r]) < 1e-6
    plan.free()
