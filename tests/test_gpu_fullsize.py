"""Parity at the full N = 1e7 workload (points uniform in the unit square, eps = 1e-3),
in the launch configuration bench.py times: sampled rows against the FP64 direct sum,
the binning permutation bit for bit, sampled CSR rows bit for bit against brute force,
and linearity / symmetry properties that hold at any size."""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_util import device, direct_rows, lib, rel_l2

pytestmark = pytest.mark.gpu

N = 10_000_000
EPS = 1e-3


@pytest.fixture(scope="module")
def big():
    import torch
    pkg = lib()
    z, f, spec = synth.make_workload("square10m")
    dmin = math.sqrt(10.0 / (math.pi * N))
    print("planning N=1e7", flush=True)
    plan = pkg.sbd_plan(torch.tensor(z, device=device()), eps=EPS, delta_min=dmin, max_rhs=2)
    return z, f, dmin, plan


def test_sampled_rows_match_direct_sum(big):
    import torch
    z, f, dmin, plan = big
    q = plan.apply(torch.tensor(f, device=device()))
    torch.cuda.synchronize()
    q = q.cpu().numpy()[0]
    rows = np.random.default_rng(11).integers(0, N, 2048)
    ref = direct_rows(z, f[0], rows)
    err = rel_l2(q[rows], ref)
    print("sampled rel l2", err, flush=True)
    assert err < EPS
    assert np.max(np.abs(q[rows] - ref)) <= 1.1 * EPS / (2 * math.pi) * np.abs(f[0]).sum()


def test_permutation_bit_exact(big):
    z, f, dmin, plan = big
    from paper_1711_07877_amd import SBD_ARR_PERM
    info = plan.info()
    keys = oracle.bin_keys(z, info["x0"], info["y0"], info["inv_c"], info["ncx"], info["ncy"], info["nsub"],
                           info["ntx"])
    assert np.array_equal(plan.export(SBD_ARR_PERM), oracle.stable_perm(keys))


def test_sampled_csr_rows_bit_exact(big):
    z, f, dmin, plan = big
    from paper_1711_07877_amd import SBD_ARR_PERM, SBD_ARR_ROWPTR, SBD_ARR_COL
    info = plan.info()
    perm = plan.export(SBD_ARR_PERM)
    rp = plan.export(SBD_ARR_ROWPTR)
    col = plan.export(SBD_ARR_COL)
    assert rp[-1] == info["nnz"] == len(col)
    zs = z[perm]
    d2max = dmin * dmin
    for i in np.random.default_rng(5).integers(0, N, 24):
        dx = zs[i, 0] - zs[:, 0]
        dy = zs[i, 1] - zs[:, 1]
        ref = np.nonzero(dx * dx + dy * dy <= d2max)[0]
        assert np.array_equal(col[rp[i]:rp[i + 1]], ref), i
    mean = info["nnz"] / N
    assert 9.0 < mean < 13.0                      # about ten neighbours plus the diagonal


def test_linearity_and_symmetry(big):
    import torch
    z, f, dmin, plan = big
    g = synth.real_rhs(N, 99)[0]
    fg = np.stack([f[0], g])
    q = plan.apply(torch.tensor(fg, device=device()))
    lin = plan.apply(torch.tensor((0.3 * f[0] - 1.7 * g)[None, :], device=device()))
    torch.cuda.synchronize()
    q = q.cpu().numpy()
    lin = lin.cpu().numpy()[0]
    assert rel_l2(lin, 0.3 * q[0] - 1.7 * q[1]) < 1e-5
    # the operator is symmetric: <g, A f> = <A g, f>
    a, b = float(np.dot(g, q[0])), float(np.dot(q[1], f[0]))
    assert abs(a - b) <= 1e-4 * np.linalg.norm(g) * np.linalg.norm(q[0])
