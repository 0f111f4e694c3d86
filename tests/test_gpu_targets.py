"""Two-set plans (targets apart from sources, the form of the paper's numerical
experiments): binning and CSR bit-exact against the oracle's cross pairs, D values,
and q against the FP64 two-set direct sum."""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_util import device, lib, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def two_disks():
    y = synth.disk_points(3000, 21)          # sources
    x = 0.9 * synth.disk_points(2500, 22)    # targets
    f = synth.real_rhs(3000, 21)[0]
    dmin = math.sqrt(10.0 / 3000)
    return x, y, f, dmin


def _plan(x, y, eps, dmin, **kw):
    import torch
    pkg = lib()
    dev = device()
    return pkg.sbd_plan_targets(torch.tensor(x, device=dev), torch.tensor(y, device=dev), eps=eps, delta_min=dmin, **kw)


def test_binning_and_cross_csr_bit_exact(two_disks):
    x, y, f, dmin = two_disks
    print("two-set plan binning", flush=True)
    plan = _plan(x, y, 1e-3, dmin)
    from paper_1711_07877_amd import (SBD_ARR_PERM, SBD_ARR_TPERM, SBD_ARR_KEYS, SBD_ARR_TKEYS, SBD_ARR_ROWPTR,
                                      SBD_ARR_COL)
    info = plan.info()
    assert info["bipartite"] == 1 and info["n"] == len(y) and info["n_targets"] == len(x)
    binning = (info["x0"], info["y0"], info["inv_c"], info["ncx"], info["ncy"], info["nsub"], info["ntx"])
    ks = oracle.bin_keys(y, *binning)
    kt = oracle.bin_keys(x, *binning)
    ps, pt = oracle.stable_perm(ks), oracle.stable_perm(kt)
    assert np.array_equal(plan.export(SBD_ARR_PERM), ps)
    assert np.array_equal(plan.export(SBD_ARR_TPERM), pt)
    assert np.array_equal(plan.export(SBD_ARR_KEYS), ks[ps])
    assert np.array_equal(plan.export(SBD_ARR_TKEYS), kt[pt])
    # rows: sorted targets; columns: sorted source positions, ascending
    k, l = oracle.near_pairs_targets(x[pt], y[ps], dmin)
    rp = np.concatenate([[0], np.cumsum(np.bincount(k, minlength=len(x)))])
    assert info["d2max"] == dmin * dmin
    assert np.array_equal(plan.export(SBD_ARR_ROWPTR), rp)
    assert np.array_equal(plan.export(SBD_ARR_COL), l)
    plan.free()


def test_cross_values_match_oracle(two_disks):
    x, y, f, dmin = two_disks
    plan = _plan(x, y, 1e-3, dmin)
    from paper_1711_07877_amd import SBD_ARR_PERM, SBD_ARR_TPERM, SBD_ARR_ROWPTR, SBD_ARR_COL, SBD_ARR_VAL
    info = plan.info()
    ps, pt = plan.export(SBD_ARR_PERM), plan.export(SBD_ARR_TPERM)
    rp, col, val = plan.export(SBD_ARR_ROWPTR), plan.export(SBD_ARR_COL), plan.export(SBD_ARR_VAL)
    rows = np.repeat(np.arange(len(x)), np.diff(rp))
    fit = oracle.fit_laplace(dmin / info["delta_max"], 1e-3, P=info["P"])
    ref = oracle.near_values_targets(x[pt], y[ps], rows, col, fit, info["delta_max"], "laplace")
    assert np.max(np.abs(val - ref)) < 1e-11
    plan.free()


@pytest.mark.parametrize("precision", [0, 1])
def test_two_set_apply_matches_direct_sum(two_disks, precision):
    import torch
    x, y, f, dmin = two_disks
    eps = 1e-3
    print(f"two-set apply precision={precision}", flush=True)
    plan = _plan(x, y, eps, dmin, precision=precision)
    q = plan.apply(torch.tensor(f[None, :], device=device()))
    torch.cuda.synchronize()
    q = q.cpu().numpy()[0]
    assert q.shape == (len(x),)
    ref = oracle.direct_sum_targets(x, y, f)
    assert rel_l2(q, ref) < eps
    assert np.max(np.abs(q - ref)) <= 1.1 * eps / (2 * math.pi) * np.abs(f).sum()
    plan.free()


def test_two_set_helmholtz_curves():
    import torch
    y = synth.star_points(2500, 31)
    x = 0.8 * synth.star_points(2000, 32)
    f = synth.complex_rhs(2500, 31, nrhs=2)
    k = 40.0
    print("two-set Helmholtz", flush=True)
    plan = _plan(x, y, 1e-4, 0.0, kind=lib().SBD_HELMHOLTZ, wavenumber=k, max_rhs=2)
    q = plan.apply(torch.tensor(f, device=device()))
    torch.cuda.synchronize()
    q = q.cpu().numpy()
    ref = oracle.direct_sum_targets(x, y, f, "helmholtz", k)
    assert rel_l2(q, ref) < 1e-4
    bound = 1.1 * 1e-4 / 4 * np.abs(f).sum(axis=1)[:, None]
    assert np.all(np.abs(q - ref) <= bound)
    plan.free()


def test_target_on_a_source_is_rejected():
    y = synth.disk_points(500, 41)
    x = np.concatenate([synth.disk_points(100, 42), y[7:8]])
    pkg = lib()
    with pytest.raises(pkg.SbdError):
        _plan(x, y, 1e-3, math.sqrt(10.0 / 500))
