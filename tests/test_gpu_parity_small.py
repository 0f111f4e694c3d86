"""GPU SBD plan/apply against the CPU oracle at sizes the oracle finishes in seconds."""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_util import device, lib, rel_l2, far_field_with_plan_spectrum

pytestmark = pytest.mark.gpu


def _plan(z, eps, kind=0, k=0.0, dmin=0.0, **kw):
    import torch
    pkg = lib()
    pts = torch.tensor(z, dtype=torch.float64, device=device())
    return pkg.sbd_plan(pts, kind=kind, eps=eps, wavenumber=k, delta_min=dmin, **kw)


def _apply(plan, f, parts=3):
    import torch
    ft = torch.tensor(np.atleast_2d(f), device=device())
    q = plan.apply(ft, parts=parts)
    torch.cuda.synchronize()
    return q.cpu().numpy()


@pytest.fixture(scope="module")
def disk():
    z, f, spec = synth.make_workload("disk4k")
    dmin = oracle.default_delta_min(z, "ten", spec["eps"], area=math.pi)
    return z, f, dmin, spec["eps"]


def test_binning_and_csr_bit_exact(disk):
    z, f, dmin, eps = disk
    print("plan disk4k fp32", flush=True)
    plan = _plan(z, eps, dmin=dmin)
    from paper_1711_07877_amd import SBD_ARR_PERM, SBD_ARR_ROWPTR, SBD_ARR_COL, SBD_ARR_KEYS
    info = plan.info()
    keys = oracle.bin_keys(z, info["x0"], info["y0"], info["inv_c"], info["ncx"], info["ncy"], info["nsub"],
                           info["ntx"])
    perm = oracle.stable_perm(keys)
    assert np.array_equal(plan.export(SBD_ARR_PERM), perm)
    assert np.array_equal(plan.export(SBD_ARR_KEYS), keys[perm])
    rp, col = oracle.csr_from_perm(z, perm, dmin)
    assert info["d2max"] == dmin * dmin
    assert np.array_equal(plan.export(SBD_ARR_ROWPTR), rp)
    assert np.array_equal(plan.export(SBD_ARR_COL), col)


def test_near_values_match_oracle(disk):
    z, f, dmin, eps = disk
    plan = _plan(z, eps, dmin=dmin)
    from paper_1711_07877_amd import SBD_ARR_PERM, SBD_ARR_ROWPTR, SBD_ARR_COL, SBD_ARR_VAL
    info = plan.info()
    perm = plan.export(SBD_ARR_PERM)
    rp = plan.export(SBD_ARR_ROWPTR)
    col = plan.export(SBD_ARR_COL)
    val = plan.export(SBD_ARR_VAL)
    rows = np.repeat(np.arange(len(z)), np.diff(rp))
    fit = oracle.fit_laplace(dmin / info["delta_max"], eps, P=info["P"])
    ref = oracle.near_values(z[perm], rows, col, fit, info["delta_max"], "laplace")
    assert np.max(np.abs(val - ref)) < 1e-11


def test_near_values_match_pair_difference_assembly(disk):
    """The plan's D (radial series) against the paper's own assembly: G at each pair
    difference minus the exponential sum over the plan's exported circle nodes."""
    from gpu_util import PlanSpectrum
    from oracle import sbd as osbd
    z, f, dmin, eps = disk
    plan = _plan(z, eps, dmin=dmin)
    from paper_1711_07877_amd import SBD_ARR_PERM, SBD_ARR_ROWPTR, SBD_ARR_COL, SBD_ARR_VAL
    info = plan.info()
    perm = plan.export(SBD_ARR_PERM)
    rp = plan.export(SBD_ARR_ROWPTR)
    col = plan.export(SBD_ARR_COL)
    val = plan.export(SBD_ARR_VAL)
    rows = np.repeat(np.arange(len(z)), np.diff(rp))
    xi, w, w0 = osbd.frequencies(PlanSpectrum(plan), info["delta_max"], "laplace", eps)
    ref = oracle.near_values_nufft(z[perm], rows, col, xi, w, w0, "laplace")
    assert np.max(np.abs(ref.imag)) < 1e-12
    assert np.max(np.abs(val - ref.real)) < 1e-11


@pytest.mark.parametrize("precision", [0, 1])
def test_apply_matches_direct_sum(disk, precision):
    z, f, dmin, eps = disk
    print(f"apply disk4k precision={precision}", flush=True)
    plan = _plan(z, eps, dmin=dmin, precision=precision)
    q = _apply(plan, f[0])[0]
    qd = oracle.direct_sum(z, f[0])
    assert rel_l2(q, qd) < eps
    assert np.max(np.abs(q - qd)) <= 1.1 * eps / (2 * math.pi) * np.abs(f[0]).sum()


@pytest.mark.parametrize("precision,tol", [(0, 0.0), (1, 1e-11)])
def test_far_field_against_exact_sums(disk, precision, tol):
    """NUFFT-isolated: GPU far field vs exact exponential sums over the plan's own frequencies."""
    z, f, dmin, eps = disk
    kw = dict(precision=precision)
    if tol:
        kw.update(nufft_tol=tol, sigma=2.0)
    plan = _plan(z, eps, dmin=dmin, **kw)
    qf = _apply(plan, f[0], parts=1)[0]
    ref = far_field_with_plan_spectrum(z, f[0], plan, "laplace", eps)[0].real
    err = rel_l2(qf, ref)
    print("far rel err", precision, err, plan.info()["w"], flush=True)
    assert err < (2e-5 if precision == 0 else 1e-9)


def test_near_part_alone(disk):
    z, f, dmin, eps = disk
    plan = _plan(z, eps, dmin=dmin, precision=1)
    qn = _apply(plan, f[0], parts=2)[0]
    out = oracle.sbd_oracle(z, f[0], eps=eps, delta_min=dmin, P=plan.info()["P"], return_parts=True)
    assert np.max(np.abs(qn - out["q_close"])) < 1e-10 * np.abs(out["q_close"]).max()


def test_multi_rhs_fused_equals_single(disk):
    z, f, dmin, eps = disk
    import torch
    fs = synth.real_rhs(len(z), 77, 3)
    plan = _plan(z, eps, dmin=dmin, max_rhs=3)
    qa = _apply(plan, fs)
    for r in range(3):
        qr = _apply(plan, fs[r])[0]
        assert rel_l2(qa[r], qr) < 1e-6


def test_helmholtz_curve_matches_direct_sum():
    z = synth.star_points(3000, 4)
    f = synth.complex_rhs(3000, 4, 2)
    eps, k = 1e-4, 40.0
    print("plan helmholtz 3000", flush=True)
    plan = _plan(z, eps, kind=1, k=k, max_rhs=2)
    q = _apply(plan, f)
    qd = oracle.direct_sum(z, f, "helmholtz", k)
    assert rel_l2(q, qd) < eps
    bound = 1.1 * eps * 0.25 * np.abs(f).sum(axis=1, keepdims=True)
    assert np.all(np.abs(q - qd) <= bound)


@pytest.mark.parametrize("precision", [0, 1])
def test_helmholtz_small_k_dini_matches_direct_sum(precision):
    """k delta_max below the first zero of Y0: the plan fits Y0 in the Dini basis (no
    kappa' rescaling, lambda = 1) with the oracle's order, and the apply meets eps."""
    z = synth.disk_points(4000, 71)
    f = synth.complex_rhs(4000, 71, 1)
    eps, k = 1e-4, 0.2
    dmin = oracle.default_delta_min(z, "ten", eps, area=math.pi)
    print(f"plan helmholtz small k precision={precision}", flush=True)
    plan = _plan(z, eps, kind=1, k=k, dmin=dmin, precision=precision)
    from paper_1711_07877_amd import SBD_ARR_RADII
    info = plan.info()
    kappa = k * info["delta_max"]
    assert kappa < oracle.sbd_fit.Y0_FIRST_ZERO
    fit = oracle.fit_helmholtz(dmin / info["delta_max"], eps, kappa)
    assert fit.robin_H > 0 and abs(info["P"] - fit.P) <= 1
    # the plan's circles are the Dini roots themselves (no kappa' dilation)
    radii = plan.export(SBD_ARR_RADII)
    n = min(len(radii), fit.P)
    assert np.allclose(radii[:n], fit.radii[:n], rtol=1e-12, atol=0)
    q = _apply(plan, f)
    qd = oracle.direct_sum(z, f, "helmholtz", k)
    assert rel_l2(q, qd) < eps
    assert np.all(np.abs(q - qd) <= 1.1 * eps * 0.25 * np.abs(f).sum(axis=1, keepdims=True))
