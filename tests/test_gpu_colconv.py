"""The compiled whole-column convolution (transform length and radices fixed at compile
time) against the generic column passes on the same plans: both compute the same
discrete convolution on the grid, so q agrees to the precision's rounding; and the full
result still meets the tolerance against the FP64 direct sum.  Covers several transform
lengths of the instance ladder, FP32 and FP64, real and complex f on Laplace plans, and
Helmholtz (complex symbol).  FP32 Laplace plans with real f run the compiled rows with
the row-pair layout (spectra of rows 2m and 2m + 1 interleaved per column, the inverse
rows two per workgroup); the FP32 grids here have ny = nty T + 8 (kernel width 7), so
with tiles of 16 or more the last group of 16 rows of the forward row remap is partial,
and two right-hand sides exercise the batch offsets."""
import math
import os

import numpy as np
import pytest

import oracle
import synth
from gpu_util import device, lib, rel_l2

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), device=device())


def _plan_both(z, **kw):
    pkg = lib()
    plans = {}
    for mode in ("1", "0"):
        os.environ["SBD_COLCONV"] = mode
        try:
            plans[mode] = pkg.sbd_plan(_t(z), **kw)
        finally:
            os.environ.pop("SBD_COLCONV", None)
    return plans["1"], plans["0"]


def _apply(plan, f, dtype=None):
    import torch
    ft = _t(np.atleast_2d(f))
    if dtype is not None:
        ft = ft.to(dtype)
    q = plan.apply(ft)
    torch.cuda.synchronize()
    return q.cpu().numpy()


@pytest.mark.parametrize("n", [4000, 20000, 60000, 200000])
@pytest.mark.parametrize("precision", [0, 1])
def test_compiled_columns_match_generic_laplace(n, precision):
    import torch
    z = synth.square_points(n, 500 + n % 97)
    f = synth.real_rhs(n, 501, 2)
    eps = 1e-3 if precision == 0 else 1e-6
    print(f"colconv laplace n={n} precision={precision}", flush=True)
    pc, pg = _plan_both(z, eps=eps, delta_min=math.sqrt(10.0 / (math.pi * n)), precision=precision, max_rhs=2)
    ic, ig = pc.info(), pg.info()
    print({k: ic[k] for k in ("nx", "ny", "Mx", "My", "colconv")}, "generic My", ig["My"], flush=True)
    assert ig["colconv"] == 0
    qc, qg = _apply(pc, f), _apply(pg, f)
    tol = 2e-6 if precision == 0 else 1e-12
    if ic["colconv"]:
        assert rel_l2(qc, qg) < tol
    # complex f on the Laplace plans takes the complex grid path through the same columns
    fz = f[0] + 1j * f[1]
    zc, zg = _apply(pc, fz, torch.complex128), _apply(pg, fz, torch.complex128)
    if ic["colconv"]:
        assert rel_l2(zc, zg) < tol
    assert rel_l2(zc[0].real, qc[0]) < tol and rel_l2(zc[0].imag, qc[1]) < tol
    rows = np.arange(0, n, max(1, n // 200))
    ref = oracle.direct_sum(z, f, rows=rows)
    assert rel_l2(qc[:, rows], ref) < eps
    pc.free()
    pg.free()


def test_some_lengths_take_the_compiled_kernel():
    pkg = lib()
    used = 0
    for n in (4000, 20000, 60000, 200000):
        z = synth.square_points(n, 502)
        p = pkg.sbd_plan(_t(z), eps=1e-3, delta_min=math.sqrt(10.0 / (math.pi * n)))
        used += p.info()["colconv"]
        p.free()
    assert used == 4


@pytest.mark.parametrize("precision", [0, 1])
def test_compiled_columns_match_generic_helmholtz(precision):
    import torch
    n = 6000
    z = synth.star_points(n, 503)
    f = synth.complex_rhs(n, 503, 1)
    k = 25.0
    eps = 1e-4 if precision == 0 else 1e-6
    pc, pg = _plan_both(z, kind=lib().SBD_HELMHOLTZ, wavenumber=k, eps=eps, precision=precision)
    ic = pc.info()
    print({kk: ic[kk] for kk in ("nx", "ny", "Mx", "My", "colconv")}, flush=True)
    dt = torch.complex64 if precision == 0 else torch.complex128
    qc, qg = _apply(pc, f, dt), _apply(pg, f, dt)
    if ic["colconv"]:
        assert rel_l2(qc, qg) < (2e-6 if precision == 0 else 1e-12)
    rows = np.arange(0, n, 37)
    ref = oracle.direct_sum(z, f, "helmholtz", k, rows=rows)
    assert rel_l2(qc[:, rows], ref) < eps
    pc.free()
    pg.free()


@pytest.mark.parametrize("precision", [0, 1])
def test_row_pairs_are_a_pure_relayout(precision):
    """The row-pair layout moves data, not arithmetic: every butterfly, twiddle and symbol
    product is the one of natural rows, so with the order-free (deterministic) spread and
    close correction q is bit-identical with SBD_ROW_PAIRS=0 (natural rows) and 1 in FP32.
    In FP64 the compiler contracts a few multiply-adds of the two-row inverse kernel
    differently from the one-row kernel, so the two agree to the last bits (relative
    1e-13).  The first size of the list whose plan takes the layout is used."""
    import torch
    pkg = lib()
    eps = 1e-3 if precision == 0 else 1e-6

    def make(z, n, mode):
        os.environ["SBD_ROW_PAIRS"] = mode
        try:
            return pkg.sbd_plan(_t(z), eps=eps, delta_min=math.sqrt(10.0 / (math.pi * n)), precision=precision,
                                max_rhs=2, deterministic=1)
        finally:
            os.environ.pop("SBD_ROW_PAIRS", None)

    for n in (60000, 200000, 20000, 1_000_000):
        z = synth.square_points(n, 777)
        p1 = make(z, n, "1")
        if p1.info()["row_pairs"]:
            break
        p1.free()
    else:
        pytest.fail(f"no candidate size takes the row-pair layout at precision {precision}")
    info = p1.info()
    print(f"row pairs relayout precision={precision} n={n} Mx={info['Mx']} My={info['My']}", flush=True)
    p0 = make(z, n, "0")
    assert p0.info()["row_pairs"] == 0
    f = synth.real_rhs(n, 778, 2)
    q0 = _apply(p0, f, torch.float64)
    q1 = _apply(p1, f, torch.float64)
    if precision == 0:
        assert np.array_equal(q0.view(np.uint8), q1.view(np.uint8))
    else:
        d = float(np.max(np.abs(q1 - q0)))
        print(f"  max |q_pairs - q_natural| = {d:.3e} (max |q| {float(np.max(np.abs(q0))):.3e})", flush=True)
        assert d <= 1e-13 * float(np.max(np.abs(q0)))
    rows = np.arange(0, n, max(1, n // 40))
    ref = oracle.direct_sum(z, f, rows=rows)
    assert rel_l2(q1[:, rows], ref) < eps
    p0.free()
    p1.free()
