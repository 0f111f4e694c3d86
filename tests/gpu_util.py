"""Helpers for GPU tests (device selection, oracle-side reconstruction of a plan's spectrum)."""
import math

import numpy as np
import pytest


def device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch.device("cuda:0")


def lib():
    import paper_1711_07877_amd as pkg
    pkg.load_library()
    return pkg


def host_threads() -> int:
    """Host threads for the oracle's sampled-row sums: the CPU affinity set, at most 16."""
    import os
    return max(1, min(16, len(os.sched_getaffinity(0))))


def direct_rows(z, f, rows, kind="laplace", wavenumber=0.0, targets=None, general=None):
    """The oracle's FP64 direct sum restricted to `rows`, computed over row blocks on all
    host threads (numpy releases the GIL inside its array operations; each block is an
    unchanged call of the oracle).  targets: two-set sum with targets apart from z;
    general: (c_log, terms) of a general radial kernel."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    rows = np.asarray(rows)
    blocks = [b for b in np.array_split(rows, max(1, min(len(rows), 4 * host_threads()))) if len(b)]

    def one(b):
        if general is not None:
            return oracle.direct_sum_general(z, f, general[0], general[1], rows=b)
        if targets is not None:
            return oracle.direct_sum_targets(targets, z, f, kind, wavenumber, rows=b)
        return oracle.direct_sum(z, f, kind, wavenumber, rows=b)

    with ThreadPoolExecutor(host_threads()) as ex:
        parts = list(ex.map(one, blocks))
    return np.concatenate(parts, axis=-1)


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


class PlanSpectrum:
    """The plan's own radial fit (exported) in the shape the oracle's frequency builder expects."""

    def __init__(self, plan):
        from paper_1711_07877_amd import SBD_ARR_COEF, SBD_ARR_RADII, SBD_ARR_M
        self.coef = plan.export(SBD_ARR_COEF)
        self.radii = plan.export(SBD_ARR_RADII)
        self.M = plan.export(SBD_ARR_M)
        self.P = len(self.coef)


def far_field_with_plan_spectrum(z, f, plan, kind, eps, wavenumber=0.0):
    """Exact-sum far field (oracle) fed the plan's coefficients and circle sizes."""
    import oracle
    from oracle import sbd as osbd
    info = plan.info()
    spec = PlanSpectrum(plan)
    xi, w, w0 = osbd.frequencies(spec, info["delta_max"], kind, eps, wavenumber)
    c = np.array([info["center_x"], info["center_y"]])
    f2 = np.atleast_2d(f).astype(np.complex128)
    return osbd.far_exact(z, f2, c, xi, w, w0)
