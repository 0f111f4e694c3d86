"""Request server: every request's result matches the same request served alone and
the FP64 direct sum (applies) or solves the exact single-layer system (GMRES)."""
import math

import numpy as np
import pytest

import oracle
from gpu_util import device, lib, rel_l2

pytestmark = pytest.mark.gpu


def test_mixed_stream_matches_isolated_and_oracle():
    device()
    lib()
    from paper_1711_07877_amd import serve
    reqs, gaps = serve.make_stream(10, seed=9, nmin=1e3, nmax=2e4)
    print("serve: 10 requests, isolated then mixed", flush=True)
    alone = serve.Server(workers=1, keep_outputs=True)
    ra = {r.rid: r for r in alone.run_stream(reqs, None)}
    alone.close()
    mixed = serve.Server(workers=4, keep_outputs=True)
    rm = {r.rid: r for r in mixed.run_stream(reqs, [g * 0.002 for g in gaps])}
    mixed.close()
    assert all(not r.error for r in ra.values()) and all(not r.error for r in rm.values())
    rng = np.random.default_rng(0)
    for q in reqs:
        a, m = ra[q.rid].out.ravel(), rm[q.rid].out.ravel()
        tol = 1e-10 if ra[q.rid].precision else 1e-6
        assert rel_l2(m, a) <= tol, (q.rid, q.kind, q.eps)
        z = q.points
        if q.kind == "apply":
            rows = rng.integers(0, len(z), 64)
            ref = oracle.direct_sum(z, q.f, rows=rows)
            assert rel_l2(a[rows], ref) <= q.eps
            assert np.max(np.abs(a[rows] - ref)) <= 1.1 * q.eps / (2 * math.pi) * np.abs(q.f).sum()
        else:
            assert ra[q.rid].relres <= q.rtol
            ax = oracle.direct_sum(z, q.weights * a) + q.diag * a
            # the solve runs on an operator planned at min(eps, rtol)
            model = 1.1 * serve.plan_eps(q) / (2 * math.pi) * np.abs(q.weights * a).sum() * math.sqrt(len(a))
            assert np.linalg.norm(ax - q.b) <= 1.01 * q.rtol * np.linalg.norm(q.b) + model
    lat = serve.percentiles(list(rm.values()))
    assert lat["errors"] == 0 and lat["p50_ms"] > 0


def test_frees_during_graph_capture_leave_solves_intact():
    """Plans are freed on the reaper thread while GMRES solves on other workers capture their
    step graphs: with the device cache on, no release waits for the whole device, so no
    capture is broken (a device-wide wait during a capture fails the solve)."""
    device()
    lib()
    from paper_1711_07877_amd import serve
    reqs, _ = serve.make_stream(48, seed=11, nmin=5e3, nmax=2e5)
    print(f"serve: {len(reqs)} requests at once, twice, 4 workers", flush=True)
    import torch
    srv = serve.Server(workers=4)
    print(f"  free {torch.cuda.mem_get_info()[0] / 1e9:.1f} GB, admission budget {srv.budget.total / 1e9:.1f} GB",
          flush=True)
    try:
        for _ in range(2):
            res = srv.run_stream(reqs, None)
            errs = sorted({f"{r.kind} n={r.n} eps={r.eps}: {r.error}" for r in res if r.error})
            assert not errs, errs[:4]
    finally:
        srv.close()
