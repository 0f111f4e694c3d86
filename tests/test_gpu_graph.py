"""sbd_apply with a caller-provided workspace enqueues kernels only (no allocation, no
memset, no synchronisation), so it can be captured into a HIP graph and replayed.
Each replay, with other eager work and synchronisation in between, must reproduce the
eager result for the same input."""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_util import device, lib, rel_l2

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", [0, 1])
def test_apply_replays_from_hip_graph(precision):
    import torch
    pkg = lib()
    dev = device()
    z, f, spec = synth.make_workload("disk4k")
    dmin = oracle.default_delta_min(z, "ten", spec["eps"], area=math.pi)
    print(f"graph capture precision={precision}", flush=True)
    plan = pkg.sbd_plan(torch.tensor(z, device=dev), eps=spec["eps"], delta_min=dmin, precision=precision)
    ws = torch.empty(plan.workspace_bytes(1), dtype=torch.uint8, device=dev)
    ws2 = torch.empty_like(ws)
    fin = torch.tensor(f, device=dev)
    q = torch.empty_like(fin)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up outside the capture
        plan.apply(fin, out=q, workspace=ws, stream=side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.apply(fin, out=q, workspace=ws, stream=torch.cuda.current_stream())
    rng = np.random.default_rng(3)
    for it in range(4):
        fin.copy_(torch.tensor(rng.standard_normal(f.shape), device=dev))
        ref = plan.apply(fin.clone(), workspace=ws2)  # eager, own workspace
        torch.cuda.synchronize()
        q.zero_()
        g.replay()
        torch.cuda.synchronize()
        got = q.cpu().numpy()
        exp = ref.cpu().numpy()
        assert rel_l2(got, exp) <= (1e-12 if precision else 1e-6), it
    plan.free()
