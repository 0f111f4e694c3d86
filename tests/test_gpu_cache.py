"""The large-block device cache (sbd_set_cache_limit): plans made while it holds blocks
released by earlier plans (temporaries at the end of sbd_plan, arrays at sbd_free) give
the same results as plans made with the cache off, across streams, and disabling it frees
what it holds."""
import numpy as np
import pytest

import synth
from gpu_util import device, lib, rel_l2

pytestmark = pytest.mark.gpu


def test_cached_blocks_give_the_same_applies():
    import torch
    pkg = lib()
    n = 200_000
    z = torch.tensor(synth.square_points(n, 901), device=device())
    f = torch.tensor(synth.real_rhs(n, 901), device=device())
    print("cache: reference plan with the cache off", flush=True)
    pkg.sbd_set_cache_limit(0)
    p0 = pkg.sbd_plan(z, eps=1e-6, precision=1)
    q0 = p0.apply(f).cpu().numpy()
    p0.free()
    try:
        pkg.sbd_set_cache_limit(8 << 30)
        streams = [torch.cuda.Stream(), torch.cuda.Stream()]
        for rep in range(4):
            s = streams[rep % 2]
            with torch.cuda.stream(s):
                p = pkg.sbd_plan(z, eps=1e-6, precision=1, stream=s)
                q = p.apply(f, stream=s)
            s.synchronize()
            held_before = pkg.sbd_cache_bytes()
            p.free()
            print(f"  pass {rep}: cache holds {held_before / 2**20:.0f} MiB in use-free state, "
                  f"{pkg.sbd_cache_bytes() / 2**20:.0f} MiB after free", flush=True)
            assert pkg.sbd_cache_bytes() > 0
            assert rel_l2(q.cpu().numpy(), q0) < 1e-13
    finally:
        pkg.sbd_set_cache_limit(0)
    assert pkg.sbd_cache_bytes() == 0
