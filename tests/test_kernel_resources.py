"""The kernels the apply can select use no scratch memory and spill no registers
(compiler resource-usage remarks recorded by the in-tree build)."""
import re

import pytest

from paper_1711_07877_amd import build


def _selectable(name: str) -> bool:
    # FFT passes: FP32 up to 24 elements per thread, FP64 up to 12 (the launcher refuses more)
    m = re.search(r"k_(?:fft_pass|rows_r2c|rows_c2r)I([fd])Li(\d+)E", name)
    if m:
        return int(m.group(2)) <= (24 if m.group(1) == "f" else 12)
    return bool(re.search(r"k_(spread|spread_fixedIf|interp_near|node_gather|near_|k_dot|gemv|reduce)", name)) or \
        any(k in name for k in ("k_dot_partials", "k_reduce_partials", "k_gemv_acc"))


def test_selectable_kernels_do_not_spill():
    res = build.kernel_resources()
    if not res:
        pytest.skip("no resource report (library not built in this tree)")
    checked = [k for k in res if _selectable(k)]
    assert len(checked) > 20
    bad = {k: v for k, v in res.items() if k in checked and (v.get("ScratchSize", 0) or v.get("VGPRs Spill", 0))}
    assert not bad, bad
