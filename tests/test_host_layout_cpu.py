"""The plan's tile-edge rule (host C++, compiled here with g++ on its own): every chosen
edge is a power of two that covers the spreading kernel's pad, makes the fine near-field
cells at least delta_min wide (so the 3 x 3 cell search of the neighbour kernels misses no
close pair) and fits the LDS of the spread and interpolation workgroups; requests no edge
can meet are refused."""
import itertools
import json
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LDS = 160 * 1024
UNIT = 512


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("layout") / "layout_driver")
    subprocess.run(["g++", "-O2", "-std=c++17", "-o", exe, os.path.join(ROOT, "tests", "layout_driver.cpp"),
                    os.path.join(ROOT, "paper_1711_07877_amd", "csrc", "host", "layout.cpp")], check=True)
    return exe


def _run(exe, T, w, h, dmin, prec, lds=LDS, unit=UNIT):
    out = subprocess.run([exe, str(T), str(w), repr(h), repr(dmin), str(prec), str(lds), str(unit)], check=True,
                         capture_output=True, text=True)
    return json.loads(out.stdout)


def test_chosen_tiles_meet_every_rule(driver):
    for T, w, ratio, prec in itertools.product([0, 8, 16, 32, 64], [4, 7, 12, 16], [0.5, 2.0, 8.4, 20.0], [0, 1]):
        h = 1e-3
        r = _run(driver, T, w, h, ratio * h, prec)
        if r["rc"] != 0:
            assert r["rc"] == -6, r
            continue
        t = r["T"]
        assert t & (t - 1) == 0 and 8 <= t <= 256
        assert t >= (T if T else 32)
        assert t >= 2 * ((w + 1) // 2)
        assert t * h >= ratio * h
        assert max(r["spread_lds"], r["interp_lds"]) <= LDS


def test_small_user_tile_grows_until_cells_cover_delta_min(driver):
    # an 8-cell tile at 8.4 cells per delta_min (eps near the fit's floor) would make the fine
    # cells narrower than delta_min; the rule doubles the edge to 16
    r = _run(driver, 8, 7, 1.0, 8.4, 0)
    assert r["rc"] == 0 and r["T"] == 16


def test_requests_no_tile_can_meet_are_refused(driver):
    assert _run(driver, 12, 7, 1.0, 1.0, 0)["rc"] == -1                # not a power of two
    assert _run(driver, 512, 7, 1.0, 1.0, 0)["rc"] == -1               # above 256
    assert _run(driver, 32, 7, 1.0, 300.0, 0)["rc"] == -6              # delta_min beyond 256 cells
    assert _run(driver, 128, 7, 1.0, 1.0, 1)["rc"] == -6               # FP64 complex tile beyond 160 KB
    assert _run(driver, 128, 7, 1.0, 1.0, 0)["rc"] == 0                # FP32 fits
