"""Host-side pieces of bench.py (no GPU): the one-GPU refusal, the accuracy check's direct
sum against the oracle's, and the stored-traffic lookup."""
import math
import os
import subprocess
import sys

import numpy as np

import bench
import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)
    assert r.stdout.strip() == "" or not r.stdout.strip().startswith("{")


def test_accuracy_rows_match_the_oracle_direct_sum():
    # bench.direct_rows is the bench's own exact sum (the self pair dropped by distance); the
    # oracle's direct_sum drops it by index: on distinct points they agree to rounding
    z = synth.disk_points(600, 31)
    f = synth.real_rhs(600, 32)[0]
    rows = np.arange(0, 600, 37)
    got = bench.direct_rows(z, z, f, rows)
    ref = oracle.direct_sum(z, f, rows=rows)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    # Helmholtz, complex f
    fc = synth.complex_rhs(600, 33)[0]
    k = 2 * math.pi * 5
    got = bench.direct_rows(z, z, fc, rows, kernel="helmholtz", wavenumber=k)
    ref = oracle.direct_sum(z, fc, kind="helmholtz", wavenumber=k, rows=rows)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_stored_traffic_lookup():
    assert bench.stored_traffic("interp_near", "no-such-workload", 0, 1) is None
    assert bench.stored_traffic("no-such-kernel", "square10m", 0, 1) is None


def test_host_threads_bounds():
    assert 1 <= bench.host_threads() <= 16
