"""Sound cancelling on the GPU (Section 7, "Sound canceling"): the far-only two-set
Helmholtz applies give the objective and gradient of the phase optimisation to the
requested tolerance against dense Hankel sums, and a short L-BFGS run lowers the
intensity in the silence zone."""
import math

import numpy as np
import pytest
import scipy.special as sp

from gpu_util import device, lib

pytestmark = pytest.mark.gpu


def test_objective_and_gradient_match_dense_sums():
    device()
    lib()
    from paper_1711_07877_amd import sound
    scene = sound.make_scene(n_sources=100, q_points=20_000, wavenumber=90.0, seed=11)
    print("sound: plans", flush=True)
    prob = sound.SoundProblem(scene, eps=1e-6)
    d = np.hypot(scene.zone[:, None, 0] - scene.sources[None, :, 0], scene.zone[:, None, 1] - scene.sources[None, :, 1])
    A = sp.hankel1(0, scene.wavenumber * d)
    phi = np.random.default_rng(12).uniform(0, 2 * math.pi, 100)
    J, g = prob.objective_and_gradient(phi)
    Jd, gd = sound.objective_and_gradient(lambda u: A @ u, lambda v: A.conj().T @ v, phi)
    assert abs(J - Jd) <= 1e-5 * Jd
    assert np.max(np.abs(g - gd)) <= 1e-5 * np.max(np.abs(gd))
    prob.free()


def test_short_optimisation_lowers_zone_intensity():
    device()
    lib()
    from paper_1711_07877_amd import sound
    scene = sound.make_scene(n_sources=100, q_points=50_000, wavenumber=90.0, seed=13)
    prob = sound.SoundProblem(scene, eps=1e-6)
    phi0 = np.random.default_rng(14).uniform(0, 2 * math.pi, 100)
    print("sound: 60 evaluations", flush=True)
    phi, J0, J1, secs, nfev = prob.optimise(phi0, max_evaluations=60)
    assert nfev <= 61
    assert 10 * math.log10(J0 / J1) > 10.0
    prob.free()
