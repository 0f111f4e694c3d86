"""Planted mistakes: each plausible error in the oracle must make a pin fail.

Mistakes are planted in the oracle on the CPU (monkeypatch), never in GPU code.
"""
import math

import numpy as np
import pytest
import scipy.special as sp
from scipy.integrate import quad

import oracle
import synth
from oracle import sbd_fit, sbd as osbd, nearfield


def _gram_quadrature_ok():
    rho, C = oracle.bessel_basis(5)
    A = sbd_fit.gram_matrix(rho, C, 0.3)
    f = lambda r: 2 * math.pi * C[0] * C[1] * rho[0] * rho[1] * r * sp.j1(rho[0] * r) * sp.j1(rho[1] * r)
    return abs(A[0, 1] - quad(f, 0.3, 1, epsabs=1e-14)[0]) < 1e-11


def _guarantee_ok(n=1200):
    z = synth.disk_points(n, 21)
    f = synth.real_rhs(n, 21)[0]
    eps = 1e-3
    dmin = math.sqrt(10 * math.pi / (math.pi * n))
    q = oracle.sbd_oracle(z, f, eps=eps, delta_min=dmin)
    qd = oracle.direct_sum(z, f)
    return np.max(np.abs(q - qd)) <= 1.1 * eps / (2 * math.pi) * np.abs(f).sum() and \
        np.linalg.norm(q - qd) / np.linalg.norm(qd) < eps


def test_unplanted_baseline_passes():
    assert _gram_quadrature_ok()
    assert _guarantee_ok()


def test_planted_gram_sign(monkeypatch):
    orig = sbd_fit._F
    monkeypatch.setattr(sbd_fit, "_F", lambda ri, rj, r: -orig(ri, rj, r))
    assert not _gram_quadrature_ok()


def test_planted_dropped_constant_node(monkeypatch):
    orig = osbd.frequencies

    def bad(*a, **k):
        xi, w, w0 = orig(*a, **k)
        return xi, w, 0.0
    monkeypatch.setattr(osbd, "frequencies", bad)
    assert not _guarantee_ok()


def test_planted_conjugate_transform(monkeypatch):
    """Using exp(+i) on both sides (a transposed/conjugated operand) breaks the far field."""
    def bad_far(z, f, c, xi, w, w0, block=2048):
        zc = np.asarray(z) - c
        E = np.exp(1j * (zc @ xi.T))
        return ((f @ E) * w[None, :]) @ E.T + w0 * np.sum(f, axis=1, keepdims=True)
    monkeypatch.setattr(osbd, "far_exact", bad_far)
    assert not _guarantee_ok()


def test_planted_scaling_garble(monkeypatch):
    """Reading 'J0(delta_max rho_p r)' literally instead of J0(rho_p r / delta_max)."""
    orig = osbd.frequencies

    def bad(fit, dmax, kind, eps, k=0.0):
        return orig(fit, 1.0 / dmax, kind, eps, k)[:2] + (orig(fit, dmax, kind, eps, k)[2],)
    monkeypatch.setattr(osbd, "frequencies", bad)
    assert not _guarantee_ok()


def test_planted_self_term_kept(monkeypatch):
    """Forgetting D_kk = -G_SBD(0) leaves the far field's self term in q."""
    orig = nearfield.near_values

    def bad(z, rows, cols, *a, **k):
        v = orig(z, rows, cols, *a, **k)
        return np.where(rows == cols, 0.0, v)
    monkeypatch.setattr(osbd, "near_values", bad)
    assert not _guarantee_ok()


def test_planted_too_few_nodes(monkeypatch):
    """Circles with M_p below rho_p violate the quadrature budget."""
    orig = sbd_fit.circle_sizes
    monkeypatch.setattr(sbd_fit, "circle_sizes", lambda x, c, e, P: np.maximum(2, (orig(x, c, e, P) * 0.6).astype(np.int64) // 2 * 2))
    assert not _guarantee_ok()
