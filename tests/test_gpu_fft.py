"""GPU FFT kernels against numpy.fft (a library transform as the reference)."""
import numpy as np
import pytest

from gpu_util import device, lib

pytestmark = pytest.mark.gpu

SIZES = [(8, 8), (60, 84), (1050, 96), (96, 10240), (1176, 1050), (2100, 64), (8505, 40), (14336, 24)]


@pytest.mark.parametrize("shape", SIZES)
@pytest.mark.parametrize("prec", ["c64", "c128"])
@pytest.mark.parametrize("direction", [-1, 1])
def test_fft2_matches_numpy(shape, prec, direction):
    import torch
    dev = device()
    pkg = lib()
    print(f"fft2 shape={shape} prec={prec} dir={direction}", flush=True)
    rng = np.random.default_rng(hash(shape) % 1000)
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    dt = torch.complex64 if prec == "c64" else torch.complex128
    t = torch.tensor(x, dtype=dt, device=dev)
    pkg.sbd_fft2(t, direction)
    torch.cuda.synchronize()
    got = t.cpu().numpy()
    ref = np.fft.fft2(x) if direction < 0 else np.fft.ifft2(x) * x.size
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    tol = 2e-6 if prec == "c64" else 1e-13
    assert err < tol, err
