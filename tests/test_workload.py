"""Statistics of the synthetic von Karman inputs (loose, statistical pins)."""
import numpy as np
from scipy import integrate, special

from paper_1408_7069_amd import workload as wl


def test_psd_constant_gives_kolmogorov_structure_function():
    # D(r) = 2 int Phi(f) (1 - J0(2 pi f r)) 2 pi f df -> 6.88 (r/r0)^(5/3)
    r0, r = 0.15, 0.3
    f = lambda q: wl.vk_psd(q * q, r0, 1e9) * (1 - special.j0(2 * np.pi * q * r)) * 2 * np.pi * q
    val = 2 * sum(integrate.quad(f, a, b_, limit=400)[0]
                  for a, b_ in [(0, 1e-3), (1e-3, 1), (1, 100), (100, 1e4)])
    assert abs(val / (6.88 * (r / r0) ** (5 / 3)) - 1) < 0.01


def test_screens_have_the_discrete_spectrum_expectation():
    # for a periodic FFT screen, E[(s(x+k) - s(x))^2] = 2 sum Phi df^2 (1 - cos 2 pi fx k dx)
    rng = np.random.default_rng(0)
    G, dx, r0, L0 = 128, 0.1, 0.2, 25.0
    s = wl.vk_screens(G, dx, r0, L0, 64, rng)
    f = np.fft.fftfreq(G, dx)
    fx, fy = np.meshgrid(f, f)
    psd = wl.vk_psd(fx * fx + fy * fy, r0, L0)
    psd[0, 0] = 0
    df = 1.0 / (G * dx)
    for k in (1, 3, 10, 40):
        expect = 2 * np.sum(psd * df * df * (1 - np.cos(2 * np.pi * fx * k * dx)))
        got = np.mean((np.roll(s, -k, axis=2) - s) ** 2)
        assert abs(got / expect - 1) < 0.05, (k, got, expect)


def test_bank_scaling_and_workloads():
    rng = np.random.default_rng(1)
    b = wl.noise_bank(8, 64, 0.5, 0.15, 25.0, 0.99, rng)
    assert b.dtype == np.float32 and b.shape == (8, 64, 64)
    raw = wl.vk_screens(64, 0.5, 0.15, 25.0, 8, np.random.default_rng(1))
    assert np.allclose(b, np.sqrt(1 - 0.99 ** 2) * raw, rtol=1e-6, atol=1e-6)
    w = wl.workloads(2)[0]
    assert (w.n_sub, w.m, w.b, w.h) == (80, 64, 4, 1)
    assert len(wl.workloads(3)) == 64
