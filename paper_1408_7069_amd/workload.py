"""Seeded synthetic inputs for the local ETKF frame.

This module only makes inputs: von Karman phase screens, the periodic
model-noise bank, true-phase sequences, measurement noise and the workload
definitions.  It holds none of the filter's arithmetic (no slope operator, no
forecast, no analysis) and imports neither the HIP library nor the oracle, so
both sides can be fed from it.

Phase screens: von Karman phase power spectrum
  Phi(f) = 0.023 r0^(-5/3) (f^2 + 1/L0^2)^(-11/6)   [rad^2 m^2]
sampled on a G x G periodic grid of spacing dx (G = 2x the node grid or more);
a screen is the real (or imaginary) part of the 2-D FFT of complex white noise
shaped by sqrt(Phi) df, df = 1/(G dx), with the zero frequency removed.  Each
pixel then has variance sum_f Phi(f) df^2.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np


def vk_psd(f2, r0: float, L0: float):
    """von Karman phase PSD at squared spatial frequency f2 (m^-2)."""
    return 0.023 * r0 ** (-5.0 / 3.0) * (f2 + 1.0 / (L0 * L0)) ** (-11.0 / 6.0)


def vk_screens(G: int, dx: float, r0: float, L0: float, n: int,
               rng: np.random.Generator) -> np.ndarray:
    """n independent periodic von Karman screens, (n, G, G) float64, rad."""
    f = np.fft.fftfreq(G, dx)
    fx, fy = np.meshgrid(f, f)
    psd = vk_psd(fx * fx + fy * fy, r0, L0)
    psd[0, 0] = 0.0
    amp = np.sqrt(psd) / (G * dx)
    out = np.empty((n, G, G))
    k = 0
    while k < n:
        c = (rng.standard_normal((G, G)) + 1j * rng.standard_normal((G, G))) * amp
        s = np.fft.fft2(c)
        out[k] = s.real
        if k + 1 < n:
            out[k + 1] = s.imag
        k += 2
    return out


def vk_covariance(G: int, dx: float, r0: float, L0: float) -> np.ndarray:
    """Exact covariance of the screens vk_screens draws, as a (G, G) table of
    periodic lags: each screen is the real (or imaginary) part of the FFT of
    complex white noise shaped by amp, so cov(s_p, s_q) = sum_f amp_f^2
    cos(2 pi f . (p - q)), the real FFT of amp^2."""
    f = np.fft.fftfreq(G, dx)
    fx, fy = np.meshgrid(f, f)
    psd = vk_psd(fx * fx + fy * fy, r0, L0)
    psd[0, 0] = 0.0
    amp2 = psd / (G * dx) ** 2
    return np.fft.fft2(amp2).real


def noise_bank(n_screens: int, side: int, pitch: float, r0: float, L0: float,
               a: float, rng: np.random.Generator) -> np.ndarray:
    """Model-noise bank (n_screens, side, side) float32: von Karman screens
    scaled by sqrt(1 - a^2), so that the AR(1) truth x <- a x + v keeps the
    von Karman statistics.  `side` must be a power of two."""
    assert side & (side - 1) == 0, "bank side must be a power of two"
    return (np.sqrt(1.0 - a * a) * vk_screens(side, pitch, r0, L0, n_screens, rng)).astype(np.float32)


def ar1_truth(n_sub: int, T: int, pitch: float, r0: float, L0: float, a: float,
              rng: np.random.Generator) -> np.ndarray:
    """(T, N+1, N+1) stationary AR(1) truth on the full node grid: a von Karman
    start and x_k = a x_{k-1} + sqrt(1-a^2) w_k with fresh von Karman w_k."""
    n1 = n_sub + 1
    G = 2 * n1
    x = vk_screens(G, pitch, r0, L0, 1, rng)[0, :n1, :n1]
    out = np.empty((T, n1, n1))
    q = np.sqrt(1.0 - a * a)
    k = 0
    while k < T:
        w = vk_screens(G, pitch, r0, L0, min(2, T - k), rng)
        for s in w:
            x = a * x + q * s[:n1, :n1]
            out[k] = x
            k += 1
    return out


def ar2_truth(n_sub: int, T: int, pitch: float, r0: float, L0: float, a1: float, a2: float,
              rng: np.random.Generator) -> np.ndarray:
    """(T, N+1, N+1) stationary AR(2) truth x_k = a1 x_{k-1} + a2 x_{k-2} + s w_k
    with fresh von Karman w_k, s the innovation scale that keeps the von
    Karman variance, started from two draws with the lag-1 correlation
    a1 / (1 - a2)."""
    n1 = n_sub + 1
    G = 2 * n1
    s = np.sqrt((1.0 + a2) * ((1.0 - a2) ** 2 - a1 * a1) / (1.0 - a2))
    r1 = a1 / (1.0 - a2)
    w = vk_screens(G, pitch, r0, L0, 2, rng)
    xm = w[0, :n1, :n1]
    x = r1 * xm + np.sqrt(1.0 - r1 * r1) * w[1, :n1, :n1]
    out = np.empty((T, n1, n1))
    k = 0
    while k < T:
        w = vk_screens(G, pitch, r0, L0, min(2, T - k), rng)
        for e in w:
            x, xm = a1 * x + a2 * xm + s * e[:n1, :n1], x
            out[k] = x
            k += 1
    return out


def frozen_flow_truth(n_sub: int, T: int, pitch: float, r0: float, L0: float,
                      layers, rate_hz: float, rng: np.random.Generator,
                      big: int = 512) -> np.ndarray:
    """(T, N+1, N+1) multi-layer frozen flow: each layer is a large periodic
    von Karman screen (weight w, wind (vx, vy) m/s) translated by v t with a
    Fourier phase ramp, summed with weights sqrt(w)."""
    n1 = n_sub + 1
    f = np.fft.fftfreq(big, 1.0)
    out = np.zeros((T, n1, n1))
    for w, vx, vy in layers:
        scr = vk_screens(big, pitch, r0, L0, 1, rng)[0]
        F = np.fft.fft2(scr)
        for k in range(T):
            sx = vx * k / rate_hz / pitch
            sy = vy * k / rate_hz / pitch
            ramp = np.exp(-2j * np.pi * (f[None, :] * sx + f[:, None] * sy))
            out[k] += np.sqrt(w) * np.fft.ifft2(F * ramp).real[:n1, :n1]
    return out


def reference_loop(seed: int = 2024, frames: int = 400):
    """The seeded loop on which the KF reference is compared (square 12 x 12
    SH, all (N+1)^2 nodes valid, a = 0.999, slope noise variance 0.04 rad^2 --
    the value of the paper's comparisons -- r0 0.15 m, pitch 0.4 m, L0 25 m):
    the truth grids (frames + 1, 13, 13), the slope noise (frames, p) and the
    parameters.  Used by the fixture script and the benchmark alike."""
    N, a, sigma, pitch, r0, L0 = 12, 0.999, 0.2, 0.4, 0.15, 25.0
    rng = np.random.default_rng(seed)
    truth = ar1_truth(N, frames + 1, pitch, r0, L0, a, rng)
    noise = gaussian_noise((frames, 2 * N * N), sigma, rng)
    return {"n_sub": N, "a": a, "sigma": sigma, "pitch": pitch, "r0": r0, "L0": L0, "burn_in": 100,
            "truth": truth, "noise": noise}


def gaussian_noise(shape, sigma, rng: np.random.Generator) -> np.ndarray:
    """Measurement noise w ~ N(0, sigma^2), float64."""
    return sigma * rng.standard_normal(shape)


@dataclass
class Workload:
    """One adaptive-optics instance of a benchmark or test workload."""
    name: str
    n_sub: int                    # N: N x N subapertures
    obscuration: float | None     # None = square pupil, else annulus ratio
    b: int                        # domain size (subapertures)
    h: int                        # halo (subapertures)
    m: int                        # ensemble size
    a: float                      # AR(1) coefficient of the filter
    rho: float                    # inflation
    sigma: float                  # slope noise std, rad per subaperture
    r0: float                     # Fried parameter (m)
    L0: float                     # outer scale (m)
    pitch: float                  # subaperture pitch (m)
    frames: int
    precision: str = "fp32"       # "fp32" (FP32 + FP64 eigensolve) or "fp64"
    taper_c: float = 0.0
    r_scale: float = 1.0
    seed: int = 0
    truth: str = "ar1"            # "ar1" or "frozen"
    extra: dict = field(default_factory=dict)


def workloads(index: int) -> list[Workload]:
    """The five workloads (list of instances), with seeds 1000 + index.

    0  8x8 square pupil, m=20, 2x2 domains, halo 1, FP64 everywhere, 100 frames.
    1  40x40, 14 % obscuration, m=50, 4x4 domains, frozen-flow truth
       (10 and 20 m/s at 500 Hz) against an AR(1) a=0.995 filter, 1000 frames.
    2  80x80, 28 % obscuration, m=64, 4x4 domains, halo 1, 500 frames.
    3  64 independent instances, N ~ U{16..48}, circular pupil, m in
       {32, 48, 64}, r0 ~ U[0.08, 0.2] m, sigma ~ U[0.05, 0.3] rad, 200 frames.
    4  as 2 with a Gaspari-Cohn taper (c = 2 pitches), T = 200 frames: the
       differentiable tuning run; a 12x12 copy serves the CPU gradient check.
    """
    seed = 1000 + index
    if index == 0:
        return [Workload("8x8 square m20", 8, None, 2, 1, 20, 0.99, 1.05, 0.1, 0.15, 25.0,
                         0.4, 100, "fp64", seed=seed)]
    if index == 1:
        return [Workload("40x40 eps0.14 m50", 40, 0.14, 4, 1, 50, 0.995, 1.05, 0.1, 0.12, 25.0,
                         0.4, 1000, seed=seed, truth="frozen",
                         extra={"layers": [(0.5, 10.0, 0.0), (0.5, 0.0, 20.0)], "rate_hz": 500.0})]
    if index == 2:
        return [Workload("80x80 eps0.28 m64", 80, 0.28, 4, 1, 64, 0.99, 1.05, 0.1, 0.15, 25.0,
                         0.5, 500, seed=seed)]
    if index == 3:
        rng = np.random.default_rng(seed)
        out = []
        for k in range(64):
            N = int(rng.integers(16, 49))
            m = int(rng.choice([32, 48, 64]))
            r0 = float(rng.uniform(0.08, 0.2))
            sig = float(rng.uniform(0.05, 0.3))
            out.append(Workload(f"inst{k} {N}x{N} m{m}", N, 0.0, 4, 1, m, 0.99, 1.05, sig, r0,
                                25.0, 0.5, 200, seed=seed * 100 + k))
        return out
    if index == 4:
        return [Workload("80x80 eps0.28 m64 taper", 80, 0.28, 4, 1, 64, 0.99, 1.05, 0.1, 0.15,
                         25.0, 0.5, 200, taper_c=2.0, seed=seed)]
    raise ValueError(f"no workload {index}")


def small_copy(w: Workload, n_sub: int = 12, frames: int | None = None) -> Workload:
    """The same physics on a smaller grid (e.g. the 12x12 gradient-check copy)."""
    return replace(w, name=f"{w.name} ({n_sub}x{n_sub} copy)", n_sub=n_sub,
                   frames=w.frames if frames is None else frames)


def truth_for(w: Workload, rng: np.random.Generator, frames: int | None = None) -> np.ndarray:
    """True phase on the full node grid for `frames` frames (default w.frames)."""
    T = w.frames if frames is None else frames
    if w.truth == "frozen":
        return frozen_flow_truth(w.n_sub, T, w.pitch, w.r0, w.L0, w.extra["layers"],
                                 w.extra["rate_hz"], rng)
    return ar1_truth(w.n_sub, T, w.pitch, w.r0, w.L0, w.a, rng)


def bank_for(w: Workload, rng: np.random.Generator, n_screens: int = 16) -> np.ndarray:
    """Model-noise bank sized for the instance's node grid."""
    side = 1
    while side < 2 * (w.n_sub + 1):
        side *= 2
    return noise_bank(n_screens, side, w.pitch, w.r0, w.L0, w.a, rng)
