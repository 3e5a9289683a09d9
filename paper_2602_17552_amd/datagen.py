"""Seeded synthetic scalar fields (float32, C order) for tests and benchmarks.

The paper evaluates on CESM climate fields (Section V-A, datasets table) that
are not available here; these generators stand in for them with the shapes,
value ranges and roughness of the workloads the benchmark names.  Nothing in
this module computes any part of the compression method: it only draws
numbers.  All generation is elementwise float64 numpy (no BLAS reductions), so
a given seed gives the same bytes on any host with the same numpy.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "gaussian_bumps_2d",
    "sinusoids_2d",
    "grf_3d",
    "noise",
    "checker_2d",
    "checker_3d",
    "climate_stand_in",
    "CLIMATE_SHAPES",
    "cfg0",
    "cfg1",
    "cfg2",
    "batch_fields",
    "serve_trace",
]


def gaussian_bumps_2d(ny: int, nx: int, nbumps: int = 40, seed: int = 0,
                      noise_sd: float = 1e-3, sigma_lo: float = 8.0,
                      sigma_hi: float = 40.0) -> np.ndarray:
    """Sum of `nbumps` isotropic Gaussian bumps plus N(0, noise_sd^2) noise.

    Centres uniform over the grid, amplitudes U[-1, 1], widths U[sigma_lo,
    sigma_hi] pixels.
    """
    rng = np.random.default_rng(seed)
    y = np.arange(ny, dtype=np.float64)[:, None]
    x = np.arange(nx, dtype=np.float64)[None, :]
    f = np.zeros((ny, nx), dtype=np.float64)
    cy = rng.uniform(0.0, ny, nbumps)
    cx = rng.uniform(0.0, nx, nbumps)
    amp = rng.uniform(-1.0, 1.0, nbumps)
    sig = rng.uniform(sigma_lo, sigma_hi, nbumps)
    for k in range(nbumps):
        gy = np.exp(-((y - cy[k]) ** 2) / (2.0 * sig[k] ** 2))
        gx = np.exp(-((x - cx[k]) ** 2) / (2.0 * sig[k] ** 2))
        f += amp[k] * (gy * gx)
    f += rng.normal(0.0, noise_sd, (ny, nx))
    return np.ascontiguousarray(f.astype(np.float32))


def sinusoids_2d(ny: int, nx: int, nwaves: int = 64, seed: int = 1,
                 noise_sd: float = 1e-2, kmax: int = 32) -> np.ndarray:
    """Climate-grid-like field: sum of random plane waves in (lat, lon).

    Each wave is A sin(2 pi (kx x / nx + ky y / ny) + phi) with integer
    wavenumbers kx, ky uniform in [1, kmax], phase uniform in [0, 2 pi) and
    amplitude A = (kx^2 + ky^2)^(-3/4), i.e. |k|^(-1.5); plus N(0, noise_sd^2).
    """
    rng = np.random.default_rng(seed)
    y = np.arange(ny, dtype=np.float64)[:, None] / ny
    x = np.arange(nx, dtype=np.float64)[None, :] / nx
    f = np.zeros((ny, nx), dtype=np.float64)
    for _ in range(nwaves):
        kx, ky = rng.integers(1, kmax + 1, 2)
        phi = rng.uniform(0.0, 2.0 * math.pi)
        amp = float(kx * kx + ky * ky) ** -0.75
        a = 2.0 * math.pi * kx * x + phi
        b = 2.0 * math.pi * ky * y
        # sin(a + b) expanded so each term is an outer product (elementwise).
        f += amp * (np.sin(a) * np.cos(b) + np.cos(a) * np.sin(b))
    f += rng.normal(0.0, noise_sd, (ny, nx))
    return np.ascontiguousarray(f.astype(np.float32))


def grf_3d(n0: int, n1: int, n2: int, seed: int = 2,
           slope: float = -5.0 / 3.0) -> np.ndarray:
    """Gaussian random field with power spectrum ~ |k|^slope, scaled to [0, 1].

    White noise is transformed with a real FFT, multiplied by sqrt(P(|k|))
    with P(0) = 0, transformed back and min-max normalised.
    """
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((n0, n1, n2))
    spec = np.fft.rfftn(w, axes=(0, 1, 2))
    k0 = np.fft.fftfreq(n0)[:, None, None]
    k1 = np.fft.fftfreq(n1)[None, :, None]
    k2 = np.fft.rfftfreq(n2)[None, None, :]
    k = np.sqrt(k0 * k0 + k1 * k1 + k2 * k2)
    k[0, 0, 0] = 1.0
    amp = k ** (0.5 * slope)
    amp[0, 0, 0] = 0.0
    f = np.fft.irfftn(spec * amp, s=(n0, n1, n2), axes=(0, 1, 2))
    lo, hi = f.min(), f.max()
    f = (f - lo) / (hi - lo) if hi > lo else np.zeros_like(f)
    return np.ascontiguousarray(f.astype(np.float32))


def noise(shape, seed: int = 0, dist: str = "normal") -> np.ndarray:
    """i.i.d. noise field (normal or uniform) for statistics and edge tests."""
    rng = np.random.default_rng(seed)
    if dist == "uniform":
        f = rng.uniform(-1.0, 1.0, shape)
    else:
        f = rng.standard_normal(shape)
    return np.ascontiguousarray(np.asarray(f, dtype=np.float32))


# Named workloads --------------------------------------------------------------

def checker_2d(ny: int, nx: int, seed: int = 0, a: float = 1.0, b: float = 0.7,
               noise_sd: float = 0.5, ramp: float = 0.05) -> np.ndarray:
    """a(-1)^x - b(-1)^y on vertical bands (where sin(x/5) > -0.3), plus a
    ramp 0.05 x and N(0, noise_sd^2) noise: dense alternating extrema and
    saddles whose neighbourhoods overlap."""
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    base = a * (-1.0) ** x - b * (-1.0) ** y
    f = base * (np.sin(x / 5.0) > -0.3) + noise_sd * rng.standard_normal((ny, nx)) + ramp * x
    return f.astype(np.float32)


def checker_3d(n0: int, n1: int, n2: int, seed: int = 0, noise_sd: float = 0.2) -> np.ndarray:
    """(-1)^x - 0.6(-1)^y + 0.3(-1)^z plus N(0, noise_sd^2) noise."""
    rng = np.random.default_rng(seed)
    z, y, x = np.mgrid[0:n0, 0:n1, 0:n2].astype(np.float64)
    f = (-1.0) ** x - 0.6 * (-1.0) ** y + 0.3 * (-1.0) ** z + noise_sd * rng.standard_normal((n0, n1, n2))
    return f.astype(np.float32)


# Grid shapes of the five CESM datasets of the paper's evaluation
# (Section V-A, datasets table).
CLIMATE_SHAPES = {"ATM": (1800, 3600), "CLIMATE": (768, 1152), "ICE": (384, 320),
                  "LAND": (192, 288), "OCEAN": (384, 320)}


def climate_stand_in(name: str, seed: int = 0) -> np.ndarray:
    """A field shaped like one of the paper's CESM datasets: 64 plane waves
    (amplitude |k|^-1.5) plus N(0, 1e-2^2) noise, min-max normalised to
    [0, 1] so that absolute bounds of 1e-3..1e-5 are relative to the range."""
    ny, nx = CLIMATE_SHAPES[name]
    f = sinusoids_2d(ny, nx, 64, seed=1000 + 17 * seed + len(name), noise_sd=1e-2).astype(np.float64)
    lo, hi = float(f.min()), float(f.max())
    return ((f - lo) / (hi - lo)).astype(np.float32)


def cfg0() -> np.ndarray:
    """512 x 512, 40 Gaussian bumps + N(0, 1e-3^2) noise, seed 0."""
    return gaussian_bumps_2d(512, 512, 40, seed=0, noise_sd=1e-3)


def cfg1() -> np.ndarray:
    """1800 x 3600 (ATM-shaped lat x lon), 64 sinusoids + N(0, 1e-2^2), seed 1."""
    return sinusoids_2d(1800, 3600, 64, seed=1, noise_sd=1e-2)


def cfg2() -> np.ndarray:
    """256^3 turbulence-like Gaussian random field, |k|^(-5/3), in [0, 1], seed 2."""
    return grf_3d(256, 256, 256, seed=2)


def _loguniform_int(rng, lo: int, hi: int) -> int:
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def batch_fields(count2d: int = 48, count3d: int = 16, seed: int = 3,
                 side2d=(128, 2048), side3d=(32, 192), scale: float = 1.0):
    """Uneven batch: 2D bump fields and 3D random fields with random bounds.

    Returns a list of (field, rel_eb).  2D sides (each axis drawn separately)
    are log-uniform in `side2d`, 3D sides in `side3d`; `scale` shrinks every
    side (for quick tests).  Bounds are drawn from {1e-2, 1e-3, 1e-4}.
    """
    rng = np.random.default_rng(seed)
    out = []
    kinds = ["2d"] * count2d + ["3d"] * count3d
    order = rng.permutation(len(kinds))
    for j in order:
        eb = float(rng.choice([1e-2, 1e-3, 1e-4]))
        sub = int(rng.integers(0, 2 ** 31 - 1))
        if kinds[j] == "2d":
            ny = max(2, int(_loguniform_int(rng, *side2d) * scale))
            nx = max(2, int(_loguniform_int(rng, *side2d) * scale))
            nb = max(4, int(40 * ny * nx / (512 * 512)))
            nb = min(nb, 400)
            s = max(ny, nx) / 512.0
            f = gaussian_bumps_2d(ny, nx, nb, seed=sub, noise_sd=1e-3,
                                  sigma_lo=max(2.0, 8.0 * s),
                                  sigma_hi=max(4.0, 40.0 * s))
        else:
            n = [max(2, int(_loguniform_int(rng, *side3d) * scale)) for _ in range(3)]
            f = grf_3d(n[0], n[1], n[2], seed=sub)
        out.append((f, eb))
    return out


def serve_trace(rate: float = 200.0, duration: float = 60.0,
                frac_compress: float = 0.7, seed: int = 4):
    """Poisson arrival trace: list of (arrival_time_s, op) with op in
    {"compress", "decompress"} drawn 70/30 by default."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= duration:
            break
        op = "compress" if rng.uniform() < frac_compress else "decompress"
        out.append((t, op))
    return out
