"""Seeded synthetic Fourier-ptychography inputs.

This module is shared by the CPU oracle, the tests and the benchmark.  It holds
only data generation: random object fields, the simulated microscope's LED
geometry and true pupil, and the measurement degradations.  It contains none of
the reconstruction method's arithmetic: it does not crop spectra, run the
forward model, or compute losses and gradients.  Clean intensity stacks are made
by whichever side (oracle or GPU library) needs them, from the ground truth
returned here.

Physical model of the simulated setup (paper Sec. 4.1 describes the same kind of
setup: an LED array under the sample, a low-NA objective, a camera):

* camera pixel ``pixel_um`` behind a ``mag`` objective gives a sample-plane pixel
  ``dx_lo = pixel_um / mag``; the low-resolution image is ``n_lo`` pixels wide,
  so the field of view is ``FOV = n_lo * dx_lo`` micrometres;
* the high-resolution object is ``n_hi = upsample * n_lo`` pixels over the same
  field of view;
* LED ``(ix, iy)`` of a square grid with pitch ``pitch_mm`` sits ``height_mm``
  below the sample; its illumination wave-vector is ``(kx, ky) = sin(theta)/lambda``
  in cycles per micrometre.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

__all__ = [
    "Optics", "Degradation", "Case", "smooth_field", "make_object", "led_grid_positions",
    "led_wavevectors", "true_pupil", "degrade", "make_case", "config_case", "config3_tiles", "centre_subgrid",
]


@dataclasses.dataclass(frozen=True)
class Optics:
    """Simulated microscope and LED array geometry."""
    n_lo: int = 32
    upsample: int = 4
    wavelength_um: float = 0.52
    na: float = 0.1
    mag: float = 4.0
    pixel_um: float = 6.5
    led_grid: int = 5            # LEDs per side of the square array
    pitch_mm: float = 4.0
    height_mm: float = 90.0

    @property
    def n_hi(self) -> int:
        return self.n_lo * self.upsample

    @property
    def dx_lo_um(self) -> float:
        return self.pixel_um / self.mag

    @property
    def n_led(self) -> int:
        return self.led_grid * self.led_grid


@dataclasses.dataclass(frozen=True)
class Degradation:
    """Measurement corruptions applied to a clean intensity stack (all optional).

    Applied in this order: radial vignetting, Poisson photon noise, additive
    Gaussian noise, salt-and-pepper, clipping at zero.
    """
    vignetting: float = 0.0          # V(rho) = 1 - vignetting * (rho / rho_max)^2
    photons: float = 0.0             # photon count at the stack maximum (0: no Poisson noise)
    gauss_sigma_rel: float = 0.0     # Gaussian sigma as a fraction of the stack maximum
    snp_prob: float = 0.0            # salt-and-pepper probability per pixel (half 0, half max)


@dataclasses.dataclass
class Case:
    """One synthetic reconstruction problem (ground truth + geometry + noise recipe)."""
    optics: Optics
    obj: np.ndarray                  # complex128 (n_hi, n_hi) ground-truth object field
    pupil: np.ndarray                # complex128 (n_lo, n_lo) true pupil of the simulated optics
    led_k: np.ndarray                # float64 (K, 2) nominal (kx, ky) used by reconstruction
    led_k_true: np.ndarray           # float64 (K, 2) wave-vectors used to simulate the data
    degradation: Degradation
    noise_seed: np.random.SeedSequence


def smooth_field(rng: np.random.Generator, n: int, sigma_px: float) -> np.ndarray:
    """U(0,1) noise smoothed by a periodic Gaussian of std ``sigma_px``, min-max scaled to [0,1]."""
    u = rng.random((n, n))
    f = np.fft.fftfreq(n)
    g = np.exp(-2.0 * (math.pi * sigma_px) ** 2 * (f[:, None] ** 2 + f[None, :] ** 2))
    s = np.real(np.fft.ifft2(np.fft.fft2(u) * g))
    s -= s.min()
    m = s.max()
    return s / m if m > 0 else s


def make_object(rng: np.random.Generator, n_hi: int, sigma_px: float = 3.0,
                amp_range=(0.2, 1.0), phase_range=(-math.pi / 2, math.pi / 2)) -> np.ndarray:
    """Complex object: smoothed amplitude in ``amp_range`` times exp(i * smoothed phase)."""
    a = amp_range[0] + (amp_range[1] - amp_range[0]) * smooth_field(rng, n_hi, sigma_px)
    p = phase_range[0] + (phase_range[1] - phase_range[0]) * smooth_field(rng, n_hi, sigma_px)
    return a * np.exp(1j * p)


def led_grid_positions(grid: int, pitch_mm: float) -> np.ndarray:
    """(K, 2) LED (x, y) positions in mm, row-major over y then x, centre LED at the origin."""
    idx = np.arange(grid) - (grid - 1) / 2.0
    yy, xx = np.meshgrid(idx, idx, indexing="ij")
    return np.stack([xx.ravel(), yy.ravel()], axis=1) * pitch_mm


def led_wavevectors(pos_mm: np.ndarray, height_mm: float, wavelength_um: float) -> np.ndarray:
    """(K, 2) illumination wave-vectors (kx, ky) = sin(theta_x, theta_y) / lambda in 1/um."""
    x, y = pos_mm[:, 0], pos_mm[:, 1]
    r = np.sqrt(x * x + y * y + height_mm * height_mm)
    return np.stack([x / r, y / r], axis=1) / wavelength_um


def centre_subgrid(grid: int, sub: int) -> np.ndarray:
    """Indices (row-major) of the centred ``sub x sub`` block of a ``grid x grid`` LED array."""
    lo = (grid - sub) // 2
    ii = [(lo + r) * grid + (lo + c) for r in range(sub) for c in range(sub)]
    return np.asarray(ii, dtype=np.int64)


def true_pupil(optics: Optics, zernike_rad: Optional[np.ndarray] = None) -> np.ndarray:
    """Pupil of the simulated objective: a disc of radius NA*FOV/lambda pixels, centred at
    (n_lo/2, n_lo/2), optionally with a phase of Noll-normalised Zernike modes
    Z4 (defocus), Z5, Z6 (astigmatism) whose coefficients are given in radians."""
    n = optics.n_lo
    fov = n * optics.dx_lo_um
    radius = optics.na * fov / optics.wavelength_um
    c = n // 2
    y, x = np.meshgrid(np.arange(n) - c, np.arange(n) - c, indexing="ij")
    d2 = (x * x + y * y).astype(np.float64)
    inside = d2 <= radius * radius * (1.0 + 1e-12)
    p = inside.astype(np.complex128)
    if zernike_rad is not None:
        rho2 = d2 / (radius * radius)
        th = np.arctan2(y, x)
        z4 = math.sqrt(3.0) * (2.0 * rho2 - 1.0)
        z5 = math.sqrt(6.0) * rho2 * np.sin(2.0 * th)
        z6 = math.sqrt(6.0) * rho2 * np.cos(2.0 * th)
        ph = zernike_rad[0] * z4 + zernike_rad[1] * z5 + zernike_rad[2] * z6
        p = p * np.exp(1j * ph)
    return p


def degrade(clean: np.ndarray, spec: Degradation, seed: np.random.SeedSequence) -> np.ndarray:
    """Corrupt a clean (K, n, n) intensity stack per ``spec``; returns float64."""
    rng = np.random.default_rng(seed)
    img = np.array(clean, dtype=np.float64, copy=True)
    n = img.shape[-1]
    if spec.vignetting:
        c = (n - 1) / 2.0
        y, x = np.meshgrid(np.arange(n) - c, np.arange(n) - c, indexing="ij")
        rho = np.sqrt(x * x + y * y)
        img *= 1.0 - spec.vignetting * (rho / rho.max()) ** 2
    peak = float(img.max()) if img.size else 0.0
    if spec.photons and peak > 0:
        s = spec.photons / peak
        img = rng.poisson(np.clip(img, 0.0, None) * s).astype(np.float64) / s
    if spec.gauss_sigma_rel:
        img += rng.normal(0.0, spec.gauss_sigma_rel * peak, size=img.shape)
    if spec.snp_prob:
        u = rng.random(img.shape)
        img[u < spec.snp_prob / 2] = 0.0
        img[(u >= spec.snp_prob / 2) & (u < spec.snp_prob)] = peak
    return np.clip(img, 0.0, None)


def make_case(optics: Optics, seed, *, zernike_std: float = 0.0, jitter_mm: float = 0.0,
              degradation: Degradation = Degradation(), led_subset: Optional[np.ndarray] = None) -> Case:
    """Build a seeded synthetic case. ``seed`` is anything SeedSequence accepts."""
    ss = np.random.SeedSequence(seed)
    s_obj, s_pup, s_noise, s_jit = ss.spawn(4)
    obj = make_object(np.random.default_rng(s_obj), optics.n_hi)
    z = None
    if zernike_std:
        z = np.random.default_rng(s_pup).normal(0.0, zernike_std, size=3)
    pupil = true_pupil(optics, z)
    pos = led_grid_positions(optics.led_grid, optics.pitch_mm)
    if led_subset is not None:
        pos = pos[led_subset]
    k_nom = led_wavevectors(pos, optics.height_mm, optics.wavelength_um)
    if jitter_mm:
        pos_j = pos + np.random.default_rng(s_jit).normal(0.0, jitter_mm, size=pos.shape)
        k_true = led_wavevectors(pos_j, optics.height_mm, optics.wavelength_um)
    else:
        k_true = k_nom.copy()
    return Case(optics, obj, pupil, k_nom, k_true, degradation, s_noise)


# The five workload presets: sizes, optics and corruptions.
_CONFIG_OPTICS = {
    1: Optics(n_lo=32, upsample=4, led_grid=5),
    2: Optics(n_lo=128, upsample=4, led_grid=15),
    4: Optics(n_lo=64, upsample=4, led_grid=11),
    5: Optics(n_lo=256, upsample=4, led_grid=15),
}

CONFIG_ITERS = {1: 50, 2: 100, 3: 100, 4: 1, 5: 100}


# Batched-tile preset: low-res sizes and LED sub-grids drawn per tile.
CONFIG3_SIZES = (64, 96, 128, 192, 256)
CONFIG3_SUBGRIDS = (7, 11, 13, 15)  # K = 49, 121, 169, 225: centred blocks of the 15 x 15 array


def config3_tiles(n_tiles: int = 64) -> list:
    """Independent seeded tiles of the batched workload: n_lo drawn uniformly from
    CONFIG3_SIZES (n_hi = 4 n_lo), the LEDs a centred sub-grid drawn from CONFIG3_SUBGRIDS,
    circular pupil, noise-free, each with its own object."""
    rng = np.random.default_rng(np.random.SeedSequence([3]))
    sizes = rng.choice(CONFIG3_SIZES, size=n_tiles)
    subs = rng.choice(CONFIG3_SUBGRIDS, size=n_tiles)
    tiles = []
    for t in range(n_tiles):
        optics = Optics(n_lo=int(sizes[t]), upsample=4, led_grid=15)
        tiles.append(make_case(optics, [3, t], led_subset=centre_subgrid(15, int(subs[t]))))
    return tiles


def config_case(config_id: int, tile_id: int = 0) -> Case:
    """Synthetic case for workload ``config_id`` (1, 2, 4 or 5; tile presets use ``make_case``)."""
    if config_id == 2:
        deg = Degradation(vignetting=0.5, photons=1e3, gauss_sigma_rel=1e-2, snp_prob=1e-3)
        return make_case(_CONFIG_OPTICS[2], [2, tile_id], zernike_std=0.5, jitter_mm=0.5,
                         degradation=deg)
    if config_id in (1, 4, 5):
        return make_case(_CONFIG_OPTICS[config_id], [config_id, tile_id])
    raise ValueError(f"no single-FOV preset for config {config_id}")
