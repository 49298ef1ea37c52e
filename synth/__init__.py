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
    "illumination_field", "poisson_rel_mad", "poisson_counts_per_unit", "SWEEP_UNIT_DF_MEAN", "SWEEP_LEVELS", "sweep_degradation",
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

    Two families.  Relative ones (``vignetting``, ``photons``, ``gauss_sigma_rel``,
    ``snp_prob``) are scaled by the stack maximum.  The noise model of Eq. (20) works in
    camera units instead: with ``unit_df_mean`` > 0 the stack is first scaled so that the
    dark-field images' mean readings have ``unit_df_mean`` as their harmonic mean, the
    per-image illumination field of strength ``illum_c`` multiplies each image, then
    Poisson noise (``poisson_nl_pct``), additive Gaussian noise (``gauss_abs``) and
    salt-and-pepper of density ``snp_density`` (salt = 1, the full-scale reading) are
    applied in those units, and the result is scaled back.

    Applied in this order: unit scaling, illumination field, radial vignetting, Poisson
    photon noise, additive Gaussian noise, salt-and-pepper, clipping at zero (a camera
    reads no negative intensity), scaling back.
    """
    vignetting: float = 0.0          # V(rho) = 1 - vignetting * (rho / rho_max)^2
    photons: float = 0.0             # photon count at the stack maximum (0: no Poisson noise)
    gauss_sigma_rel: float = 0.0     # Gaussian sigma as a fraction of the stack maximum
    snp_prob: float = 0.0            # salt-and-pepper probability per pixel (half 0, half max)
    unit_df_mean: float = 0.0        # > 0: camera units (harmonic mean of the dark-field mean readings)
    illum_c: float = 0.0             # Eq. 20's c: each image times (1 - c) + c u_n
    illum_waist_px: float = 15.0     # 1/e^2 radius of the Gaussian blur that makes u_n
    poisson_nl_pct: float = 0.0      # Poisson counts set for this Eq. 21 noise level (0: none)
    gauss_abs: float = 0.0           # Eq. 20's a for Gaussian noise, in camera units
    snp_density: float = 0.0         # Eq. 20's a for salt-and-pepper (half 0, half 1)


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


def illumination_field(rng: np.random.Generator, n: int, waist_px: float) -> np.ndarray:
    """u_n of Eq. (20): standard normal noise blurred (periodically) by a Gaussian of 1/e^2
    radius ``waist_px`` (std waist/2), min-max scaled to [0, 1]."""
    z = rng.standard_normal((n, n))
    f = np.fft.fftfreq(n)
    sig = waist_px / 2.0
    g = np.exp(-2.0 * (math.pi * sig) ** 2 * (f[:, None] ** 2 + f[None, :] ** 2))
    s = np.real(np.fft.ifft2(np.fft.fft2(z) * g))
    s -= s.min()
    m = s.max()
    return s / m if m > 0 else s


def poisson_rel_mad(mu: np.ndarray) -> np.ndarray:
    """E|X - mu| / mu for X ~ Poisson(mu), mu > 0: the mean absolute deviation of the
    Poisson law is 2 mu^(k+1) e^-mu / k! with k = floor(mu), so the ratio is
    2 mu^k e^-mu / k!, continuous and decreasing in mu (2 as mu -> 0)."""
    from scipy.special import gammaln
    mu = np.asarray(mu, dtype=np.float64)
    k = np.floor(mu)
    return 2.0 * np.exp(k * np.log(mu) - mu - gammaln(k + 1.0))


def poisson_counts_per_unit(images: np.ndarray, nl_pct: float) -> float:
    """Counts per camera unit s at which Poisson noise alone has expected Eq. 21 level
    nl_pct over ``images`` (readings in camera units): the mean over images of
    sum_p E|X_p - s r_p| / sum_p s r_p, X_p ~ Poisson(s r_p).  The mean is decreasing in
    s; bisection on a log scale."""
    target = nl_pct / 100.0
    r = np.asarray(images, dtype=np.float64).reshape(len(images), -1)
    tot = r.sum(axis=1)
    if not 0.0 < target < 2.0 or r.size == 0 or np.any(tot <= 0) or np.any(r < 0):
        raise ValueError("a Poisson noise level lies in (0, 200) % over non-negative, non-empty images")
    pos = r > 0

    def level(s):
        mu = s * r
        mad = np.where(pos, mu * poisson_rel_mad(np.where(pos, mu, 1.0)), 0.0)
        return float((mad.sum(axis=1) / (s * tot)).mean())

    lo, hi = 1e-6 / r.max(), 1e8 * r.shape[1] / tot.min()
    for _ in range(80):
        mid = math.sqrt(lo * hi)
        if level(mid) > target:
            lo = mid
        else:
            hi = mid
    return math.sqrt(lo * hi)


def degrade(clean: np.ndarray, spec: Degradation, seed: np.random.SeedSequence,
            dark: Optional[np.ndarray] = None) -> np.ndarray:
    """Corrupt a clean (K, n, n) intensity stack per ``spec``; returns float64.  ``dark``
    (a boolean per image) marks the dark-field images; camera units need it."""
    rng = np.random.default_rng(seed)
    img = np.array(clean, dtype=np.float64, copy=True)
    n = img.shape[-1]
    unit = 1.0
    if spec.unit_df_mean:
        if dark is None or not np.any(dark):
            raise ValueError("camera units need the dark-field images (dark)")
        means = img[np.asarray(dark, dtype=bool)].mean(axis=(1, 2))
        if np.any(means <= 0.0):
            raise ValueError("a dark-field image is empty")
        unit = spec.unit_df_mean * float(np.mean(1.0 / means))
        img *= unit
    if spec.illum_c:
        for k in range(img.shape[0]):
            img[k] *= (1.0 - spec.illum_c) + spec.illum_c * illumination_field(rng, n, spec.illum_waist_px)
    if spec.vignetting:
        c = (n - 1) / 2.0
        y, x = np.meshgrid(np.arange(n) - c, np.arange(n) - c, indexing="ij")
        rho = np.sqrt(x * x + y * y)
        img *= 1.0 - spec.vignetting * (rho / rho.max()) ** 2
    peak = float(img.max()) if img.size else 0.0
    if spec.photons and peak > 0:
        s = spec.photons / peak
        img = rng.poisson(np.clip(img, 0.0, None) * s).astype(np.float64) / s
    if spec.poisson_nl_pct:
        if not spec.unit_df_mean:
            raise ValueError("Poisson noise by level needs camera units")
        s = poisson_counts_per_unit(img[np.asarray(dark, dtype=bool)][:, ::4, ::4], spec.poisson_nl_pct)
        img = rng.poisson(np.clip(img, 0.0, None) * s).astype(np.float64) / s
    if spec.gauss_sigma_rel:
        img += rng.normal(0.0, spec.gauss_sigma_rel * peak, size=img.shape)
    if spec.gauss_abs:
        img += rng.normal(0.0, spec.gauss_abs, size=img.shape)
    if spec.snp_prob:
        u = rng.random(img.shape)
        img[u < spec.snp_prob / 2] = 0.0
        img[(u >= spec.snp_prob / 2) & (u < spec.snp_prob)] = peak
    if spec.snp_density:
        u = rng.random(img.shape)
        img[u < spec.snp_density / 2] = 0.0
        img[(u >= spec.snp_density / 2) & (u < spec.snp_density)] = 1.0
    img = np.clip(img, 0.0, None)
    return img / unit if unit != 1.0 else img


# Eq. (20)'s noise grid in camera units.  Table 1 prints the dark-field noise level of
# Eq. (21) per level.  Additive Gaussian noise of std a, clipped at zero, leaves a mean
# absolute error of a / sqrt(2 pi) on a dark pixel, and Table 1's Gaussian row grows as
# about 7.7e5 a percent, which puts the dark-field readings at about 5.2e-5 units (the
# harmonic mean of the images' mean readings, as Eq. 21 averages per-image ratios).
SWEEP_UNIT_DF_MEAN = 5.2e-5
SWEEP_LEVELS = {
    "gaussian": (1e-5, 1e-4, 1e-3, 1e-2),      # a, Table 1
    "snp": (1e-3, 1e-2, 1e-1, 2e-1),           # density a, Table 1
    "poisson": (36.37, 66.13, 81.07, 94.23),   # Lv 1-4: Table 1's noise level (%) at c = 0.25
}


def sweep_degradation(noise: str, level: int, c: float) -> Degradation:
    """Eq. (20) at Table 1's level ``level`` (0-3) of ``noise`` with illumination strength c.
    Poisson Lv n has no printed photon count: its counts per unit give Poisson noise alone,
    on the illuminated dark-field images (every fourth pixel in each direction), the
    expected noise level Table 1 prints for Lv n at c = 0.25."""
    if noise not in SWEEP_LEVELS:
        raise ValueError(f"unknown noise type {noise!r}")
    a = SWEEP_LEVELS[noise][level]
    kw = dict(unit_df_mean=SWEEP_UNIT_DF_MEAN, illum_c=c)
    if noise == "gaussian":
        return Degradation(gauss_abs=a, **kw)
    if noise == "snp":
        return Degradation(snp_density=a, **kw)
    return Degradation(poisson_nl_pct=a, **kw)


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
