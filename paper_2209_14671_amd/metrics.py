"""Reconstruction-quality metrics of Sec. 4.1, on host arrays (evaluation only, not part
of the iteration): the linear-regressed SNR of Eq. (22) and the noise level of
Eq. (21) over the dark-field images."""
from __future__ import annotations

import math

import numpy as np


def lsnr(phi: np.ndarray, phi_true: np.ndarray) -> float:
    """Eq. (22): max over an additive constant b of 10 log10(||true||^2 / ||true - (phi + b)||^2).
    The maximising b is the mean of (true - phi)."""
    phi = np.asarray(phi, dtype=np.float64)
    phi_true = np.asarray(phi_true, dtype=np.float64)
    resid = phi_true - phi
    resid = resid - resid.mean()
    den = float(np.vdot(resid, resid).real)
    num = float(np.vdot(phi_true, phi_true).real)
    return math.inf if den == 0.0 else 10.0 * math.log10(num / den)


def dark_field(led_k: np.ndarray, n_lo: int, dx_lo_um: float, wavelength_um: float, na: float) -> np.ndarray:
    """LEDs whose illumination direction lies outside the objective's passband: the
    spectral offset round(k FOV) is farther from the centre than the pupil radius."""
    fov = n_lo * dx_lo_um
    off = np.sign(led_k * fov) * np.floor(np.abs(led_k * fov) + 0.5)
    return np.hypot(off[:, 0], off[:, 1]) > na * fov / wavelength_um


def noise_level(clean: np.ndarray, noisy: np.ndarray, dark: np.ndarray) -> float:
    """Eq. (21): mean over the dark-field images of ||clean - noisy||_1 / ||clean||_1, in percent."""
    idx = np.flatnonzero(dark)
    if idx.size == 0:
        return 0.0
    r = [np.abs(clean[k] - noisy[k]).sum() / np.abs(clean[k]).sum() for k in idx]
    return 100.0 * float(np.mean(r))
