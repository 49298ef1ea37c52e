"""Small seeded problems shared by the tests (no method arithmetic here)."""
import numpy as np

import synth


def small_optics(n_lo=8, upsample=2, grid=3, na=0.15, pitch_mm=4.0):
    return synth.Optics(n_lo=n_lo, upsample=upsample, na=na, led_grid=grid, pitch_mm=pitch_mm)


def rand_complex(rng, shape, scale=1.0):
    return scale * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)


def smooth_object(seed, n_hi, amp=(0.5, 1.0), phase=(-1.0, 1.0)):
    """A smooth object whose phase stays well inside (-pi, pi)."""
    rng = np.random.default_rng(seed)
    return synth.make_object(rng, n_hi, sigma_px=1.5, amp_range=amp, phase_range=phase)


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))
