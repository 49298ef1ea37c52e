"""Host metrics of the package (Eq. 21, 22) against closed forms and the oracle's copies."""
import math

import numpy as np

import oracle as orc
import synth
from paper_2209_14671_amd import metrics


def test_lsnr_closed_forms_and_offset_invariance():
    x = np.array([3.0, 4.0])
    assert metrics.lsnr(x + 5.0, x) == math.inf
    phi = x + np.array([1.0, -1.0])
    assert abs(metrics.lsnr(phi, x) - 10 * math.log10(25.0 / 2.0)) < 1e-12
    assert abs(metrics.lsnr(phi - 7.0, x) - metrics.lsnr(phi, x)) < 1e-12
    rng = np.random.default_rng(1)
    a, b = rng.random((16, 16)), rng.random((16, 16))
    assert abs(metrics.lsnr(a, b) - orc.lsnr(a, b)) < 1e-12


def test_noise_level_closed_forms():
    rng = np.random.default_rng(0)
    clean = rng.random((4, 5, 5)) + 0.1
    dark = np.array([True, False, True, True])
    assert metrics.noise_level(clean, clean, dark) == 0.0
    assert abs(metrics.noise_level(clean, clean * 1.5, np.ones(4, bool)) - 50.0) < 1e-12
    noisy = clean + rng.normal(0, 0.1, clean.shape)
    assert abs(metrics.noise_level(clean, noisy, dark) - orc.noise_level(clean, noisy, dark)) < 1e-12


def test_dark_field_split_of_the_config2_array():
    """15 x 15 LEDs, R = 40 px: the LEDs within 40 px of the axis (offsets of 17 px per
    grid step near the centre) are bright field; the 5 x 5 centre block and its neighbours
    inside the disc."""
    case = synth.config_case(2)
    o = case.optics
    dark = metrics.dark_field(case.led_k, o.n_lo, o.dx_lo_um, o.wavelength_um, o.na)
    prob = orc.problem_from_optics(o, case.led_k)
    off = orc.led_offsets(prob)
    ref = np.hypot(off[:, 0], off[:, 1]) > orc.pupil_radius_px(prob)
    assert np.array_equal(dark, ref)
    assert 0 < int((~dark).sum()) < 40 and dark.sum() > 180
