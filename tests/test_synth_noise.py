"""The Eq. (20) noise model of the sweep's inputs (CPU): closed forms of each corruption in
camera units, and Table 1's Gaussian row reproduced on a synthetic stack."""
import math

import numpy as np
import pytest

import oracle as orc
import synth
from paper_2209_14671_amd import metrics


def test_poisson_relative_mad_matches_the_pmf_sum():
    """2 mu^k e^-mu / k! (k = floor mu) against E|X - mu| / mu summed over the pmf."""
    for mu in (0.05, 0.7, 1.0, 1.5, 2.999, 4.8, 20.0, 150.0):
        x = np.arange(0, int(mu + 40 * math.sqrt(mu) + 40))
        logp = x * math.log(mu) - mu - np.array([math.lgamma(v + 1.0) for v in x])
        brute = float(np.sum(np.exp(logp) * np.abs(x - mu))) / mu
        assert abs(float(synth.poisson_rel_mad(mu)) - brute) < 1e-10 * max(1.0, brute), mu


def test_poisson_counts_reach_the_level_on_uniform_images():
    """Uniform images: the solved counts put E|X - mu|/mu on the target, and a large draw
    measures that level (Eq. 21) within sampling error."""
    r = np.full((3, 64, 64), 2e-5)
    r[1] *= 3.0
    for nl in (36.37, 81.07, 94.23):
        s = synth.poisson_counts_per_unit(r, nl)
        lvl = float(np.mean([synth.poisson_rel_mad(s * v) for v in (2e-5, 6e-5, 2e-5)]))
        assert abs(lvl - nl / 100.0) < 1e-9
    clean = np.full((2, 256, 256), 1.0)
    dark = np.array([True, True])
    deg = synth.Degradation(unit_df_mean=3e-5, poisson_nl_pct=66.13)
    noisy = synth.degrade(clean, deg, np.random.SeedSequence(1), dark=dark)
    assert abs(metrics.noise_level(clean, noisy, dark) - 66.13) < 1.0


def test_camera_units_scale_back_and_take_the_harmonic_mean():
    rng = np.random.default_rng(0)
    clean = rng.random((4, 16, 16)) + 0.1
    dark = np.array([False, True, True, True])
    out = synth.degrade(clean, synth.Degradation(unit_df_mean=5.2e-5), np.random.SeedSequence(2), dark=dark)
    assert np.allclose(out, clean, rtol=1e-14, atol=0)
    with pytest.raises(ValueError):
        synth.degrade(clean, synth.Degradation(unit_df_mean=5.2e-5), np.random.SeedSequence(2))


def test_clipped_gaussian_noise_level_closed_form():
    """Dark images of constant reading x_k (harmonic mean m in camera units), additive
    N(0, a^2) clipped at zero: E|max(x + n, 0) - x| = a (2 phi(0) - phi(x/a)) + x Phi(-x/a),
    so Eq. 21 gives the mean over k of that divided by x_k."""
    m, a = 5.2e-5, 1e-4
    xs = m * np.array([0.5, 1.0, 3.0])
    xs = xs * m * np.mean(1.0 / xs)            # harmonic mean exactly m
    clean = np.stack([np.full((512, 512), x) for x in xs])
    dark = np.ones(3, dtype=bool)
    noisy = synth.degrade(clean, synth.Degradation(unit_df_mean=m, gauss_abs=a), np.random.SeedSequence(3), dark=dark)
    phi = lambda t: math.exp(-0.5 * t * t) / math.sqrt(2 * math.pi)  # noqa: E731
    Phi = lambda t: 0.5 * math.erfc(-t / math.sqrt(2))  # noqa: E731
    want = 100 * np.mean([(a * (2 * phi(0) - phi(x / a)) + x * Phi(-x / a)) / x for x in xs])
    got = metrics.noise_level(clean, noisy, dark)
    assert abs(got / want - 1) < 5e-3, (got, want)


def test_salt_and_pepper_density_and_values():
    clean = np.full((1, 512, 512), 0.25)
    dark = np.array([True])
    out = synth.degrade(clean, synth.Degradation(unit_df_mean=0.25, snp_density=0.1), np.random.SeedSequence(4),
                        dark=dark)
    n = out.size
    salt = out == 1.0                          # camera unit = 1 here: salt reads 1
    pepper = out == 0.0
    sd = math.sqrt(0.05 * 0.95 / n)
    assert abs(salt.mean() - 0.05) < 5 * sd and abs(pepper.mean() - 0.05) < 5 * sd
    assert np.all(out[~(salt | pepper)] == 0.25)


def test_illumination_field_spans_one_minus_c_to_one():
    u = synth.illumination_field(np.random.default_rng(5), 128, 15.0)
    assert u.min() == 0.0 and u.max() == 1.0
    clean = np.ones((3, 128, 128))
    dark = np.ones(3, dtype=bool)
    out = synth.degrade(clean, synth.Degradation(unit_df_mean=1.0, illum_c=0.75), np.random.SeedSequence(6),
                        dark=dark)
    for k in range(3):
        assert abs(out[k].min() - 0.25) < 1e-12 and abs(out[k].max() - 1.0) < 1e-12
    assert not np.allclose(out[0], out[1])     # one field per image


def test_sweep_levels_and_table1_gaussian_row():
    """Table 1's Gaussian row (c = 0.25 and 0.75) within 10 % on a synthetic stack: pins the
    camera-unit constant and the illumination reading (its NL at the smallest a)."""
    table = {0.25: (20.49, 99.18, 800.10, 7669.71), 0.75: (41.98, 107.06, 793.00, 7656.55)}
    optics = synth.Optics(n_lo=32, upsample=4, led_grid=9)
    case = synth.make_case(optics, [7, 0])
    sim = orc.problem_from_optics(optics, case.led_k_true, flags=orc.PUPIL_SUPPORT)
    clean = orc.intensities(orc.spectrum_from_object(case.obj), case.pupil, sim)
    dark = metrics.dark_field(case.led_k_true, optics.n_lo, optics.dx_lo_um, optics.wavelength_um, optics.na)
    for c, row in table.items():
        for lv, want in enumerate(row):
            noisy = synth.degrade(clean, synth.sweep_degradation("gaussian", lv, c), np.random.SeedSequence([lv]),
                                  dark=dark)
            got = metrics.noise_level(clean, noisy, dark)
            assert abs(got / want - 1) < 0.1, (c, lv, got, want)
    for noise in ("gaussian", "snp", "poisson"):
        for lv in range(4):
            d = synth.sweep_degradation(noise, lv, 0.5)
            assert d.illum_c == 0.5 and d.unit_df_mean == synth.SWEEP_UNIT_DF_MEAN
    with pytest.raises(ValueError):
        synth.sweep_degradation("speckle", 0, 0.5)
