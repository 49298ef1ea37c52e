"""Pins of the oracle's Eq. (19) update, the pupil pre-filter, the metrics of Sec. 4.1,
the automatic penalty weight (Eq. 16-17) and a noise-free recovery (Algorithm 1)."""
import math

import numpy as np
import pytest

import oracle as orc
import synth


def scalar_prob(**kw):
    return orc.Problem(n_lo=2, upsample=1, led_k=np.zeros((1, 2)), wavelength_um=1.0, na=0.1,
                       dx_lo_um=1.0, **kw)


def test_adabelief_first_step_closed_form():
    """From mu = v = 0, delta = delta0 at t = 1: mu_hat = g, v_hat = (1-g1)^2 |g|^2, so the step
    is (sqrt(delta0) + eta) * g / ((1 - g1)|g| + eta) -> magnitude lr / 0.9 for |g| >> eta."""
    prob = scalar_prob(lr=1e-2)
    g = np.array([3.0 - 4.0j, 1e-3 + 2e-3j, -7.0 + 0j])
    x0 = np.array([1.0 + 1.0j, 0.5j, 2.0])
    d0 = np.full(3, prob.lr ** 2)
    x, mu, v, delta = orc.adabelief(x0, g, np.zeros(3, complex), np.zeros(3), d0, 1, prob)
    gm = np.abs(g)
    step = (prob.lr + prob.eta_opt) * g / (0.9 * gm + prob.eta_opt)
    assert np.max(np.abs((x0 - x) - step)) < 1e-15
    assert np.allclose(np.abs(x0 - x), prob.lr / 0.9, rtol=1e-5)
    assert np.allclose(mu, 0.1 * g) and np.allclose(v, 0.001 * 0.81 * gm ** 2)
    assert np.allclose(delta, 0.9 * prob.lr ** 2 + 0.1 * np.abs(step) ** 2)


def test_adabelief_constant_gradient_moments():
    """Constant g: mu_t = (1 - g1^t) g (so mu_hat = g) and
    v_t = (1 - g2) |g|^2 g1^2 (g2^t - g1^(2t)) / (g2 - g1^2) (geometric series)."""
    prob = scalar_prob(lr=0.1)
    g1, g2 = prob.gamma1, prob.gamma2
    g = np.array([0.3 - 0.4j])
    x, mu, v, d = np.zeros(1, complex), np.zeros(1, complex), np.zeros(1), np.full(1, prob.lr ** 2)
    for t in range(1, 31):
        x, mu, v, d = orc.adabelief(x, g, mu, v, d, t, prob)
        assert abs(mu[0] - (1 - g1 ** t) * g[0]) < 1e-15
        vt = (1 - g2) * abs(g[0]) ** 2 * g1 ** 2 * (g2 ** t - g1 ** (2 * t)) / (g2 - g1 ** 2)
        assert abs(v[0] - vt) < 1e-14 * max(vt, 1e-30)
    # the iterate moves against g
    assert np.real(np.vdot(g, x))[()] < 0


def test_gauss3_weights_closed_form():
    w = orc.gauss3_weights()
    z = 1.0 + 4.0 * math.exp(-0.5) + 4.0 * math.exp(-1.0)
    assert abs(w[1, 1] - 1.0 / z) < 1e-15 and abs(w[1, 1] - 0.20418) < 1e-5
    assert abs(w[0, 1] - math.exp(-0.5) / z) < 1e-15 and abs(w[0, 1] - 0.12384) < 1e-5
    assert abs(w[0, 0] - math.exp(-1.0) / z) < 1e-15 and abs(w[0, 0] - 0.07511) < 1e-5
    P = np.full((7, 7), 2.0 - 1.0j)
    out = orc.gauss3(P)
    assert np.allclose(out[1:-1, 1:-1], P[1:-1, 1:-1], atol=1e-15)
    assert abs(out[0, 0] - (2.0 - 1.0j) * (w[1, 1] + w[0, 1] * 2 + w[0, 0])) < 1e-14


def test_lsnr_closed_forms():
    x = np.array([3.0, 4.0])
    assert orc.lsnr(x + 5.0, x) == math.inf
    phi = x + np.array([1.0, -1.0])
    assert abs(orc.lsnr(phi, x) - 10 * math.log10(25.0 / 2.0)) < 1e-12
    # an additive constant on the estimate does not change the score
    assert abs(orc.lsnr(phi + 3.0, x) - orc.lsnr(phi, x)) < 1e-12


def test_noise_level_zero_for_clean_data():
    rng = np.random.default_rng(0)
    clean = rng.random((4, 5, 5)) + 0.1
    assert orc.noise_level(clean, clean, np.array([True, False, True, True])) == 0.0
    noisy = clean * 1.5
    assert abs(orc.noise_level(clean, noisy, np.ones(4, bool)) - 50.0) < 1e-12


def test_auto_penalty_closed_forms():
    H, W = 6, 9
    yy, xx = np.meshgrid(np.arange(H, dtype=float), np.arange(W, dtype=float), indexing="ij")
    aff = np.stack([2.0 + 0.5 * xx - 0.25 * yy] * 3)
    assert orc.auto_penalty(aff, orc.FID_INTENSITY) == 0.0
    checker = np.stack([1.0 + (-1.0) ** xx] * 2)  # columns alternate 2, 0: deviation +-1, |conv| = 16
    expect = 0.2 * math.sqrt(math.pi / 2) * 16.0 * (H - 2) * (W - 2) / (W * H)
    assert abs(orc.auto_penalty(checker, orc.FID_INTENSITY) - expect) < 1e-12


def test_noise_free_recovery_config1():
    """Algorithm 1 on the noise-free config-1 stack, pupil held fixed (intensity fidelity,
    lr = 1e-2, 50 iterations).  Thresholds stated from the oracle run: amplitude LSNR
    >= 30 dB, phase LSNR >= 17 dB (reached: 34.3 / 20.1), loss down >= 10x."""
    case = synth.config_case(1)
    sim = orc.problem_from_optics(case.optics, case.led_k_true)
    meas = orc.intensities(orc.spectrum_from_object(case.obj), case.pupil, sim)
    prob = orc.problem_from_optics(case.optics, case.led_k, flags=orc.PUPIL_SUPPORT)
    st = orc.init_state(meas, prob)
    st, hist = orc.run(st, meas, prob, 50)
    O = orc.object_from_spectrum(st.psi)
    assert orc.lsnr(np.abs(O), np.abs(case.obj)) >= 30.0
    assert orc.lsnr(np.angle(O), np.angle(case.obj)) >= 17.0
    assert hist[-1, 3] < 0.1 * hist[0, 3]
    assert st.t == 50


def test_pupil_learning_keeps_support_and_reduces_loss():
    case = synth.config_case(1)
    sim = orc.problem_from_optics(case.optics, case.led_k_true)
    meas = orc.intensities(orc.spectrum_from_object(case.obj), case.pupil, sim)
    flags = orc.LEARN_PUPIL | orc.PUPIL_SUPPORT | orc.PUPIL_FILTER
    prob = orc.problem_from_optics(case.optics, case.led_k, flags=flags)
    st = orc.init_state(meas, prob)
    st, hist = orc.run(st, meas, prob, 40)
    S = orc.pupil_support(prob)
    assert np.all(st.P[~S] == 0)
    assert hist[-1, 3] < 0.5 * hist[0, 3]  # reached: 3002 -> 846
