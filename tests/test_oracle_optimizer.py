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


@pytest.mark.parametrize("fidelity,gamma", [(orc.FID_AMPLITUDE, 0.5), (orc.FID_GAMMA, 0.25), (orc.FID_LOG, 0.5)])
def test_auto_penalty_sees_the_scaled_stack(fidelity, gamma):
    """The mask is applied to g(I): a stack whose g(I) is affine gives 0, and the value is
    the intensity rule applied to g(I)."""
    H, W = 7, 8
    yy, xx = np.meshgrid(np.arange(H, dtype=float), np.arange(W, dtype=float), indexing="ij")
    aff = 1.0 + 0.2 * xx + 0.1 * yy
    inv = {orc.FID_AMPLITUDE: aff ** 2, orc.FID_GAMMA: aff ** (1.0 / gamma), orc.FID_LOG: np.expm1(aff)}[fidelity]
    assert abs(orc.auto_penalty(np.stack([inv] * 2), fidelity, gamma)) < 1e-12
    rng = np.random.default_rng(5)
    I = rng.random((3, H, W)) + 0.1
    gI = {orc.FID_AMPLITUDE: np.sqrt(I), orc.FID_GAMMA: I ** gamma, orc.FID_LOG: np.log1p(I)}[fidelity]
    assert abs(orc.auto_penalty(I, fidelity, gamma) - orc.auto_penalty(gI, orc.FID_INTENSITY)) < 1e-14


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


# --- the optimisers compared in Sec. 6.2: SGD, NAdam, AdaBelief (published definitions) ---

def test_sgd_on_a_quadratic_is_a_geometric_contraction():
    """L = |x - c|^2 has dL/d(conj x) = x - c, so x_t - c = (1 - lr)^t (x_0 - c)."""
    prob = scalar_prob(lr=0.3, optimizer=orc.OPT_SGD)
    c = np.array([1.0 - 2.0j, 0.5 + 0.0j])
    x = np.array([4.0 + 1.0j, -3.0 + 2.0j])
    x0 = x.copy()
    mu, v, d = np.zeros(2, complex), np.zeros(2), np.zeros(2)
    for t in range(1, 11):
        x, mu, v, d = orc.optimizer_step(x, x - c, mu, v, d, t, prob)
    assert np.max(np.abs((x - c) - 0.7 ** 10 * (x0 - c))) < 1e-14


def test_nadam_first_step_and_limits():
    """First step from zero moments: v_hat = |g|^2 and m_hat = g (1 + g1 / (1 + g1)), so the
    step has length lr (1 + g1 / (1 + g1)) for |g| >> eps; with a constant gradient the
    look-ahead mean tends to g and the step to lr g / |g|; with g1 = g2 = 0 every step is
    lr g / (|g| + eps) (normalised gradient descent)."""
    prob = scalar_prob(lr=1e-2, optimizer=orc.OPT_NADAM)
    g = np.array([3.0 - 4.0j, -0.5 + 0.0j])
    x0 = np.zeros(2, complex)
    x, mu, v, d = orc.optimizer_step(x0, g, np.zeros(2, complex), np.zeros(2), np.zeros(2), 1, prob)
    assert np.allclose(np.abs(x0 - x), prob.lr * (1 + 0.9 / 1.9), rtol=1e-7)
    unit = (x0 - x) * np.abs(g) / g  # the step is a real multiple of g / |g|
    assert np.allclose(unit, unit[0]) and abs(unit[0].imag) < 1e-15
    for t in range(2, 400):
        xp = x
        x, mu, v, d = orc.optimizer_step(x, g, mu, v, d, t, prob)
    assert np.allclose(xp - x, prob.lr * g / np.abs(g), rtol=1e-6)
    flat = scalar_prob(lr=0.05, optimizer=orc.OPT_NADAM, gamma1=0.0, gamma2=0.0)
    rng = np.random.default_rng(3)
    x = np.zeros(2, complex)
    mu, v = np.zeros(2, complex), np.zeros(2)
    for t in range(1, 6):
        gt = rng.standard_normal(2) + 1j * rng.standard_normal(2)
        xn, mu, v, d = orc.optimizer_step(x, gt, mu, v, d, t, flat)
        assert np.allclose(x - xn, flat.lr * gt / (np.abs(gt) + flat.eta_opt), rtol=1e-12)
        x = xn


def test_adabelief_plain_first_step_and_constant_gradient():
    """First step: m_hat = g, s_hat = g1^2 |g|^2 + eps / (1 - g2), so the step has length
    lr / g1 for |g| >> eps.  Constant gradient: m_hat = g at every t and
    s_t = (1 - g2) |g|^2 g1^2 (g2^t - g1^(2t)) / (g2 - g1^2) + eps (1 - g2^t) / (1 - g2)."""
    prob = scalar_prob(lr=1e-2, optimizer=orc.OPT_ADABELIEF)
    g1, g2, eps = prob.gamma1, prob.gamma2, prob.eta_opt
    g = np.array([0.3 - 0.4j])
    x, mu, s, d = np.zeros(1, complex), np.zeros(1, complex), np.zeros(1), np.zeros(1)
    x, mu, s, d = orc.optimizer_step(x, g, mu, s, d, 1, prob)
    first = prob.lr * g[0] / (math.sqrt(g1 ** 2 * abs(g[0]) ** 2 + eps / (1 - g2)) + eps)
    assert abs(-x[0] - first) < 1e-15
    assert abs(abs(x[0]) - prob.lr / g1) < 1e-4 * prob.lr
    for t in range(2, 40):
        xp = x
        x, mu, s, d = orc.optimizer_step(x, g, mu, s, d, t, prob)
        st = (1 - g2) * abs(g[0]) ** 2 * g1 ** 2 * (g2 ** t - g1 ** (2 * t)) / (g2 - g1 ** 2) \
            + eps * (1 - g2 ** t) / (1 - g2)
        assert abs(s[0] - st) < 1e-13 * st
        expect = prob.lr * g[0] / (math.sqrt(st / (1 - g2 ** t)) + eps)
        assert abs((xp - x)[0] - expect) < 1e-12 * abs(expect)


@pytest.mark.parametrize("opt", [orc.OPT_SGD, orc.OPT_NADAM, orc.OPT_ADABELIEF])
def test_every_optimiser_reduces_the_config1_loss(opt):
    """Algorithm 1 with the Sec. 6.2 alternatives on the noise-free config-1 stack."""
    case = synth.config_case(1)
    sim = orc.problem_from_optics(case.optics, case.led_k_true)
    meas = orc.intensities(orc.spectrum_from_object(case.obj), case.pupil, sim)
    lr = {orc.OPT_SGD: 3e-2, orc.OPT_NADAM: 1e-2, orc.OPT_ADABELIEF: 1e-2}[opt]
    prob = orc.problem_from_optics(case.optics, case.led_k, flags=orc.PUPIL_SUPPORT, optimizer=opt, lr=lr)
    st = orc.init_state(meas, prob)
    st, hist = orc.run(st, meas, prob, 20)
    assert np.all(np.isfinite(hist))
    assert hist[-1, 3] < 0.9 * hist[0, 3]  # reached: SGD 0.16, NAdam 0.82, AdaBelief 0.74


def test_eq19_beats_nadam_and_adabelief_at_the_same_step_size():
    """Sec. 6.2 (Fig. 13a): with the same parameters the proposed update lowers the loss
    faster than NAdam and AdaBelief.  Config-1 noise-free stack, lr = 1e-2, 20 iterations
    (reached: Eq. 19 0.58, AdaBelief 0.74, NAdam 0.82 of the initial loss)."""
    case = synth.config_case(1)
    sim = orc.problem_from_optics(case.optics, case.led_k_true)
    meas = orc.intensities(orc.spectrum_from_object(case.obj), case.pupil, sim)
    final = {}
    for opt in (orc.OPT_ELFPIE, orc.OPT_NADAM, orc.OPT_ADABELIEF):
        prob = orc.problem_from_optics(case.optics, case.led_k, flags=orc.PUPIL_SUPPORT, optimizer=opt, lr=1e-2)
        _, hist = orc.run(orc.init_state(meas, prob), meas, prob, 20)
        final[opt] = hist[-1, 3]
    assert final[orc.OPT_ELFPIE] < final[orc.OPT_ADABELIEF] < final[orc.OPT_NADAM]
