"""Pins of the oracle's closed-form gradients (Eq. 9-18) against central finite
differences of its loss (Eq. 4-8), plus brute-force loss values and the zero-residual
invariant.  The loss itself is pinned by an independent per-pixel loop evaluation.

For a real loss L and complex variable z, the directional derivative along d is
2 Re <dL/d(conj z), d>, so the check is (L(z + h d) - L(z - h d)) / (2h) against
2 Re vdot(g, d).  The L1 terms are smoothed (l1_eps > 0) and eta_h = 0 so that the
loss is differentiable and the gradient exact.
"""
import math

import numpy as np
import pytest

import oracle as orc
import synth
from helpers import rand_complex, smooth_object


def make_problem(fidelity, norm, *, n_lo=8, upsample=2, grid=3, na=0.15, eps=1e-2,
                 alpha=0.3, beta=0.2, flags=orc.PUPIL_SUPPORT, seed=0, gamma=0.5):
    optics = synth.Optics(n_lo=n_lo, upsample=upsample, na=na, led_grid=grid)
    pos = synth.led_grid_positions(grid, optics.pitch_mm)
    k = synth.led_wavevectors(pos, optics.height_mm, optics.wavelength_um)
    prob = orc.problem_from_optics(optics, k, fidelity=fidelity, norm=norm, l1_eps=eps,
                                   eta_h=0.0, alpha=alpha, beta=beta, flags=flags, fid_gamma=gamma)
    rng = np.random.default_rng(seed)
    O = smooth_object(seed, prob.n_hi)
    psi = orc.spectrum_from_object(O)
    P = np.exp(0.3j * rng.standard_normal((n_lo, n_lo))) * (0.8 + 0.2 * rng.random((n_lo, n_lo)))
    O2 = smooth_object(seed + 1, prob.n_hi)
    meas = orc.intensities(orc.spectrum_from_object(O2), P, prob) * (1 + 0.1 * rng.random((prob.K, n_lo, n_lo)))
    return prob, psi, P, meas


def fd_check(fun, z, g, rng, n_dir=4, h=1e-5):
    worst = 0.0
    for _ in range(n_dir):
        d = rand_complex(rng, z.shape)
        d /= np.linalg.norm(d)
        fd = (fun(z + h * d) - fun(z - h * d)) / (2 * h)
        an = 2.0 * float(np.real(np.vdot(g, d)))
        worst = max(worst, abs(fd - an) / max(abs(an), 1e-3))
    return worst


CASES = [(f, n) for f in (orc.FID_AMPLITUDE, orc.FID_INTENSITY) for n in (orc.NORM_ANISO, orc.NORM_ISO)]
# the scalings g(x) = x^gamma and ln(x + 1) of Sec. 6.3, as (fidelity, gamma)
SCALINGS = [(orc.FID_GAMMA, 0.125), (orc.FID_GAMMA, 0.375), (orc.FID_GAMMA, 0.875), (orc.FID_LOG, 0.5)]
GCASES = [(f, n, g) for f, n in CASES for g in (0.5,)] + [(f, n, g) for f, g in SCALINGS
                                                         for n in (orc.NORM_ANISO, orc.NORM_ISO)]


@pytest.mark.parametrize("fidelity,norm,gamma", GCASES)
def test_psi_gradient_matches_finite_differences(fidelity, norm, gamma):
    prob, psi, P, meas = make_problem(fidelity, norm, gamma=gamma)
    _, g_psi, _ = orc.loss_and_grad(psi, P, meas, prob)
    err = fd_check(lambda z: orc.loss(z, P, meas, prob), psi, g_psi, np.random.default_rng(1))
    assert err < 1e-6, err


@pytest.mark.parametrize("fidelity,norm,gamma", GCASES)
def test_pupil_gradient_matches_finite_differences(fidelity, norm, gamma):
    prob, psi, P, meas = make_problem(fidelity, norm, flags=0, gamma=gamma)
    _, _, g_P = orc.loss_and_grad(psi, P, meas, prob)
    err = fd_check(lambda z: orc.loss(psi, z, meas, prob), P, g_P, np.random.default_rng(2))
    assert err < 1e-6, err


def test_pupil_gradient_with_support_is_masked_derivative():
    prob, psi, P, meas = make_problem(orc.FID_INTENSITY, orc.NORM_ANISO, flags=orc.PUPIL_SUPPORT, na=0.1)
    S = orc.pupil_support(prob)
    assert 0 < S.sum() < S.size
    _, _, g_P = orc.loss_and_grad(psi, P, meas, prob)
    assert np.all(g_P[~S] == 0)
    err = fd_check(lambda z: orc.loss(psi, z, meas, prob), P, g_P, np.random.default_rng(3))
    assert err < 1e-6, err


@pytest.mark.parametrize("norm", [orc.NORM_ANISO, orc.NORM_ISO])
@pytest.mark.parametrize("which", ["amp", "phase"])
def test_hessian_gradients_match_finite_differences(norm, which):
    alpha, beta = (1.0, 0.0) if which == "amp" else (0.0, 1.0)
    prob, psi, P, meas = make_problem(orc.FID_INTENSITY, norm, alpha=alpha, beta=beta)
    LA0, LP0, gH = orc.hessian_loss_and_grad(psi, prob)

    def f(z):
        LA, LP, _ = orc.hessian_loss_and_grad(z, prob, want_grad=False)
        return alpha * LA + beta * LP
    err = fd_check(f, psi, gH, np.random.default_rng(4))
    assert err < 1e-6, err


def test_fd_error_shrinks_quadratically():
    prob, psi, P, meas = make_problem(orc.FID_AMPLITUDE, orc.NORM_ISO)
    _, g, _ = orc.loss_and_grad(psi, P, meas, prob)
    rng = np.random.default_rng(9)
    d = rand_complex(rng, psi.shape)
    d /= np.linalg.norm(d)
    an = 2.0 * float(np.real(np.vdot(g, d)))
    errs = []
    for h in (1e-2, 5e-3, 2.5e-3):
        fd = (orc.loss(psi + h * d, P, meas, prob) - orc.loss(psi - h * d, P, meas, prob)) / (2 * h)
        errs.append(abs(fd - an))
    # second order: halving h divides the error by about 4
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0, errs


def brute_fidelity(psi, P, meas, prob):
    """Eq. (4)/(5) with explicit loops: o by explicit sums, gradients by explicit differences."""
    n, r = prob.n_lo, prob.upsample
    fov = prob.n_lo * prob.dx_lo_um
    R = prob.na * fov / prob.wavelength_um
    total = 0.0
    for kk in range(prob.K):
        offx = int(math.copysign(math.floor(abs(prob.led_k[kk, 0] * fov) + 0.5), prob.led_k[kk, 0]))
        offy = int(math.copysign(math.floor(abs(prob.led_k[kk, 1] * fov) + 0.5), prob.led_k[kk, 1]))
        o = np.zeros((n, n), dtype=complex)
        for yy in range(n):
            for xx in range(n):
                acc = 0j
                for v in range(-n // 2, n // 2):
                    for u in range(-n // 2, n // 2):
                        if u * u + v * v > R * R * (1 + 1e-12):
                            continue
                        val = P[v + n // 2, u + n // 2] * psi[prob.n_hi // 2 + offy + v, prob.n_hi // 2 + offx + u]
                        acc += val * complex(math.cos(2 * math.pi * (u * xx + v * yy) / n),
                                             math.sin(2 * math.pi * (u * xx + v * yy) / n))
                o[yy, xx] = acc / (r * n)
        if prob.fidelity == orc.FID_AMPLITUDE:
            e = np.abs(o) - np.sqrt(meas[kk])
        elif prob.fidelity == orc.FID_GAMMA:
            e = np.array([[math.pow(abs(o[yy, xx]) ** 2, prob.fid_gamma) - math.pow(meas[kk, yy, xx], prob.fid_gamma)
                           for xx in range(n)] for yy in range(n)])
        elif prob.fidelity == orc.FID_LOG:
            e = np.array([[math.log(1 + abs(o[yy, xx]) ** 2) - math.log(1 + meas[kk, yy, xx])
                           for xx in range(n)] for yy in range(n)])
        else:
            e = np.abs(o) ** 2 - meas[kk]
        for yy in range(n):
            for xx in range(n):
                gx = e[yy, xx + 1] - e[yy, xx] if xx + 1 < n else 0.0
                gy = e[yy + 1, xx] - e[yy, xx] if yy + 1 < n else 0.0
                if prob.norm == orc.NORM_ANISO:
                    total += abs(gx) + abs(gy)
                else:
                    total += math.hypot(gx, gy)
    return total


@pytest.mark.parametrize("fidelity,norm,gamma", GCASES)
def test_fidelity_loss_matches_brute_force(fidelity, norm, gamma):
    prob, psi, P, meas = make_problem(fidelity, norm, eps=0.0, n_lo=6, upsample=2, grid=2, na=0.2, gamma=gamma)
    Lf, _, _ = orc.fidelity_loss_and_grad(psi, P, meas, prob, want_grad=False)
    assert abs(Lf - brute_fidelity(psi, P, meas, prob)) < 1e-10 * max(1.0, Lf)


def test_hessian_loss_matches_brute_force():
    prob, psi, P, meas = make_problem(orc.FID_INTENSITY, orc.NORM_ANISO, eps=0.0)
    O = orc.object_from_spectrum(psi)
    n = O.shape[0]
    la = lp = 0.0
    for f, acc_name in ((np.abs(O), "a"), (np.arctan2(O.imag, O.real), "p")):
        s = 0.0
        for yy in range(n):
            for xx in range(n):
                if 1 <= xx <= n - 2:
                    s += abs(f[yy, xx - 1] - 2 * f[yy, xx] + f[yy, xx + 1])
                if 1 <= yy <= n - 2:
                    s += abs(f[yy - 1, xx] - 2 * f[yy, xx] + f[yy + 1, xx])
                if xx <= n - 2 and yy <= n - 2:
                    s += abs(f[yy, xx] - f[yy, xx + 1] - f[yy + 1, xx] + f[yy + 1, xx + 1])
        if acc_name == "a":
            la = s
        else:
            lp = s
    LA, LP, _ = orc.hessian_loss_and_grad(psi, prob, want_grad=False)
    assert abs(LA - la) < 1e-10 * la and abs(LP - lp) < 1e-10 * lp


def test_zero_residual_gives_zero_fidelity_and_gradient():
    prob, psi, P, _ = make_problem(orc.FID_INTENSITY, orc.NORM_ANISO, eps=0.0)
    meas = orc.intensities(psi, P, prob)
    Lf, g_psi, g_P = orc.fidelity_loss_and_grad(psi, P, meas, prob)
    assert Lf == 0.0
    assert np.all(g_psi == 0) and np.all(g_P == 0)


def test_amplitude_zero_residual_is_tiny():
    prob, psi, P, _ = make_problem(orc.FID_AMPLITUDE, orc.NORM_ISO, eps=1e-3)
    meas = orc.intensities(psi, P, prob)
    Lf, g_psi, _ = orc.fidelity_loss_and_grad(psi, P, meas, prob)
    assert Lf < 1e-10
    assert np.max(np.abs(g_psi)) < 1e-10


def test_phase_gradient_is_tangent_to_object_modulus():
    """Eq. (14) only rotates O: the space-domain phase gradient is i*O*real, so it changes the
    phase of every pixel without changing |O| to first order."""
    prob, psi, P, meas = make_problem(orc.FID_INTENSITY, orc.NORM_ANISO, alpha=0.0, beta=1.0)
    _, _, gH = orc.hessian_loss_and_grad(psi, prob)
    G = orc.object_from_spectrum(gH)
    O = orc.object_from_spectrum(psi)
    assert np.max(np.abs(np.real(np.conj(O) * G))) < 1e-12 * np.max(np.abs(G))


@pytest.mark.parametrize("gamma,same_as", [(0.5, orc.FID_AMPLITUDE), (1.0, orc.FID_INTENSITY)])
@pytest.mark.parametrize("norm", [orc.NORM_ANISO, orc.NORM_ISO])
def test_gamma_scaling_reduces_to_amplitude_and_intensity(gamma, same_as, norm):
    """g(x) = x^gamma is Eq. (4) at gamma = 1/2 and Eq. (5) at gamma = 1 (Sec. 6.3): the
    general branch must give their losses and gradients."""
    prob_g, psi, P, meas = make_problem(orc.FID_GAMMA, norm, gamma=gamma, flags=0)
    prob_r, _, _, _ = make_problem(same_as, norm, flags=0)
    lg, gg, pg = orc.loss_and_grad(psi, P, meas, prob_g)
    lr, gr, pr = orc.loss_and_grad(psi, P, meas, prob_r)
    assert np.allclose(lg, lr, rtol=1e-12, atol=0)
    assert np.linalg.norm(gg - gr) <= 1e-12 * np.linalg.norm(gr)
    assert np.linalg.norm(pg - pr) <= 1e-12 * np.linalg.norm(pr)


@pytest.mark.parametrize("fidelity,gamma", SCALINGS)
def test_scaling_zero_residual(fidelity, gamma):
    """With I from the forward model itself, every scaling gives a zero loss and gradient."""
    prob, psi, P, _ = make_problem(fidelity, orc.NORM_ANISO, eps=0.0, gamma=gamma)
    meas = orc.intensities(psi, P, prob)
    Lf, g_psi, g_P = orc.fidelity_loss_and_grad(psi, P, meas, prob)
    assert Lf < 1e-9
    assert np.max(np.abs(g_psi)) < 1e-9 and np.max(np.abs(g_P)) < 1e-9


def test_log_scaling_slope_is_exact_at_zero():
    """ln(x + 1) is smooth at x = 0 (slope 1), unlike the powers, whose slope is taken as 0."""
    x = np.array([0.0, 1.0, 3.0])
    assert np.allclose(orc.scaling_slope(x, orc.FID_LOG), [1.0, 0.5, 0.25])
    assert np.allclose(orc.scaling_slope(x, orc.FID_GAMMA, 0.5), [0.0, 0.5, 0.5 / math.sqrt(3.0)])


def _l1_features(psi, P, meas, prob, part):
    """Every feature the L1 terms see: the image differences of the fidelity residual of
    each LED (Eq. 4 / 5), or the Hessian components of |O| and angle(O) (Eq. 6, 7)."""
    if part == "fidelity":
        e = [orc.fidelity_residual(o, m, prob.fidelity, prob.fid_gamma)
             for o, m in zip(orc.fields(psi, P, prob), meas)]
        return np.concatenate([np.stack([orc.dx(x), orc.dy(x)]).ravel() for x in e])
    O = orc.object_from_spectrum(psi)
    src = [np.abs(O), np.arctan2(O.imag, O.real)]
    return np.concatenate([H(s).ravel() for s in src for H in (orc.hxx, orc.hyy, orc.hxy)])


@pytest.mark.parametrize("part", ["fidelity", "hessian"])
@pytest.mark.parametrize("norm", [orc.NORM_ANISO, orc.NORM_ISO])
@pytest.mark.parametrize("fidelity", [orc.FID_INTENSITY, orc.FID_AMPLITUDE])
def test_exact_l1_gradient_matches_finite_differences_between_kinks(fidelity, norm, part):
    """l1_eps = 0: the literal L1 of Eq. 4-7 with omega = sign (anisotropic) or c / |c|
    (isotropic) of Eq. 12 and the zero subgradient of Sec. 3.3.  Between the points where
    a feature (or, isotropic, a feature pair or triple) vanishes the loss is smooth, so a
    central difference whose step moves no feature across zero pins omega exactly.  The
    step is shrunk until no feature changes sign between z - h d and z + h d (checked),
    and the phase differences stay far from the branch cut of angle()."""
    alpha, beta = ((0.0, 0.0) if part == "fidelity" else (0.7, 0.4))
    prob, psi, P, meas = make_problem(fidelity, norm, eps=0.0, alpha=alpha, beta=beta)
    rng = np.random.default_rng(11)
    if part == "fidelity":
        _, g, _ = orc.loss_and_grad(psi, P, meas, prob)
        fun = lambda z: orc.loss(z, P, meas, prob)  # noqa: E731
    else:
        _, _, g = orc.hessian_loss_and_grad(psi, prob)

        def fun(z):
            LA, LP, _ = orc.hessian_loss_and_grad(z, prob, want_grad=False)
            return alpha * LA + beta * LP
    c0 = _l1_features(psi, P, meas, prob, part)
    assert np.min(np.abs(c0[c0 != 0])) > 0
    worst = 0.0
    for _ in range(4):
        d = rand_complex(rng, psi.shape)
        d /= np.linalg.norm(d)
        h = 1e-5
        for _ in range(6):
            cp = _l1_features(psi + h * d, P, meas, prob, part)
            cm = _l1_features(psi - h * d, P, meas, prob, part)
            same = np.array_equal(np.sign(cp), np.sign(c0)) and np.array_equal(np.sign(cm), np.sign(c0))
            if same and np.max(np.abs(cp - cm)) < 1.0:
                break
            h /= 4.0
        else:
            pytest.fail("no step without a kink crossing")
        fd = (fun(psi + h * d) - fun(psi - h * d)) / (2 * h)
        an = 2.0 * float(np.real(np.vdot(g, d)))
        worst = max(worst, abs(fd - an) / max(abs(an), 1e-3))
    assert worst < 1e-6, worst


def test_exact_l1_subgradient_is_zero_at_zero():
    """Sec. 3.3: the subgradient of |x| at 0 is taken as 0; an isotropic normaliser of a
    zero feature pair is 0 as well."""
    z = np.zeros(4)
    c = np.array([0.0, 2.0, -3.0, 0.0])
    val, (om,) = orc.l1_value_and_omega([c], orc.NORM_ANISO, 0.0)
    assert val == 5.0 and list(om) == [0.0, 1.0, -1.0, 0.0]
    val, (ox, oy) = orc.l1_value_and_omega([c, z], orc.NORM_ISO, 0.0)
    assert val == 5.0 and list(ox) == [0.0, 1.0, -1.0, 0.0] and list(oy) == [0.0] * 4
    val, (ox, oy) = orc.l1_value_and_omega([np.array([3.0, 0.0]), np.array([4.0, 0.0])], orc.NORM_ISO, 0.0)
    assert val == 5.0 and np.allclose(ox, [0.6, 0.0], rtol=0, atol=1e-15) and np.allclose(oy, [0.8, 0.0], rtol=0,
                                                                                          atol=1e-15)
