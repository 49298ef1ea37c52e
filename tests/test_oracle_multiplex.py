"""Pins of the oracle's multiplexed forward model and gradients (Eq. 1 with M > 1: each
image is the sum of the intensities of its M LEDs)."""
import math

import numpy as np
import pytest

import oracle as orc
import synth
from helpers import rand_complex, smooth_object


def mux_problem(mux, fidelity=orc.FID_INTENSITY, norm=orc.NORM_ANISO, *, n_lo=8, upsample=2, grid=3, na=0.15,
                eps=1e-2, gamma=0.5, flags=0, seed=0, alpha=0.3, beta=0.2):
    """A grid x grid LED array, grouped M at a time in row-major order (the last LEDs are
    dropped when grid^2 is not a multiple of M)."""
    optics = synth.Optics(n_lo=n_lo, upsample=upsample, na=na, led_grid=grid)
    pos = synth.led_grid_positions(grid, optics.pitch_mm)
    k = synth.led_wavevectors(pos, optics.height_mm, optics.wavelength_um)
    k = k[: (k.shape[0] // mux) * mux]
    prob = orc.problem_from_optics(optics, k, fidelity=fidelity, norm=norm, l1_eps=eps, eta_h=0.0, alpha=alpha,
                                   beta=beta, flags=flags, fid_gamma=gamma, mux=mux)
    rng = np.random.default_rng(seed)
    psi = orc.spectrum_from_object(smooth_object(seed, prob.n_hi))
    P = np.exp(0.3j * rng.standard_normal((n_lo, n_lo))) * (0.8 + 0.2 * rng.random((n_lo, n_lo)))
    meas = orc.intensities(orc.spectrum_from_object(smooth_object(seed + 1, prob.n_hi)), P, prob)
    meas = meas * (1 + 0.1 * rng.random(meas.shape))
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


def test_image_count_and_shapes():
    prob, psi, P, meas = mux_problem(3)
    assert prob.n_led == 9 and prob.K == 3
    assert orc.fields(psi, P, prob).shape == (9, 8, 8)
    assert meas.shape == (3, 8, 8)


CASES = [(m, f, n, g) for m in (2, 3)
         for f, g in ((orc.FID_INTENSITY, 0.5), (orc.FID_AMPLITUDE, 0.5), (orc.FID_GAMMA, 0.375), (orc.FID_LOG, 0.5))
         for n in (orc.NORM_ANISO, orc.NORM_ISO)]


@pytest.mark.parametrize("mux,fidelity,norm,gamma", CASES)
def test_multiplexed_gradients_match_finite_differences(mux, fidelity, norm, gamma):
    prob, psi, P, meas = mux_problem(mux, fidelity, norm, gamma=gamma)
    _, g_psi, g_P = orc.loss_and_grad(psi, P, meas, prob)
    rng = np.random.default_rng(mux * 10 + fidelity)
    assert fd_check(lambda z: orc.loss(z, P, meas, prob), psi, g_psi, rng) < 1e-6
    assert fd_check(lambda z: orc.loss(psi, z, meas, prob), P, g_P, rng) < 1e-6


def test_identical_leds_scale_loss_and_gradient():
    """M copies of the same LED: S = M |o|^2, so with I = M I_1 the intensity residual is M times
    the single-LED one; the exact L1 scales by M, and so does the gradient (each copy
    back-projects the same q o)."""
    one, psi, P, meas1 = mux_problem(1, eps=0.0)
    M = 3
    rep = orc.Problem(**{**one.__dict__, "led_k": np.repeat(one.led_k, M, axis=0), "mux": M})
    l1, g1, p1 = orc.fidelity_loss_and_grad(psi, P, meas1, one)
    lM, gM, pM = orc.fidelity_loss_and_grad(psi, P, M * meas1, rep)
    assert abs(lM - M * l1) < 1e-10 * lM
    assert np.linalg.norm(gM - M * g1) < 1e-10 * np.linalg.norm(gM)
    assert np.linalg.norm(pM - M * p1) < 1e-10 * np.linalg.norm(pM)


def test_multiplexed_plane_wave_counts_bright_leds():
    """A plane wave at integer frequency u0: each LED sees |o|^2 = 1 (inside the passband) or
    0, so an image of M LEDs is the number of them that are bright (Eq. 1)."""
    optics = synth.Optics(n_lo=32, upsample=4, led_grid=4)
    pos = synth.led_grid_positions(optics.led_grid, optics.pitch_mm)
    k = synth.led_wavevectors(pos, optics.height_mm, optics.wavelength_um)
    prob = orc.problem_from_optics(optics, k, mux=4)
    fov = optics.n_lo * optics.dx_lo_um
    n = optics.n_hi
    yy, xx = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    P = orc.pupil_support(prob).astype(np.complex128)
    cutoff = optics.na / optics.wavelength_um
    checked, counts = 0, set()
    for ux, uy in [(0, 0), (6, -2), (-9, 4), (3, 3), (-4, -7), (12, 0), (0, 10), (-15, -3)]:
        O = np.exp(2j * math.pi * (ux * xx + uy * yy) / n)
        inten = orc.intensities(orc.spectrum_from_object(O), P, prob)
        dist = np.linalg.norm(np.array([ux, uy]) / fov - k, axis=1)
        near_edge = np.abs(dist - cutoff) * fov < 1.5
        for img in range(prob.K):
            group = slice(img * 4, img * 4 + 4)
            if near_edge[group].any():
                continue
            bright = int(np.sum(dist[group] < cutoff))
            assert np.max(np.abs(inten[img] - bright)) < 1e-12
            checked += 1
            counts.add(bright)
    assert checked >= 8 and len(counts) >= 3, (checked, counts)


def test_multiplexed_zero_residual():
    prob, psi, P, _ = mux_problem(2, eps=0.0)
    meas = orc.intensities(psi, P, prob)
    L, g_psi, g_P = orc.fidelity_loss_and_grad(psi, P, meas, prob)
    assert L == 0.0 and np.all(g_psi == 0) and np.all(g_P == 0)


def test_multiplexed_loss_matches_explicit_loops():
    """Eq. (5) with M = 2 by explicit sums: o by explicit DFT sums, S = |o_1|^2 + |o_2|^2."""
    prob, psi, P, meas = mux_problem(2, eps=0.0, n_lo=6, grid=2, na=0.2)
    n, r = prob.n_lo, prob.upsample
    fov = prob.n_lo * prob.dx_lo_um
    total = 0.0
    for img in range(prob.K):
        S = np.zeros((n, n))
        for kk in (2 * img, 2 * img + 1):
            offx = int(math.copysign(math.floor(abs(prob.led_k[kk, 0] * fov) + 0.5), prob.led_k[kk, 0]))
            offy = int(math.copysign(math.floor(abs(prob.led_k[kk, 1] * fov) + 0.5), prob.led_k[kk, 1]))
            for yy in range(n):
                for xx in range(n):
                    acc = 0j
                    for v in range(-n // 2, n // 2):
                        for u in range(-n // 2, n // 2):
                            val = P[v + n // 2, u + n // 2] * psi[prob.n_hi // 2 + offy + v, prob.n_hi // 2 + offx + u]
                            acc += val * complex(math.cos(2 * math.pi * (u * xx + v * yy) / n),
                                                 math.sin(2 * math.pi * (u * xx + v * yy) / n))
                    S[yy, xx] += abs(acc / (r * n)) ** 2
        e = S - meas[img]
        for yy in range(n):
            for xx in range(n):
                total += abs(e[yy, xx + 1] - e[yy, xx]) if xx + 1 < n else 0.0
                total += abs(e[yy + 1, xx] - e[yy, xx]) if yy + 1 < n else 0.0
    # flags = 0: no support mask, P acts on the whole window
    L, _, _ = orc.fidelity_loss_and_grad(psi, P, meas, prob, want_grad=False)
    assert abs(L - total) < 1e-10 * total
