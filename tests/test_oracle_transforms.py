"""Pins of the oracle's transforms, windows and stencils against textbook definitions.

Each check is computed here from a definition that does not go through the
oracle's own code path: explicit DFT sums, Parseval's identity, the physical
cut-off NA/lambda of the objective, dot-product adjoint identities and closed-form
derivatives of polynomials.
"""
import math

import numpy as np
import pytest

import oracle as orc
import synth
from helpers import rand_complex, small_optics


def brute_centred_dft(x):
    """Unitary 2-D DFT with frequency index u = k - n/2 written as an explicit sum."""
    n = x.shape[0]
    out = np.zeros((n, n), dtype=np.complex128)
    for ky in range(n):
        for kx in range(n):
            uy, ux = ky - n // 2, kx - n // 2
            acc = 0j
            for yy in range(n):
                for xx in range(n):
                    acc += x[yy, xx] * complex(math.cos(-2 * math.pi * (uy * yy + ux * xx) / n),
                                               math.sin(-2 * math.pi * (uy * yy + ux * xx) / n))
            out[ky, kx] = acc / n
    return out


@pytest.mark.parametrize("n", [4, 6, 8, 12, 16])
def test_spectrum_matches_brute_force_dft(n):
    rng = np.random.default_rng(n)
    O = rand_complex(rng, (n, n))
    ref = brute_centred_dft(O)
    got = orc.spectrum_from_object(O)
    assert np.max(np.abs(got - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref)))
    back = orc.object_from_spectrum(got)
    assert np.max(np.abs(back - O)) < 1e-13


@pytest.mark.parametrize("n,r", [(4, 2), (8, 2), (8, 4), (6, 3)])
def test_lowres_operator_matches_brute_force(n, r):
    # o(x) = (1 / (r n)) * sum_u X[u + n/2] exp(+2 pi i u.x / n)
    rng = np.random.default_rng(100 + n)
    X = rand_complex(rng, (n, n))
    ref = np.zeros((n, n), dtype=np.complex128)
    for yy in range(n):
        for xx in range(n):
            acc = 0j
            for ky in range(n):
                for kx in range(n):
                    ph = 2 * math.pi * ((ky - n // 2) * yy + (kx - n // 2) * xx) / n
                    acc += X[ky, kx] * complex(math.cos(ph), math.sin(ph))
            ref[yy, xx] = acc / (r * n)
    got = orc.lowres_field(X, r)
    assert np.max(np.abs(got - ref)) < 1e-13


def test_parseval():
    rng = np.random.default_rng(7)
    O = rand_complex(rng, (64, 64))
    psi = orc.spectrum_from_object(O)
    assert abs(np.linalg.norm(psi) / np.linalg.norm(O) - 1.0) < 1e-14


def _problem_for(optics, led_k, **kw):
    return orc.problem_from_optics(optics, led_k, **kw)


def test_uniform_object_gives_uniform_field_on_axis():
    optics = synth.Optics(n_lo=16, upsample=4, led_grid=3)
    c = 0.7 - 0.2j
    O = np.full((optics.n_hi, optics.n_hi), c)
    k_axis = np.zeros((1, 2))
    prob = _problem_for(optics, k_axis)
    P = orc.pupil_support(prob).astype(np.complex128)
    o = orc.fields(orc.spectrum_from_object(O), P, prob)[0]
    assert np.max(np.abs(o - c)) < 1e-13


def test_plane_wave_bright_dark_classification():
    """A plane-wave object at spatial frequency f0 is seen by LED k iff |f0 - k| <= NA/lambda;
    the image is then uniform with |o|^2 = 1, else it is zero (physical cut-off of the lens)."""
    optics = synth.Optics(n_lo=32, upsample=4, led_grid=5)
    pos = synth.led_grid_positions(optics.led_grid, optics.pitch_mm)
    k = synth.led_wavevectors(pos, optics.height_mm, optics.wavelength_um)
    prob = _problem_for(optics, k)
    fov = optics.n_lo * optics.dx_lo_um
    n = optics.n_hi
    yy, xx = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    cutoff = optics.na / optics.wavelength_um
    P = orc.pupil_support(prob).astype(np.complex128)
    checked = 0
    for (ux, uy) in [(0, 0), (5, -3), (12, 2), (-7, 9), (20, 0)]:
        O = np.exp(2j * math.pi * (ux * xx + uy * yy) / n)
        inten = orc.intensities(orc.spectrum_from_object(O), P, prob)
        f0 = np.array([ux, uy]) / fov
        for kk in range(k.shape[0]):
            dist = np.linalg.norm(f0 - k[kk])
            # stay clear of the rounded disc edge (LED offsets are rounded to whole pixels)
            if abs(dist - cutoff) * fov < 1.5:
                continue
            expect = 1.0 if dist < cutoff else 0.0
            assert np.max(np.abs(inten[kk] - expect)) < 1e-12
            checked += 1
    assert checked > 60


def test_window_offsets_against_config_geometry():
    """Config-1 optics: dx = 1.625 um, FOV = 52 um, R = 10 px; offsets 0, +-4, +-9 per axis."""
    case = synth.config_case(1)
    prob = _problem_for(case.optics, case.led_k)
    assert abs(orc.pupil_radius_px(prob) - 10.0) < 1e-12
    off = orc.led_offsets(prob)
    assert sorted(set(off[:, 0].tolist())) == [-9, -4, 0, 4, 9]
    assert int(orc.pupil_support(prob).sum()) == 317


def test_config2_support_and_coverage_counts():
    """Config-2 geometry: R = 40 px, 5025 support pixels, coverage of the spectrum by the
    225 LED discs has max 22 and covers 95965 pixels (integer counts, no floating point)."""
    case = synth.make_case(synth.Optics(n_lo=128, upsample=4, led_grid=15), [2, 0])
    prob = _problem_for(case.optics, case.led_k)
    S = orc.pupil_support(prob)
    assert int(S.sum()) == 5025
    cov = np.zeros((prob.n_hi, prob.n_hi), dtype=np.int64)
    for o in orc.window_origins(prob):
        cov[o[0]:o[0] + 128, o[1]:o[1] + 128] += S
    assert int(cov.max()) == 22
    assert int((cov > 0).sum()) == 95965


def _dot(a, b):
    return np.vdot(a.ravel(), b.ravel())


@pytest.mark.parametrize("op,opT", [
    (orc.dx, orc.dx_T), (orc.dy, orc.dy_T), (orc.hxx, orc.hxx_T),
    (orc.hyy, orc.hyy_T), (orc.hxy, orc.hxy_T)])
def test_stencil_adjoints(op, opT):
    rng = np.random.default_rng(3)
    x = rng.standard_normal((9, 11))
    y = rng.standard_normal((9, 11))
    assert abs(_dot(op(x), y) - _dot(x, opT(y))) < 1e-12


def test_transform_adjoints():
    rng = np.random.default_rng(4)
    x = rand_complex(rng, (8, 8))
    y = rand_complex(rng, (8, 8))
    assert abs(_dot(orc.lowres_field(x, 2), y) - _dot(x, orc.lowres_field_adjoint(y, 2))) < 1e-13
    # object_from_spectrum is unitary: its adjoint is its inverse
    assert abs(_dot(orc.object_from_spectrum(x), y) - _dot(x, orc.spectrum_from_object(y))) < 1e-12
    big = rand_complex(rng, (16, 16))
    w = rand_complex(rng, (8, 8))
    assert abs(_dot(orc.crop(big, (3, 5), 8), w) - _dot(big, orc.crop_adjoint(w, (3, 5), 16))) < 1e-12


def test_stencil_closed_forms():
    n = 10
    yy, xx = np.meshgrid(np.arange(n, dtype=float), np.arange(n, dtype=float), indexing="ij")
    aff = 1.5 + 0.3 * xx - 0.7 * yy
    for op in (orc.hxx, orc.hyy, orc.hxy):
        assert np.max(np.abs(op(aff))) < 1e-12
    assert np.allclose(orc.hxx(xx ** 2)[:, 1:-1], 2.0)
    assert np.allclose(orc.hxx(xx ** 2)[:, [0, -1]], 0.0)
    assert np.allclose(orc.hyy(yy ** 2)[1:-1, :], 2.0)
    assert np.allclose(orc.hxy(xx * yy)[:-1, :-1], 1.0)
    assert np.allclose(orc.hxy(xx * yy)[-1, :], 0.0)
    assert np.allclose(orc.dx(xx)[:, :-1], 1.0) and np.allclose(orc.dx(xx)[:, -1], 0.0)
    assert np.allclose(orc.dy(yy)[:-1, :], 1.0) and np.allclose(orc.dy(yy)[-1, :], 0.0)


def test_window_outside_spectrum_is_rejected():
    optics = synth.Optics(n_lo=16, upsample=2, led_grid=3)
    far = np.array([[5.0, 0.0]])  # 5 cycles/um * 26 um = 130 px: far outside
    prob = _problem_for(optics, far)
    with pytest.raises(ValueError):
        orc.window_origins(prob)


def test_initial_state_of_uniform_stack_is_uniform_object():
    """A uniform stack I = c^2 must initialise Psi to the spectrum of the uniform object c:
    a single DC term c * n_hi (unitary transform), so that O0 = c everywhere."""
    optics = synth.Optics(n_lo=16, upsample=4, led_grid=3)
    pos = synth.led_grid_positions(3, optics.pitch_mm)
    k = synth.led_wavevectors(pos, optics.height_mm, optics.wavelength_um)
    prob = _problem_for(optics, k, flags=orc.PUPIL_SUPPORT)
    c = 0.8
    st = orc.init_state(np.full((prob.K, 16, 16), c * c), prob)
    n = prob.n_hi
    assert abs(st.psi[n // 2, n // 2] - c * n) < 1e-12
    st.psi[n // 2, n // 2] = 0
    assert np.max(np.abs(st.psi)) < 1e-12
    O0 = orc.object_from_spectrum(orc.init_state(np.full((prob.K, 16, 16), c * c), prob).psi)
    assert np.max(np.abs(O0 - c)) < 1e-12
