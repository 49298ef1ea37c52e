"""Plain FP64 CPU oracle for one Elfpie iteration.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call this
module: only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark use it.  It shares no code with the HIP library; the only module both
sides use is ``synth`` (seeded data generation, no method arithmetic).

Everything is NumPy complex128 / float64, written to be read against the paper
(Zhang, Berendschot, Zhou, "ELFPIE: an error-laxity Fourier ptychographic
iterative engine", arXiv 2209.14671):

* forward model, Sec. 3.1 Eq. (1), one LED per exposure (M = 1, Sec. 4.1) or M
  LEDs lit together (multiplexed illumination, the general form of Eq. 1);
* data fidelity on image gradients, Sec. 3.2 Eq. (4) amplitude / Eq. (5) intensity,
  with the L1 normaliser of Eq. (12) (anisotropic sign or isotropic), and the other
  scalings g of Eq. (3) that Sec. 6.3 tries: x^gamma and ln(x + 1);
* Hessian penalties on amplitude and phase, Eq. (6), (7), combined by Eq. (8);
* closed-form Wirtinger gradients, Eq. (9)-(11), (13)-(15) for the spectrum and
  Eq. (18) for the pupil;
* the modified AdaBelief update, Eq. (19), and the order of Algorithm 1, including
  the 3x3 Gaussian pre-filter of the pupil noted under Algorithm 1; for the
  comparison of Sec. 6.2 also plain gradient descent, NAdam and AdaBelief, from
  their published definitions;
* the automatic penalty weight of Eq. (16) / (17).

Where the paper is silent or inconsistent the readings below are used (each is
listed with its reason in the design notes):

* transforms: Psi is the centred unitary forward DFT of O,
  ``Psi = fftshift(fft2(O)) / n_hi`` and ``O = n_hi * ifft2(ifftshift(Psi))``;
  the low-resolution operator is ``o = (n_lo / r) * ifft2(ifftshift(P * crop(Psi)))``,
  so a uniform object c gives o = c under the on-axis LED;
* LED k crops the n_lo x n_lo window of Psi centred at ``n_hi/2 + round(k * FOV)``
  (round half away from zero), rows = y, columns = x;
* pupil support: the disc ``(x - n/2)^2 + (y - n/2)^2 <= R^2 (1 + 1e-12)`` with
  ``R = NA * FOV / lambda``; with the support flag the effective pupil is ``P * 1_S``;
* image gradient: forward differences, zero in the last column / row;
  Hessian: [1,-2,1] along x and along y, and the forward mixed difference,
  each zero where its stencil leaves the grid;
* L1 terms use rho(x) = sqrt(x^2 + eps^2) - eps (eps = 0 gives |x| with the
  subgradient 0 at 0, as stated in Sec. 3.3);
* gradients are the exact dL/d(conj Psi): the amplitude fidelity carries the
  Wirtinger factor 1/2 (Eq. (10) as printed omits it), and the intensity fidelity
  differentiates |o|^2 - I (Eq. (11) as printed repeats the amplitude residual);
* Eq. (19): g = dL/d(conj Psi), delta^0 = lr^2, t counts from 1 and is shared by
  Psi and P; two separate small constants eta_h (Eq. 14) and eta_opt (Eq. 19).

Pins (tests, CPU): brute-force DFT sums, Parseval, closed-form forward cases,
adjoint dot products, stencil closed forms, central finite differences of the
loss against every gradient term, the zero-residual case, closed-form AdaBelief
steps, the Gaussian weights, and a noise-free recovery.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

FID_AMPLITUDE = 0
FID_INTENSITY = 1
FID_GAMMA = 2     # g(x) = x^gamma in Eq. (3), Sec. 6.3
FID_LOG = 3       # g(x) = ln(x + 1) in Eq. (3), Sec. 6.3
NORM_ANISO = 0
NORM_ISO = 1
LEARN_PUPIL = 1
PUPIL_SUPPORT = 2
PUPIL_FILTER = 4
# optimisers compared in Sec. 6.2 (Fig. 13): the paper's Eq. (19) and three published ones
OPT_ELFPIE = 0      # Eq. (19)
OPT_SGD = 1         # plain gradient descent
OPT_NADAM = 2       # Nesterov-accelerated Adam (Dozat, 2016), constant momentum
OPT_ADABELIEF = 3   # AdaBelief (Zhuang et al., 2020)


@dataclasses.dataclass
class Problem:
    """Problem statement (Algorithm 1 inputs plus the optics of Sec. 4.1)."""
    n_lo: int
    upsample: int
    led_k: np.ndarray                 # (K, 2) (kx, ky) in 1/um
    wavelength_um: float
    na: float
    dx_lo_um: float
    alpha: float = 1e-3               # Eq. (8)
    beta: float = 1e-3                # Eq. (8)
    lr: float = 1e-2                  # Eq. (19): delta^0 = lr^2
    gamma1: float = 0.9               # Eq. (19)
    gamma2: float = 0.999             # Eq. (19)
    eta_opt: float = 1e-8             # Eq. (19)
    eta_h: float = 1e-6               # Eq. (14)
    l1_eps: float = 0.0               # smoothing of the L1 terms (0 = exact)
    fidelity: int = FID_INTENSITY     # Eq. (4), Eq. (5), or g of Eq. (3) (Sec. 6.3)
    norm: int = NORM_ANISO            # Eq. (12)
    flags: int = PUPIL_SUPPORT
    fid_gamma: float = 0.5            # the exponent of FID_GAMMA
    optimizer: int = OPT_ELFPIE       # update rule for Psi and P (Sec. 6.2)
    mux: int = 1                      # M of Eq. (1): LEDs lit together per image

    @property
    def n_hi(self) -> int:
        return self.n_lo * self.upsample

    @property
    def n_led(self) -> int:
        """Number of LEDs (rows of led_k); image n is lit by LEDs n M .. n M + M - 1."""
        return int(self.led_k.shape[0])

    @property
    def K(self) -> int:
        """Number of images (N of Eq. 1)."""
        return self.n_led // self.mux

    @property
    def fov_um(self) -> float:
        return self.n_lo * self.dx_lo_um


@dataclasses.dataclass
class State:
    """Optimised variables and the Eq. (19) moments for Psi and for P."""
    psi: np.ndarray
    P: np.ndarray
    mu_psi: np.ndarray
    v_psi: np.ndarray
    delta_psi: np.ndarray
    mu_P: np.ndarray
    v_P: np.ndarray
    delta_P: np.ndarray
    t: int = 0

    def copy(self) -> "State":
        return State(*(np.array(getattr(self, f.name), copy=True) if f.name != "t" else self.t
                       for f in dataclasses.fields(self)))


# ----------------------------------------------------------------------------
# Plan: LED windows and pupil support (Sec. 3.1, M_{n,m} and P)
# ----------------------------------------------------------------------------

def round_half_away(x):
    x = np.asarray(x, dtype=np.float64)
    return (np.sign(x) * np.floor(np.abs(x) + 0.5)).astype(np.int64)


def led_offsets(prob: Problem) -> np.ndarray:
    """(n_led, 2) integer spectral offsets (off_x, off_y) = round(k * FOV)."""
    return round_half_away(prob.led_k * prob.fov_um)


def window_origins(prob: Problem) -> np.ndarray:
    """(n_led, 2) top-left corner (row y0, column x0) of each LED's crop window in Psi."""
    off = led_offsets(prob)
    c = prob.n_hi // 2 - prob.n_lo // 2
    y0 = c + off[:, 1]
    x0 = c + off[:, 0]
    if (y0.min() < 0 or x0.min() < 0 or y0.max() + prob.n_lo > prob.n_hi
            or x0.max() + prob.n_lo > prob.n_hi):
        raise ValueError("an LED window falls outside the high-resolution spectrum")
    return np.stack([y0, x0], axis=1)


def pupil_radius_px(prob: Problem) -> float:
    return prob.na * prob.fov_um / prob.wavelength_um


def pupil_support(prob: Problem) -> np.ndarray:
    """Boolean (n_lo, n_lo) disc of the objective's passband, centred at (n_lo/2, n_lo/2)."""
    n = prob.n_lo
    r = pupil_radius_px(prob)
    idx = np.arange(n) - n // 2
    d2 = idx[None, :] ** 2 + idx[:, None] ** 2
    return d2 <= r * r * (1.0 + 1e-12)


def effective_pupil(P: np.ndarray, prob: Problem) -> np.ndarray:
    return P * pupil_support(prob) if prob.flags & PUPIL_SUPPORT else P


def crop(psi: np.ndarray, origin, n: int) -> np.ndarray:
    """M_k Psi: the n x n window of Psi whose top-left corner is ``origin``."""
    y0, x0 = int(origin[0]), int(origin[1])
    return psi[y0:y0 + n, x0:x0 + n]


def crop_adjoint(w: np.ndarray, origin, n_hi: int) -> np.ndarray:
    """M_k^T w: place the window back into an all-zero n_hi x n_hi spectrum."""
    out = np.zeros((n_hi, n_hi), dtype=np.result_type(w, np.complex128))
    y0, x0 = int(origin[0]), int(origin[1])
    n = w.shape[0]
    out[y0:y0 + n, x0:x0 + n] = w
    return out


# ----------------------------------------------------------------------------
# Centred unitary transforms (F_A, F_B of Sec. 3.1)
# ----------------------------------------------------------------------------

def spectrum_from_object(O: np.ndarray) -> np.ndarray:
    """Psi = fftshift(fft2(O)) / n   (unitary, DC at [n/2, n/2])."""
    n = O.shape[-1]
    return np.fft.fftshift(np.fft.fft2(O), axes=(-2, -1)) / n


def object_from_spectrum(psi: np.ndarray) -> np.ndarray:
    """O = n * ifft2(ifftshift(Psi))   (inverse of ``spectrum_from_object``)."""
    n = psi.shape[-1]
    return n * np.fft.ifft2(np.fft.ifftshift(psi, axes=(-2, -1)))


def lowres_field(X: np.ndarray, upsample: int) -> np.ndarray:
    """o = (n_lo / r) * ifft2(ifftshift(X)): F_B applied to a pupil-filtered window."""
    n = X.shape[-1]
    return (n / upsample) * np.fft.ifft2(np.fft.ifftshift(X, axes=(-2, -1)))


def lowres_field_adjoint(w: np.ndarray, upsample: int) -> np.ndarray:
    """Adjoint of ``lowres_field``: fftshift(fft2(w)) / (r * n_lo)."""
    n = w.shape[-1]
    return np.fft.fftshift(np.fft.fft2(w), axes=(-2, -1)) / (upsample * n)


# ----------------------------------------------------------------------------
# Forward model, Eq. (1)
# ----------------------------------------------------------------------------

def fields(psi: np.ndarray, P: np.ndarray, prob: Problem) -> np.ndarray:
    """(n_led, n_lo, n_lo) complex low-resolution fields o_k = F_B P M_k Psi, one per LED."""
    org = window_origins(prob)
    Pe = effective_pupil(P, prob)
    out = np.empty((prob.n_led, prob.n_lo, prob.n_lo), dtype=np.complex128)
    for k in range(prob.n_led):
        out[k] = lowres_field(Pe * crop(psi, org[k], prob.n_lo), prob.upsample)
    return out


def intensities(psi: np.ndarray, P: np.ndarray, prob: Problem) -> np.ndarray:
    """Ideal measured stack, Eq. (1): image n is sum_m |o_(n, m)|^2 over its M LEDs."""
    p = np.abs(fields(psi, P, prob)) ** 2
    return p.reshape(prob.K, prob.mux, prob.n_lo, prob.n_lo).sum(axis=1)


# ----------------------------------------------------------------------------
# Finite-difference operators: image gradient (Theta = grad, Sec. 3.2) and the
# Hessian H = grad grad (Eq. 6-7)
# ----------------------------------------------------------------------------

def dx(f):
    out = np.zeros_like(f)
    out[..., :, :-1] = f[..., :, 1:] - f[..., :, :-1]
    return out


def dy(f):
    out = np.zeros_like(f)
    out[..., :-1, :] = f[..., 1:, :] - f[..., :-1, :]
    return out


def dx_T(w):
    """Adjoint of ``dx``: each output w[.., x] (x < n-1) adds +w to x+1 and -w to x."""
    out = np.zeros_like(w)
    wv = w[..., :, :-1]
    out[..., :, 1:] += wv
    out[..., :, :-1] -= wv
    return out


def dy_T(w):
    out = np.zeros_like(w)
    wv = w[..., :-1, :]
    out[..., 1:, :] += wv
    out[..., :-1, :] -= wv
    return out


def hxx(f):
    out = np.zeros_like(f)
    out[..., :, 1:-1] = f[..., :, :-2] - 2.0 * f[..., :, 1:-1] + f[..., :, 2:]
    return out


def hyy(f):
    out = np.zeros_like(f)
    out[..., 1:-1, :] = f[..., :-2, :] - 2.0 * f[..., 1:-1, :] + f[..., 2:, :]
    return out


def hxy(f):
    out = np.zeros_like(f)
    out[..., :-1, :-1] = f[..., :-1, :-1] - f[..., :-1, 1:] - f[..., 1:, :-1] + f[..., 1:, 1:]
    return out


def hxx_T(w):
    out = np.zeros_like(w)
    wv = w[..., :, 1:-1]
    out[..., :, :-2] += wv
    out[..., :, 1:-1] -= 2.0 * wv
    out[..., :, 2:] += wv
    return out


def hyy_T(w):
    out = np.zeros_like(w)
    wv = w[..., 1:-1, :]
    out[..., :-2, :] += wv
    out[..., 1:-1, :] -= 2.0 * wv
    out[..., 2:, :] += wv
    return out


def hxy_T(w):
    out = np.zeros_like(w)
    wv = w[..., :-1, :-1]
    out[..., :-1, :-1] += wv
    out[..., :-1, 1:] -= wv
    out[..., 1:, :-1] -= wv
    out[..., 1:, 1:] += wv
    return out


# ----------------------------------------------------------------------------
# L1 terms and their normaliser omega, Eq. (12)
# ----------------------------------------------------------------------------

def l1_value_and_omega(comps, norm: int, eps: float):
    """Sum of rho over the components ``comps`` (list of equal-shape real arrays) and the
    per-component derivative omega.  Anisotropic: sum_c rho(c); isotropic: rho(||c||_2)."""
    if norm == NORM_ANISO:
        val = 0.0
        om = []
        for c in comps:
            if eps > 0:
                r = np.sqrt(c * c + eps * eps)
                val += float(np.sum(r - eps))
                om.append(c / r)
            else:
                val += float(np.sum(np.abs(c)))
                om.append(np.sign(c))
        return val, om
    sq = sum(c * c for c in comps)
    if eps > 0:
        r = np.sqrt(sq + eps * eps)
        val = float(np.sum(r - eps))
        return val, [c / r for c in comps]
    r = np.sqrt(sq)
    val = float(np.sum(r))
    inv = np.divide(1.0, r, out=np.zeros_like(r), where=r > 0)
    return val, [c * inv for c in comps]


# ----------------------------------------------------------------------------
# Loss and closed-form gradients
# ----------------------------------------------------------------------------

def scaling(x: np.ndarray, fidelity: int, gamma: float = 0.5) -> np.ndarray:
    """The pixel-wise scaling g of Eq. (3) applied to intensities x >= 0: sqrt (Eq. 4),
    identity (Eq. 5), x^gamma or ln(x + 1) (Sec. 6.3)."""
    if fidelity == FID_AMPLITUDE:
        return np.sqrt(x)
    if fidelity == FID_GAMMA:
        return x ** gamma
    if fidelity == FID_LOG:
        return np.log1p(x)
    return x


def scaling_slope(x: np.ndarray, fidelity: int, gamma: float = 0.5) -> np.ndarray:
    """g'(x) for x > 0; 0 where x = 0 for the powers (their slope is unbounded there)."""
    if fidelity == FID_AMPLITUDE:
        return np.divide(0.5, np.sqrt(x), out=np.zeros_like(x), where=x > 0)
    if fidelity == FID_GAMMA:
        return np.where(x > 0, gamma * np.power(np.where(x > 0, x, 1.0), gamma - 1.0), 0.0)
    if fidelity == FID_LOG:
        return 1.0 / (1.0 + x)
    return np.ones_like(x)


def fidelity_residual(o: np.ndarray, meas: np.ndarray, fidelity: int, gamma: float = 0.5):
    """Residual inside the gradient operator, g(|o|^2) - g(I): |o| - sqrt(I) (Eq. 4),
    |o|^2 - I (Eq. 5), or the gamma / log scalings of Sec. 6.3 (negative readings of a
    noisy I are taken as 0 wherever g needs x >= 0)."""
    if fidelity == FID_AMPLITUDE:
        return np.abs(o) - np.sqrt(np.clip(meas, 0.0, None))
    if fidelity == FID_INTENSITY:
        return np.abs(o) ** 2 - meas
    return scaling(np.abs(o) ** 2, fidelity, gamma) - scaling(np.clip(meas, 0.0, None), fidelity, gamma)


def fidelity_loss_and_grad(psi, P, meas, prob: Problem, want_grad: bool = True):
    """L_fid and its Wirtinger gradients wrt conj(Psi) (Eq. 9) and conj(P) (Eq. 18).

    For every image n: o_m = F_B P M_(n, m) Psi for its M LEDs, S = sum_m |o_m|^2
    (Eq. 1); e = g(S) - g(I_n); L += rho(grad e); dL/de = grad^T omega;
    dL/d(conj o_m) = dL/de * g'(S) * o_m, which is dL/de * o / (2|o|) for the
    amplitude and dL/de * o for the intensity when M = 1; back-projection
    Y_m = F_B^H dL/d(conj o_m); then g_Psi += M^T (conj(P) Y_m) and
    g_P += conj(M Psi) Y_m, LEDs in ascending order.
    """
    org = window_origins(prob)
    Pe = effective_pupil(P, prob)
    n = prob.n_lo
    L = 0.0
    g_psi = np.zeros_like(psi, dtype=np.complex128) if want_grad else None
    g_P = np.zeros((n, n), dtype=np.complex128) if want_grad else None
    for img in range(prob.K):
        leds = range(img * prob.mux, (img + 1) * prob.mux)
        cs = [crop(psi, org[k], n) for k in leds]
        os_ = [lowres_field(Pe * c, prob.upsample) for c in cs]
        if prob.mux == 1:
            e = fidelity_residual(os_[0], meas[img], prob.fidelity, prob.fid_gamma)
        else:
            S = sum(np.abs(o) ** 2 for o in os_)
            if prob.fidelity == FID_INTENSITY:
                e = S - meas[img]
            else:
                e = scaling(S, prob.fidelity, prob.fid_gamma) - scaling(np.clip(meas[img], 0.0, None),
                                                                        prob.fidelity, prob.fid_gamma)
        val, (wx, wy) = l1_value_and_omega([dx(e), dy(e)], prob.norm, prob.l1_eps)
        L += val
        if not want_grad:
            continue
        q = dx_T(wx) + dy_T(wy)
        for k, c, o in zip(leds, cs, os_):
            if prob.mux > 1:
                dob = q * scaling_slope(S, prob.fidelity, prob.fid_gamma) * o
            elif prob.fidelity == FID_AMPLITUDE:
                a = np.abs(o)
                dob = np.divide(q * o, 2.0 * a, out=np.zeros_like(o), where=a > 0)
            elif prob.fidelity == FID_INTENSITY:
                dob = q * o
            else:
                dob = q * scaling_slope(np.abs(o) ** 2, prob.fidelity, prob.fid_gamma) * o
            Y = lowres_field_adjoint(dob, prob.upsample)
            g_psi[org[k][0]:org[k][0] + n, org[k][1]:org[k][1] + n] += np.conj(Pe) * Y
            g_P += np.conj(c) * Y
    if want_grad and prob.flags & PUPIL_SUPPORT:
        g_P *= pupil_support(prob)
    return L, g_psi, g_P


def hessian_loss_and_grad(psi, prob: Problem, want_grad: bool = True):
    """L_A = ||H|O|||_1 (Eq. 6), L_Phi = ||H angle(O)||_1 (Eq. 7) and the gradient
    alpha * Eq. (13) + beta * Eq. (14) wrt conj(Psi)."""
    O = object_from_spectrum(psi)
    a = np.abs(O)
    ph = np.arctan2(O.imag, O.real)
    LA, (oxx, oyy, oxy) = l1_value_and_omega([hxx(a), hyy(a), hxy(a)], prob.norm, prob.l1_eps)
    LP, (pxx, pyy, pxy) = l1_value_and_omega([hxx(ph), hyy(ph), hxy(ph)], prob.norm, prob.l1_eps)
    if not want_grad:
        return LA, LP, None
    qa = hxx_T(oxx) + hyy_T(oyy) + hxy_T(oxy)
    qp = hxx_T(pxx) + hyy_T(pyy) + hxy_T(pxy)
    unit = np.divide(O, a, out=np.zeros_like(O), where=a > 0)
    den = a * a + prob.eta_h
    phase_dir = np.divide(O, den, out=np.zeros_like(O), where=den > 0)
    G = prob.alpha * 0.5 * qa * unit + prob.beta * 0.5j * qp * phase_dir
    g = spectrum_from_object(G)
    return LA, LP, g


def loss_and_grad(psi, P, meas, prob: Problem, want_grad: bool = True):
    """Eq. (8) loss terms [L_fid, L_A, L_Phi, L] and Eq. (15) / Eq. (18) gradients."""
    Lf, g_psi, g_P = fidelity_loss_and_grad(psi, P, meas, prob, want_grad)
    LA, LP, gH = hessian_loss_and_grad(psi, prob, want_grad)
    loss4 = np.array([Lf, LA, LP, Lf + prob.alpha * LA + prob.beta * LP])
    if want_grad:
        g_psi = g_psi + gH
    return loss4, g_psi, g_P


def loss(psi, P, meas, prob: Problem) -> float:
    return float(loss_and_grad(psi, P, meas, prob, want_grad=False)[0][3])


# ----------------------------------------------------------------------------
# Optimiser, Eq. (19), and the pupil pre-filter noted under Algorithm 1
# ----------------------------------------------------------------------------

def adabelief(x, g, mu, v, delta, t: int, prob: Problem):
    """One modified-AdaBelief step (Eq. 19) at step count ``t`` (>= 1); returns new
    (x, mu, v, delta).  All arrays elementwise; |.|^2 is the squared modulus."""
    g1, g2, eta = prob.gamma1, prob.gamma2, prob.eta_opt
    mu = g1 * mu + (1.0 - g1) * g
    v = g2 * v + (1.0 - g2) * np.abs(mu - g) ** 2
    mu_hat = mu / (1.0 - g1 ** t)
    v_hat = v / (1.0 - g2 ** t)
    step = (np.sqrt(delta) + eta) / (np.sqrt(v_hat) + eta) * (g1 * mu_hat + (1.0 - g1) * g)
    x = x - step
    delta = g1 * delta + (1.0 - g1) * np.abs(step) ** 2
    return x, mu, v, delta


def sgd(x, g, prob: Problem):
    """Gradient descent with step lr along g = dL/d(conj x)."""
    return x - prob.lr * g


def nadam(x, g, m, v, t: int, prob: Problem):
    """Adam with a Nesterov look-ahead of the first moment (Dozat, 2016; constant
    momentum gamma1): m and v are the usual moments (v of the squared modulus), the
    step uses gamma1 m_t / (1 - gamma1^(t+1)) + (1 - gamma1) g / (1 - gamma1^t)."""
    g1, g2, eps = prob.gamma1, prob.gamma2, prob.eta_opt
    m = g1 * m + (1.0 - g1) * g
    v = g2 * v + (1.0 - g2) * np.abs(g) ** 2
    m_hat = g1 * m / (1.0 - g1 ** (t + 1)) + (1.0 - g1) * g / (1.0 - g1 ** t)
    v_hat = v / (1.0 - g2 ** t)
    return x - prob.lr * m_hat / (np.sqrt(v_hat) + eps), m, v


def adabelief_plain(x, g, m, s, t: int, prob: Problem):
    """AdaBelief (Zhuang et al., 2020): the second moment tracks (g - m)^2 (squared
    modulus here) plus eps; step lr * m_hat / (sqrt(s_hat) + eps)."""
    g1, g2, eps = prob.gamma1, prob.gamma2, prob.eta_opt
    m = g1 * m + (1.0 - g1) * g
    s = g2 * s + (1.0 - g2) * np.abs(g - m) ** 2 + eps
    m_hat = m / (1.0 - g1 ** t)
    s_hat = s / (1.0 - g2 ** t)
    return x - prob.lr * m_hat / (np.sqrt(s_hat) + eps), m, s


def optimizer_step(x, g, mu, v, delta, t: int, prob: Problem):
    """The update rule selected by prob.optimizer; returns (x, mu, v, delta).  delta is
    used by Eq. (19) only, mu and v by the moment methods."""
    if prob.optimizer == OPT_SGD:
        return sgd(x, g, prob), mu, v, delta
    if prob.optimizer == OPT_NADAM:
        x, mu, v = nadam(x, g, mu, v, t, prob)
        return x, mu, v, delta
    if prob.optimizer == OPT_ADABELIEF:
        x, mu, v = adabelief_plain(x, g, mu, v, t, prob)
        return x, mu, v, delta
    return adabelief(x, g, mu, v, delta, t, prob)


def gauss3_weights() -> np.ndarray:
    """Normalised 3x3 Gaussian kernel of standard deviation 1 pixel."""
    d = np.arange(-1, 2)
    w = np.exp(-(d[:, None] ** 2 + d[None, :] ** 2) / 2.0)
    return w / w.sum()


def gauss3(P: np.ndarray) -> np.ndarray:
    """3x3 Gaussian filter with zero padding (pre-filter of P before its update)."""
    w = gauss3_weights()
    n0, n1 = P.shape
    pad = np.zeros((n0 + 2, n1 + 2), dtype=P.dtype)
    pad[1:-1, 1:-1] = P
    out = np.zeros_like(P)
    for i in range(3):
        for j in range(3):
            out += w[i, j] * pad[i:i + n0, j:j + n1]
    return out


# ----------------------------------------------------------------------------
# Algorithm 1
# ----------------------------------------------------------------------------

def new_state(psi0: np.ndarray, P0: np.ndarray, prob: Problem) -> State:
    return State(
        psi=np.array(psi0, dtype=np.complex128), P=np.array(P0, dtype=np.complex128),
        mu_psi=np.zeros_like(psi0, dtype=np.complex128), v_psi=np.zeros(psi0.shape),
        delta_psi=np.full(psi0.shape, prob.lr ** 2),
        mu_P=np.zeros_like(P0, dtype=np.complex128), v_P=np.zeros(P0.shape),
        delta_P=np.full(P0.shape, prob.lr ** 2), t=0)


def init_state(meas: np.ndarray, prob: Problem) -> State:
    """Initial guess: the on-axis-most LED's window holds the unitary-scaled spectrum of
    sqrt(I) on the pupil support (the whole window without the support flag), zeros
    elsewhere; P0 = 1 there."""
    org = window_origins(prob)
    kc = int(np.argmin(np.sum(prob.led_k ** 2, axis=1)))
    n = prob.n_lo
    S = pupil_support(prob) if prob.flags & PUPIL_SUPPORT else np.ones((n, n), dtype=bool)
    img = kc // prob.mux  # the image that the on-axis-most LED lights
    spec = (prob.upsample / n) * np.fft.fftshift(np.fft.fft2(np.sqrt(np.clip(meas[img], 0, None))))
    psi0 = np.zeros((prob.n_hi, prob.n_hi), dtype=np.complex128)
    psi0[org[kc][0]:org[kc][0] + n, org[kc][1]:org[kc][1] + n] = spec * S
    return new_state(psi0, S.astype(np.complex128), prob)


def step(state: State, meas: np.ndarray, prob: Problem):
    """One Elfpie iteration (Algorithm 1).  Returns (new_state, loss4 at the old state)."""
    loss4, g_psi, g_P = loss_and_grad(state.psi, state.P, meas, prob)
    s = state.copy()
    s.t = state.t + 1
    s.psi, s.mu_psi, s.v_psi, s.delta_psi = optimizer_step(
        state.psi, g_psi, state.mu_psi, state.v_psi, state.delta_psi, s.t, prob)
    if prob.flags & LEARN_PUPIL:
        P = gauss3(state.P) if prob.flags & PUPIL_FILTER else state.P
        s.P, s.mu_P, s.v_P, s.delta_P = optimizer_step(
            P, g_P, state.mu_P, state.v_P, state.delta_P, s.t, prob)
        if prob.flags & PUPIL_SUPPORT:
            s.P = s.P * pupil_support(prob)
    return s, loss4


def run(state: State, meas: np.ndarray, prob: Problem, n_iter: int):
    hist = np.zeros((n_iter, 4))
    for i in range(n_iter):
        state, hist[i] = step(state, meas, prob)
    return state, hist


# ----------------------------------------------------------------------------
# Evaluation metrics (Sec. 4.1) and the automatic penalty weight (Eq. 16-17)
# ----------------------------------------------------------------------------

def lsnr(phi: np.ndarray, phi_true: np.ndarray) -> float:
    """Eq. (22): max over a scalar offset b of 10 log10(||true||^2 / ||true - (phi + b)||^2).
    The optimum offset is b* = mean(true - phi)."""
    b = float(np.mean(phi_true - phi))
    den = float(np.sum((phi_true - phi - b) ** 2))
    num = float(np.sum(phi_true ** 2))
    return math.inf if den == 0 else 10.0 * math.log10(num / den)


def noise_level(clean: np.ndarray, noisy: np.ndarray, dark: np.ndarray) -> float:
    """Eq. (21): mean over dark-field images of ||I_simu - I_noised||_1 / ||I_simu||_1, in %."""
    r = [np.sum(np.abs(clean[k] - noisy[k])) / np.sum(np.abs(clean[k])) for k in np.flatnonzero(dark)]
    return 100.0 * float(np.mean(r)) if r else 0.0


def auto_penalty(meas: np.ndarray, fidelity: int, gamma: float = 0.5) -> float:
    """Eq. (16) (intensity) / Eq. (17) (amplitude): alpha = beta from the stack, with the
    3x3 mask as printed and a 'valid' convolution averaged over W*H pixels.  For the
    Sec. 6.3 scalings the mask is applied to g(I), as Eq. (17) applies it to sqrt(I)."""
    mask = np.array([[-1.0, 2.0, -1.0], [-2.0, 4.0, -2.0], [-1.0, 2.0, -1.0]])
    if fidelity == FID_INTENSITY:
        src = meas
    else:
        src = scaling(np.clip(meas, 0, None), fidelity, gamma)
    K, H, W = src.shape
    acc = 0.0
    for k in range(K):
        conv = np.zeros((H - 2, W - 2))
        for i in range(3):
            for j in range(3):
                # convolution flips the kernel; the mask is symmetric under the flip
                conv += mask[2 - i, 2 - j] * src[k, i:i + H - 2, j:j + W - 2]
        acc += np.sum(np.abs(conv)) / (W * H)
    return 0.2 * math.sqrt(math.pi / 2.0) * acc / K


def problem_from_optics(optics, led_k, **kw) -> Problem:
    """Build a Problem from a ``synth.Optics`` and LED wave-vectors."""
    return Problem(n_lo=optics.n_lo, upsample=optics.upsample, led_k=np.asarray(led_k, float),
                   wavelength_um=optics.wavelength_um, na=optics.na, dx_lo_um=optics.dx_lo_um, **kw)
