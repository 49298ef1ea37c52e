"""Sign decisions at near-zero features of the literal L1 (l1_eps = 0), for the GPU tests.

With l1_eps = 0 the normaliser omega of Eq. 12 is the sign of each feature: of the image
differences of the fidelity residual (Eq. 4 / 5) and of the Hessian components of |O| and
angle(O) (Eq. 6, 7).  Sec. 3.3 takes the subgradient 0 at 0.  Where a feature lies within
the FP32 rounding of the library's arithmetic of zero, FP32 and the FP64 oracle may take
different signs there; both are correct evaluations of the method, so these positions
("ties") are where the two may legitimately differ.

The gradient is linear in omega (Eq. 9-11, 13, 14: q = D^T omega or H^T omega, then
pointwise factors, transforms, crops and sums).  So the library's gradient minus the
oracle's is a sum of one known column per tie whose sign differs, times the change of
omega there, plus FP32 rounding.  `infer` lists the ties from the oracle's own values and
a stated FP32 error bound, and finds the library's decision at each tie (coordinate
descent over the allowed sign changes, each column's coefficient by projection).  The
oracle gradient with those decisions (`g_psi`, `g_P`) and the Eq. 19 step built from it
with the oracle's own update functions (`step_from`) are then the references, held to
the usual bounds.  A decision can change only at a listed tie, so an error anywhere else
is not absorbed.

Only the anisotropic form (the default) has sign ties; the isotropic normaliser c / |c|
is continuous away from c = 0 and is compared directly.  Single-LED images only (mux 1).
This module holds test logic; it calls the oracle's functions and adds no arithmetic of
the method beyond the linear columns above.
"""
from __future__ import annotations

import dataclasses

import numpy as np

import oracle as orc

U32 = 2.0 ** -24  # unit roundoff of FP32
# FP32 error of a transformed value, in units of U32 times the rms of the transformed
# array: two radix passes of a 128- or 512-point transform per dimension, FP32 twiddles
# and the crop product leave a few tens of roundings along each path; 64 covers them.
KAPPA = 64.0


@dataclasses.dataclass
class Ties:
    n_fid: int            # fidelity ties listed
    n_hess: int           # Hessian ties listed
    flips_fid: int        # ties where the library's sign differs from the oracle's
    flips_hess: int
    max_abs_flipped: float  # largest |feature| / bound among the flipped ties (<= 1)
    g_psi: np.ndarray     # oracle gradient with the library's decisions
    g_P: np.ndarray
    loss4: np.ndarray     # oracle loss terms (ties change them by less than their bounds)


def _allowed(s):
    """Changes of omega from the oracle's sign s to each sign in {-1, 0, 1}."""
    return np.array([-1.0 - s, 0.0 - s, 1.0 - s])


def _snap(coef, s):
    opts = _allowed(s)
    return float(opts[np.argmin(np.abs(opts - coef))])


def _fidelity_ties(psi, P, meas, prob):
    """Per LED: the fields, the residual's error bound and the tie positions of dx(e), dy(e)."""
    org = orc.window_origins(prob)
    Pe = orc.effective_pupil(P, prob)
    n = prob.n_lo
    out = []
    for k in range(prob.K):
        o = orc.lowres_field(Pe * orc.crop(psi, org[k], n), prob.upsample)
        e = orc.fidelity_residual(o, meas[k], prob.fidelity, prob.fid_gamma)
        rms = np.sqrt(np.mean(np.abs(o) ** 2))
        if prob.fidelity == orc.FID_INTENSITY:
            err = KAPPA * U32 * 2.0 * np.abs(o) * rms + U32 * (np.abs(o) ** 2 + np.abs(meas[k]))
        else:  # amplitude: |o| - sqrt(I)
            err = KAPPA * U32 * rms + 2.0 * U32 * (np.abs(o) + np.sqrt(np.clip(meas[k], 0.0, None)))
        cx, cy = orc.dx(e), orc.dy(e)
        bx = err.copy()
        bx[:, :-1] += err[:, 1:]
        by = err.copy()
        by[:-1, :] += err[1:, :]
        tx = (np.abs(cx) <= bx) & (bx > 0)  # a zero bound: exact zeros on both sides
        tx[:, -1] = False  # structurally zero on both sides
        ty = (np.abs(cy) <= by) & (by > 0)
        ty[-1, :] = False
        items = [(0, y, x, np.sign(cx[y, x]), abs(cx[y, x]) / bx[y, x]) for y, x in zip(*np.nonzero(tx))]
        items += [(1, y, x, np.sign(cy[y, x]), abs(cy[y, x]) / by[y, x]) for y, x in zip(*np.nonzero(ty))]
        out.append((o, items))
    return out


def _fid_column(o, comp, y, x, prob):
    """dL/d(conj o) for a unit change of omega at one feature (before the transform):
    q from the oracle's own adjoint difference, then the fidelity's pointwise factor."""
    w = np.zeros(o.shape)
    w[y, x] = 1.0
    dq = orc.dx_T(w) if comp == 0 else orc.dy_T(w)
    if prob.fidelity == orc.FID_INTENSITY:
        return dq * o
    a = np.abs(o)
    return np.divide(dq * o, 2.0 * a, out=np.zeros_like(o), where=a > 0)


def _hessian_ties(psi, prob):
    O = orc.object_from_spectrum(psi)
    a = np.abs(O)
    ph = np.arctan2(O.imag, O.real)
    rms = np.sqrt(np.mean(a ** 2))
    errO = KAPPA * U32 * rms
    err_a = errO + 2.0 * U32 * a
    err_p = np.divide(errO, a, out=np.full_like(a, np.inf), where=a > 0) + 4.0 * U32 * np.abs(ph)
    items = []
    for f, (src, err) in enumerate(((a, err_a), (ph, err_p))):
        for c, (H, Ht) in enumerate(((orc.hxx, orc.hxx_T), (orc.hyy, orc.hyy_T), (orc.hxy, orc.hxy_T))):
            h = H(src)
            b = np.zeros_like(src)  # sum of |coefficient| x error over the stencil
            if c == 0:
                b[:, 1:-1] = err[:, :-2] + 2.0 * err[:, 1:-1] + err[:, 2:]
            elif c == 1:
                b[1:-1, :] = err[:-2, :] + 2.0 * err[1:-1, :] + err[2:, :]
            else:
                b[:-1, :-1] = err[:-1, :-1] + err[:-1, 1:] + err[1:, :-1] + err[1:, 1:]
            tie = (np.abs(h) <= b) & (b > 0)
            for y, x in zip(*np.nonzero(tie)):
                items.append((f, c, y, x, np.sign(h[y, x]), abs(h[y, x]) / b[y, x]))
    return O, a, items


def _hess_column(O, a, f, c, y, x, prob):
    """G (object domain) for a unit change of omega at one Hessian component, as a
    list of (y, x, value) on the pixels of the oracle's own adjoint stencil."""
    w = np.zeros(a.shape)
    w[y, x] = 1.0
    dq = (orc.hxx_T, orc.hyy_T, orc.hxy_T)[c](w)
    out = []
    for yy, xx in zip(*np.nonzero(dq)):
        Ov, av, q = O[yy, xx], a[yy, xx], dq[yy, xx]
        if f == 0:
            v = prob.alpha * 0.5 * q * (Ov / av if av > 0 else 0.0)
        else:
            den = av * av + prob.eta_h
            v = prob.beta * 0.5j * q * (Ov / den if den > 0 else 0.0)
        out.append((yy, xx, v))
    return out


def infer(pair, g_psi_gpu, g_P_gpu, sweeps=3) -> Ties:
    """The oracle gradient at the pair's state with the library's sign decisions at ties."""
    prob = pair.oprob
    assert prob.l1_eps == 0 and prob.norm == orc.NORM_ANISO and prob.mux == 1
    psi, P, meas = pair.psi, pair.P, pair.meas
    loss4, g0, gP0 = orc.loss_and_grad(psi, P, meas, prob)
    org = orc.window_origins(prob)
    Pe = orc.effective_pupil(P, prob)
    sup = orc.pupil_support(prob) if prob.flags & orc.PUPIL_SUPPORT else np.ones((prob.n_lo,) * 2, bool)
    n = prob.n_lo

    fid = _fidelity_ties(psi, P, meas, prob)
    fcols = []  # (k, sign, ratio, dC (n x n), dD (n x n))
    for k, (o, items) in enumerate(fid):
        crop_k = orc.crop(psi, org[k], n)
        for comp, y, x, s, ratio in items:
            Y = orc.lowres_field_adjoint(_fid_column(o, comp, y, x, prob), prob.upsample)
            fcols.append((k, s, ratio, np.conj(Pe) * Y, np.conj(crop_k) * Y * sup))
    O, a, hitems = _hessian_ties(psi, prob)
    hcols = [(s, ratio, _hess_column(O, a, f, c, y, x, prob)) for f, c, y, x, s, ratio in hitems]

    r_psi = np.asarray(g_psi_gpu, np.complex128) - g0
    r_P = np.asarray(g_P_gpu, np.complex128) - gP0
    d_f = np.zeros(len(fcols))
    d_h = np.zeros(len(hcols))
    for _ in range(sweeps):
        # Hessian columns live in the object domain (the transform is unitary)
        r_obj = orc.object_from_spectrum(r_psi)
        for i, (s, _, col) in enumerate(hcols):
            nrm = sum(abs(v) ** 2 for _, _, v in col)
            if nrm == 0:
                continue
            for yy, xx, v in col:  # take the current decision out
                r_obj[yy, xx] += d_h[i] * v
            coef = sum((np.conj(v) * r_obj[yy, xx]).real for yy, xx, v in col) / nrm
            d_h[i] = _snap(coef, s)
            for yy, xx, v in col:
                r_obj[yy, xx] -= d_h[i] * v
        r_psi = orc.spectrum_from_object(r_obj)
        for i, (k, s, _, dC, dD) in enumerate(fcols):
            y0, x0 = org[k]
            win = r_psi[y0:y0 + n, x0:x0 + n]
            nrm = float(np.sum(np.abs(dC) ** 2) + np.sum(np.abs(dD) ** 2))
            if nrm == 0:
                continue
            win += d_f[i] * dC
            r_P += d_f[i] * dD
            coef = float(np.sum(np.conj(dC) * win).real + np.sum(np.conj(dD) * r_P).real) / nrm
            d_f[i] = _snap(coef, s)
            win -= d_f[i] * dC
            r_P -= d_f[i] * dD
    g_psi = np.asarray(g_psi_gpu, np.complex128) - r_psi
    g_P = np.asarray(g_P_gpu, np.complex128) - r_P
    flipped = [fcols[i][2] for i in np.flatnonzero(d_f)] + [hcols[i][1] for i in np.flatnonzero(d_h)]
    return Ties(len(fcols), len(hcols), int(np.count_nonzero(d_f)), int(np.count_nonzero(d_h)),
                float(max(flipped)) if flipped else 0.0, g_psi, g_P, loss4)


def step_from(pair, g_psi, g_P):
    """Algorithm 1's update of the pair's state with the given gradients, from the
    oracle's own update functions (Eq. 19, the pupil pre-filter and the support mask)."""
    prob, st = pair.oprob, pair.state
    t = st.t + 1
    psi, mu, v, d = orc.optimizer_step(st.psi, g_psi, st.mu_psi, st.v_psi, st.delta_psi, t, prob)
    out = {"psi": psi, "mu_psi": mu, "v_psi": v, "delta_psi": d, "P": st.P}
    if prob.flags & orc.LEARN_PUPIL:
        P0 = orc.gauss3(st.P) if prob.flags & orc.PUPIL_FILTER else st.P
        Pn, muP, vP, dP = orc.optimizer_step(P0, g_P, st.mu_P, st.v_P, st.delta_P, t, prob)
        if prob.flags & orc.PUPIL_SUPPORT:
            Pn = Pn * orc.pupil_support(prob)
        out.update(P=Pn, mu_P=muP, v_P=vP, delta_P=dP)
    return out


def elementwise_excess(got, want, c=KAPPA):
    """Largest ratio of |got - want| to the FP32 bound c U32 (|want| + rms(want)), per
    element: <= 1 means every element lies within the stated rounding of the reference."""
    got = np.asarray(got)
    want = np.asarray(want)
    rms = np.sqrt(np.mean(np.abs(want) ** 2))
    bound = c * U32 * (np.abs(want) + rms)
    return float(np.max(np.abs(got - want) / bound))
