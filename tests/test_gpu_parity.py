"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Tolerances (relative L2 unless noted), derived from the arithmetic:
* FP64 plans: 1e-12 for every array.
* FP32 plans: per-iteration state (psi, P after one step from identical states)
  within 1e-5; fields, intensities and losses within 1e-5 (a few FP32 roundings
  through two length-n FFT passes, ~log2(n) eps); gradients within 1e-4, because
  the smoothed L1 normaliser amplifies FP32 rounding of the image differences by up
  to 1/l1_eps where |difference| < l1_eps.
The smoothed L1 mode (l1_eps > 0) is used where the comparison must be elementwise;
with l1_eps = 0 the sign of a near-zero difference may legitimately differ between
FP32 and FP64, so that mode is compared with a looser bound on the gradient.
"""
import numpy as np
import pytest

import oracle as orc
from helpers import rel_l2
from pairs import make_pair

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def E():
    import paper_2209_14671_amd as E_
    return E_


def dev(x, f32):
    t = torch.from_numpy(np.ascontiguousarray(x))
    if np.iscomplexobj(x):
        t = t.to(torch.complex64 if f32 else torch.complex128)
    else:
        t = t.to(torch.float32 if f32 else torch.float64)
    return t.cuda()


def host(t):
    return t.detach().cpu().numpy().astype(np.complex128 if t.is_complex() else np.float64)


def make_plan(pair, f32):
    e = E()
    prob = e.Problem(precision=e.F32 if f32 else e.F64, **pair.kw)
    return e.Plan(prob)


def gpu_state(plan, pair, f32):
    e = E()
    st = pair.state
    S = e.State(psi=dev(st.psi, f32), P=dev(st.P, f32), mu_psi=dev(st.mu_psi, f32),
                v_psi=torch.from_numpy(st.v_psi.copy()).cuda(), delta_psi=dev(st.delta_psi, f32),
                mu_P=dev(st.mu_P, f32), v_P=torch.from_numpy(st.v_P.copy()).cuda(), delta_P=dev(st.delta_P, f32),
                t=torch.tensor([st.t], dtype=torch.int64).cuda())
    return S


TOL = {True: dict(field=1e-5, loss=1e-5, grad=1e-4, state=1e-5), False: dict(field=1e-12, loss=1e-12, grad=1e-11,
                                                                              state=1e-12)}


def elementwise(got, want, f32, smoothed=False):
    """Largest ratio, over elements, of |got - want| to the rounding bound of the precision:
    64 units of roundoff (FP32 2^-24, FP64 2^-53) times |want| + rms(want), the scale of a
    transformed value's error.  <= 1: every element is within the bound, so an error
    confined to low-magnitude elements (the edge of the synthetic aperture) is seen.  The
    smoothed L1 (l1_eps > 0) multiplies the FP32 rounding of a feature c by up to 1 / l1_eps
    in omega = c / sqrt(c^2 + eps^2) where |c| < eps (the reason its gradients are held to
    1e-4 rather than 1e-5): its FP32 states get 16 times the bound (measured up to 2.7)."""
    import ties
    c = 64.0 if f32 else 64.0 * 2.0 ** -29
    return ties.elementwise_excess(got, want, c * (16.0 if smoothed and f32 else 1.0))

SIZES = [(32, 4, 5, False), (32, 4, 5, True), (64, 4, 7, True), (64, 2, 5, False), (128, 4, 9, True)]


@pytest.mark.parametrize("n_lo,up,grid,f32", SIZES)
def test_forward_fields_intensities_loss(n_lo, up, grid, f32):
    pair = make_pair(n_lo, up, grid, f32=f32)
    plan = make_plan(pair, f32)
    out = plan.forward(dev(pair.psi, f32), dev(pair.P, f32), dev(pair.meas, f32), fields=True, intens=True,
                       loss=True)
    torch.cuda.synchronize()
    ref_f = orc.fields(pair.psi, pair.P, pair.oprob)
    ref_l = orc.loss_and_grad(pair.psi, pair.P, pair.meas, pair.oprob, want_grad=False)[0]
    ef = rel_l2(host(out["fields"]), ref_f)
    ei = rel_l2(host(out["intens"]), np.abs(ref_f) ** 2)
    el = np.abs(host(out["loss4"]) - ref_l) / np.abs(ref_l)
    xf, xi = elementwise(host(out["fields"]), ref_f, f32), elementwise(host(out["intens"]), np.abs(ref_f) ** 2, f32)
    print(f"n_lo={n_lo} f32={f32}: fields {ef:.2e} intens {ei:.2e} loss {el} elementwise {xf:.3f} {xi:.3f}")
    tol = TOL[f32]
    assert ef < tol["field"] and ei < tol["field"]
    assert xf <= 1.0 and xi <= 1.0
    assert np.all(el < tol["loss"])


GRAD_CASES = [(f, n, f32, 0.5) for f in (orc.FID_INTENSITY, orc.FID_AMPLITUDE) for n in (orc.NORM_ANISO, orc.NORM_ISO)
              for f32 in (False, True)]
# the Sec. 6.3 scalings g(x) = x^gamma and ln(x + 1)
GRAD_CASES += [(orc.FID_GAMMA, n, f32, g) for g in (0.375, 0.875) for n in (orc.NORM_ANISO, orc.NORM_ISO)
               for f32 in (False, True)]
GRAD_CASES += [(orc.FID_LOG, n, f32, 0.5) for n in (orc.NORM_ANISO, orc.NORM_ISO) for f32 in (False, True)]


@pytest.mark.parametrize("fidelity,norm,f32,gamma", GRAD_CASES)
def test_gradients_match_oracle(fidelity, norm, f32, gamma):
    pair = make_pair(32, 4, 5, f32=f32, fidelity=fidelity, norm=norm, fid_gamma=gamma)
    plan = make_plan(pair, f32)
    l4, g, gP = plan.grad(dev(pair.psi, f32), dev(pair.P, f32), dev(pair.meas, f32))
    torch.cuda.synchronize()
    rl4, rg, rgP = orc.loss_and_grad(pair.psi, pair.P, pair.meas, pair.oprob)
    eg, egp = rel_l2(host(g), rg), rel_l2(host(gP), rgP)
    el = np.abs(host(l4) - rl4) / np.abs(rl4)
    print(f"fid={fidelity} gamma={gamma} norm={norm} f32={f32}: g_psi {eg:.2e} g_P {egp:.2e} loss {el}")
    tol = TOL[f32]
    assert eg < tol["grad"] and egp < tol["grad"]
    assert np.all(el < tol["loss"])


@pytest.mark.parametrize("fidelity,norm,f32,gamma", GRAD_CASES)
def test_step_matches_oracle(fidelity, norm, f32, gamma):
    pair = make_pair(32, 4, 5, f32=f32, fidelity=fidelity, norm=norm, fid_gamma=gamma)
    plan = make_plan(pair, f32)
    st = gpu_state(plan, pair, f32)
    l4 = plan.step(st, dev(pair.meas, f32))
    torch.cuda.synchronize()
    ref, rl4 = orc.step(pair.state, pair.meas, pair.oprob)
    res = {k: rel_l2(host(getattr(st, k)), getattr(ref, k)) for k in ("psi", "P", "mu_psi", "mu_P", "delta_psi")}
    res["v_psi"] = rel_l2(host(st.v_psi), ref.v_psi)
    xs, xp = elementwise(host(st.psi), ref.psi, f32, True), elementwise(host(st.P), ref.P, f32, True)
    print(f"fid={fidelity} gamma={gamma} norm={norm} f32={f32}: " +
          " ".join(f"{k} {v:.2e}" for k, v in res.items()) + f" elementwise {xs:.3f} {xp:.3f}")
    assert int(st.t.item()) == ref.t
    tol = TOL[f32]
    assert res["psi"] < tol["state"] and res["P"] < tol["state"]
    assert xs <= 1.0 and xp <= 1.0
    assert np.all(np.abs(host(l4) - rl4) / np.abs(rl4) < tol["loss"])


OPT_CASES = [(o, f32) for o in (orc.OPT_SGD, orc.OPT_NADAM, orc.OPT_ADABELIEF) for f32 in (False, True)]


@pytest.mark.parametrize("opt,f32", OPT_CASES)
def test_step_with_other_optimisers_matches_oracle(opt, f32):
    """The Sec. 6.2 alternatives to Eq. 19, with pupil learning and non-trivial moments."""
    pair = make_pair(32, 4, 5, f32=f32, optimizer=opt)
    plan = make_plan(pair, f32)
    st = gpu_state(plan, pair, f32)
    l4 = plan.step(st, dev(pair.meas, f32))
    torch.cuda.synchronize()
    ref, rl4 = orc.step(pair.state, pair.meas, pair.oprob)
    res = {k: rel_l2(host(getattr(st, k)), getattr(ref, k)) for k in ("psi", "P", "mu_psi", "mu_P")}
    res["v_psi"] = rel_l2(host(st.v_psi), ref.v_psi) if opt != orc.OPT_SGD else 0.0
    print(f"opt={opt} f32={f32}: " + " ".join(f"{k} {v:.2e}" for k, v in res.items()))
    tol = TOL[f32]
    assert int(st.t.item()) == ref.t
    assert res["psi"] < tol["state"] and res["P"] < tol["state"]
    if opt != orc.OPT_SGD:
        assert res["mu_psi"] < tol["grad"] and res["v_psi"] < tol["grad"]
    assert np.all(np.abs(host(l4) - rl4) / np.abs(rl4) < tol["loss"])


def test_run_with_nadam_equals_repeated_steps():
    """Bias corrections of NAdam use t and t + 1 across graph replays."""
    pair = make_pair(32, 4, 5, f32=False, optimizer=orc.OPT_NADAM)
    plan = make_plan(pair, False)
    meas = dev(pair.meas, False)
    a = gpu_state(plan, pair, False)
    b = a.clone()
    plan.run(a, meas, 9)
    for _ in range(9):
        plan.step(b, meas)
    torch.cuda.synchronize()
    for k in ("psi", "P", "mu_psi", "v_psi", "mu_P", "v_P", "t"):
        assert torch.equal(getattr(a, k), getattr(b, k)), k
    ref, _ = orc.run(pair.state, pair.meas, pair.oprob, 9)
    assert rel_l2(host(a.psi), ref.psi) < 1e-11


@pytest.mark.parametrize("fidelity,gamma", [(orc.FID_INTENSITY, 0.5), (orc.FID_AMPLITUDE, 0.5),
                                            (orc.FID_GAMMA, 0.375), (orc.FID_LOG, 0.5)])
@pytest.mark.parametrize("f32", [False, True])
def test_auto_penalty_matches_oracle(fidelity, gamma, f32):
    pair = make_pair(64, 4, 7, f32=f32, fidelity=fidelity, fid_gamma=gamma, warm_steps=0)
    plan = make_plan(pair, f32)
    a = plan.auto_penalty(dev(pair.meas, f32))
    ref = orc.auto_penalty(pair.meas, fidelity, gamma)
    print(f"auto alpha fid={fidelity} f32={f32}: {a:.6e} vs {ref:.6e}")
    assert abs(a - ref) <= 1e-12 * ref


def test_set_penalty_changes_the_loss_weights():
    """New weights reach a plan whose graphs were captured with the old ones."""
    pair = make_pair(32, 4, 5, f32=False, warm_steps=0)
    plan = make_plan(pair, False)
    meas = dev(pair.meas, False)
    st = gpu_state(plan, pair, False)
    plan.run(st, meas, 1)  # captures graphs for these pointers, old weights
    plan.set_penalty(0.05, 0.02)
    hist = plan.run(st, meas, 1)
    torch.cuda.synchronize()
    mid, _ = orc.run(pair.state, pair.meas, pair.oprob, 1)
    oprob = orc.Problem(**{**pair.oprob.__dict__, "alpha": 0.05, "beta": 0.02})
    ref, rh = orc.run(mid, pair.meas, oprob, 1)
    assert np.max(np.abs(host(hist) - rh) / np.abs(rh)) < 1e-12
    assert rel_l2(host(st.psi), ref.psi) < 1e-12


EXACT_SIGN_CASES = [(32, 4, True, orc.FID_INTENSITY), (32, 4, False, orc.FID_INTENSITY),
                    (64, 4, True, orc.FID_AMPLITUDE), (64, 4, False, orc.FID_AMPLITUDE),
                    (128, 4, True, orc.FID_INTENSITY), (256, 2, True, orc.FID_INTENSITY),
                    (256, 2, True, orc.FID_AMPLITUDE)]


@pytest.mark.parametrize("n_lo,up,f32,fidelity", EXACT_SIGN_CASES)
def test_exact_sign_mode_gradient_matches_oracle_at_its_decisions(n_lo, up, f32, fidelity):
    """l1_eps = 0 (the literal L1, anisotropic: omega = sign, Eq. 12; the kernels'
    branch-free feature loops, in the LDS tile and in the 256^2 column kernel).  Where a
    feature is within FP32 rounding of zero, FP32 and the FP64 oracle may take opposite
    signs; `ties` lists those positions from the oracle's values and a stated FP32 error
    bound and infers the library's decision at each from its gradient.  With those
    decisions the oracle gradient must match to 1e-5 (rel-L2) and every element to within
    64 FP32 roundings of |ref| + rms(ref).  FP64 takes the oracle's decisions: 1e-9 raw."""
    import ties
    pair = make_pair(n_lo, up, 5 if n_lo <= 64 else 3, f32=f32, l1_eps=0.0, fidelity=fidelity)
    plan = make_plan(pair, f32)
    l4, g, gP = plan.grad(dev(pair.psi, f32), dev(pair.P, f32), dev(pair.meas, f32))
    rl4, rg, rgP = orc.loss_and_grad(pair.psi, pair.P, pair.meas, pair.oprob)
    gh, gph = host(g), host(gP)
    assert np.all(np.abs(host(l4) - rl4) / np.abs(rl4) < (1e-5 if f32 else 1e-12))
    if not f32:
        eg, egp = rel_l2(gh, rg), rel_l2(gph, rgP)
        print(f"exact-sign n_lo={n_lo} f64 fid={fidelity}: g_psi {eg:.2e} g_P {egp:.2e}")
        assert eg < 1e-9 and egp < 1e-9
        return
    T = ties.infer(pair, gh, gph)
    raw, rawp = rel_l2(gh, rg), rel_l2(gph, rgP)
    eg, egp = rel_l2(gh, T.g_psi), rel_l2(gph, T.g_P)
    xg, xgp = ties.elementwise_excess(gh, T.g_psi), ties.elementwise_excess(gph, T.g_P)
    print(f"exact-sign n_lo={n_lo} fid={fidelity}: raw g_psi {raw:.2e} g_P {rawp:.2e}; ties fid {T.n_fid} "
          f"hess {T.n_hess}, flips fid {T.flips_fid} hess {T.flips_hess} (max |c|/bound {T.max_abs_flipped:.2f}); "
          f"at the library's decisions g_psi {eg:.2e} g_P {egp:.2e}, elementwise {xg:.2f} {xgp:.2f}")
    assert eg < 1e-5 and egp < 1e-5
    assert xg <= 1.0 and xgp <= 1.0


ISO_EXACT_CASES = [(32, 4, True, orc.FID_INTENSITY), (32, 4, False, orc.FID_AMPLITUDE),
                   (64, 4, True, orc.FID_AMPLITUDE), (128, 4, True, orc.FID_INTENSITY),
                   (256, 2, True, orc.FID_INTENSITY)]


@pytest.mark.parametrize("n_lo,up,f32,fidelity", ISO_EXACT_CASES)
def test_exact_isotropic_gradient_and_step_match_oracle(n_lo, up, f32, fidelity):
    """l1_eps = 0 with the isotropic normaliser c / |c| (Eq. 12, 0 at c = 0): continuous
    wherever a feature pair (Hessian triple) is nonzero, so compared directly; FP32 rounding
    of c is amplified by 1 / |c| where |c| is small, as in the smoothed mode (bounds 1e-4
    for the gradient, 1e-5 for the state after one step)."""
    pair = make_pair(n_lo, up, 5 if n_lo <= 64 else 3, f32=f32, l1_eps=0.0, fidelity=fidelity, norm=orc.NORM_ISO)
    plan = make_plan(pair, f32)
    l4, g, gP = plan.grad(dev(pair.psi, f32), dev(pair.P, f32), dev(pair.meas, f32))
    rl4, rg, rgP = orc.loss_and_grad(pair.psi, pair.P, pair.meas, pair.oprob)
    st = gpu_state(plan, pair, f32)
    plan.step(st, dev(pair.meas, f32))
    torch.cuda.synchronize()
    ref, _ = orc.step(pair.state, pair.meas, pair.oprob)
    eg, egp = rel_l2(host(g), rg), rel_l2(host(gP), rgP)
    es, esp = rel_l2(host(st.psi), ref.psi), rel_l2(host(st.P), ref.P)
    print(f"exact iso n_lo={n_lo} f32={f32} fid={fidelity}: g_psi {eg:.2e} g_P {egp:.2e} step psi {es:.2e} "
          f"P {esp:.2e}")
    tol = TOL[f32]
    assert eg < tol["grad"] and egp < tol["grad"]
    assert es < tol["state"] and esp < tol["state"]
    assert np.all(np.abs(host(l4) - rl4) / np.abs(rl4) < tol["loss"])


def test_transforms_match_oracle():
    for f32 in (False, True):
        pair = make_pair(64, 4, 3, f32=f32)
        plan = make_plan(pair, f32)
        O = plan.object_from_spectrum(dev(pair.psi, f32))
        ref = orc.object_from_spectrum(pair.psi)
        e1 = rel_l2(host(O), ref)
        back = plan.spectrum_from_object(dev(ref, f32))
        e2 = rel_l2(host(back), orc.spectrum_from_object(ref.astype(np.complex64).astype(complex) if f32 else ref))
        print(f"f32={f32}: object {e1:.2e} spectrum {e2:.2e}")
        tol = 1e-6 if f32 else 1e-13
        assert e1 < tol and e2 < tol


def test_run_equals_repeated_steps_bitwise_and_tracks_oracle():
    pair = make_pair(32, 4, 5, f32=False)
    plan = make_plan(pair, False)
    meas = dev(pair.meas, False)
    a = gpu_state(plan, pair, False)
    b = a.clone()
    hist = plan.run(a, meas, 11)  # one 8-iteration graph, then three 1-iteration graphs
    hs = [plan.step(b, meas) for _ in range(11)]
    torch.cuda.synchronize()
    for k in ("psi", "P", "mu_psi", "v_psi", "delta_psi", "mu_P", "v_P", "delta_P", "t"):
        assert torch.equal(getattr(a, k), getattr(b, k)), k
    assert torch.equal(hist, torch.stack(hs))
    ref, rh = orc.run(pair.state, pair.meas, pair.oprob, 11)
    e = rel_l2(host(a.psi), ref.psi)
    print(f"11 FP64 iterations: psi {e:.2e}")
    assert e < 1e-11
    assert np.max(np.abs(host(hist) - rh) / np.abs(rh)) < 1e-11


@pytest.mark.parametrize("f32", [True, False])
def test_long_segment_lists_match_oracle(f32):
    """121 LEDs 0.5 mm apart under a 0.3 NA: every window covers nearly the same pixels,
    so a 16-column segment of a spectrum row meets up to 121 LED runs (more than the 32
    that the update keeps in lanes; the rest each lane reads itself).  Gradient and
    one step against the oracle."""
    pair = make_pair(32, 4, 11, f32=f32, na=0.3, pitch_mm=0.5)
    org, sup = orc.window_origins(pair.oprob), orc.pupil_support(pair.oprob)
    count = {}
    for y0, x0 in org:
        for dy in range(pair.oprob.n_lo):
            xs = np.nonzero(sup[dy])[0]
            if len(xs):
                for g in range((x0 + xs[0]) // 16, (x0 + xs[-1]) // 16 + 1):
                    count[(y0 + dy, g)] = count.get((y0 + dy, g), 0) + 1
    assert max(count.values()) > 32
    plan = make_plan(pair, f32)
    psi, P, meas = dev(pair.psi, f32), dev(pair.P, f32), dev(pair.meas, f32)
    l4, g, gP = plan.grad(psi, P, meas)
    rl4, rg, rgP = orc.loss_and_grad(pair.psi, pair.P, pair.meas, pair.oprob)
    st = gpu_state(plan, pair, f32)
    plan.step(st, meas)
    torch.cuda.synchronize()
    ref, _ = orc.step(pair.state, pair.meas, pair.oprob)
    t = TOL[f32]
    eg, egp, es = rel_l2(host(g), rg), rel_l2(host(gP), rgP), rel_l2(host(st.psi), ref.psi)
    print(f"long lists ({'f32' if f32 else 'f64'}): g_psi {eg:.2e} g_P {egp:.2e} step {es:.2e}")
    assert eg < t["grad"] and egp < t["grad"]
    assert es < t["state"] and rel_l2(host(st.P), ref.P) < t["state"]


def test_chained_runs_equal_repeated_steps():
    """Runs of 5, 19 and 45 iterations (graphs of 32, 8 and 1 iterations that open,
    continue and close a chain: 5 x 1, 8 + 8 + 3 x 1, 32 + 8 + 5 x 1) against 69 single
    steps, bit for bit, FP32 and FP64."""
    for f32 in (True, False):
        pair = make_pair(64, 4, 7, f32=f32)
        plan = make_plan(pair, f32)
        meas = dev(pair.meas, f32)
        a = gpu_state(plan, pair, f32)
        b = a.clone()
        h = [plan.run(a, meas, n) for n in (5, 19, 45)]
        hs = [plan.step(b, meas) for _ in range(69)]
        torch.cuda.synchronize()
        for k in ("psi", "P", "mu_psi", "v_psi", "delta_psi", "mu_P", "v_P", "delta_P", "t"):
            assert torch.equal(getattr(a, k), getattr(b, k)), (f32, k)
        assert torch.equal(torch.cat(h), torch.stack(hs))


def test_init_state_matches_oracle():
    for f32 in (False, True):
        pair = make_pair(32, 4, 5, f32=f32)
        plan = make_plan(pair, f32)
        st = plan.init_state(dev(pair.meas, f32))
        ref = orc.init_state(pair.meas, pair.oprob)
        e = rel_l2(host(st.psi), ref.psi)
        assert e < (1e-6 if f32 else 1e-13), e
        assert np.array_equal(host(st.P), ref.P)
        assert int(st.t.item()) == 0
        assert np.allclose(host(st.delta_psi), pair.oprob.lr ** 2)


def _config2_pair(l1_eps, config=2):
    import synth
    case = synth.config_case(config)
    o = case.optics
    flags = orc.LEARN_PUPIL | orc.PUPIL_SUPPORT | orc.PUPIL_FILTER
    oprob = orc.problem_from_optics(o, case.led_k, flags=flags, l1_eps=l1_eps)
    sim = orc.problem_from_optics(o, case.led_k_true)
    clean = orc.intensities(orc.spectrum_from_object(case.obj), case.pupil, sim)
    meas = synth.degrade(clean, case.degradation, case.noise_seed).astype(np.float32).astype(np.float64)
    st = orc.init_state(meas, oprob)
    for _ in range(2):
        st, _ = orc.step(st, meas, oprob)
    f = lambda a: a.astype(np.complex64).astype(np.complex128)  # noqa: E731
    r = lambda a: a.astype(np.float32).astype(np.float64)  # noqa: E731
    st = orc.State(f(st.psi), f(st.P), f(st.mu_psi), st.v_psi, r(st.delta_psi), f(st.mu_P), st.v_P, r(st.delta_P),
                   st.t)
    kw = dict(n_lo=o.n_lo, upsample=o.upsample, led_k=case.led_k, wavelength_um=o.wavelength_um, na=o.na,
              dx_lo_um=o.dx_lo_um, l1_eps=l1_eps, flags=flags)
    from pairs import Pair
    return Pair(oprob, kw, st.psi, st.P, meas, st)


def test_config2_full_size_step_smoothed():
    """The benchmark workload at full size (512^2, K = 225, 128^2, FP32) with the smoothed
    L1 (l1_eps = 1e-3), one iteration through elfpie_run (its opening graph and close): the
    state after the step against the oracle, rel-L2 1e-5, and every element of psi and P
    within the smoothed mode's elementwise bound (see `elementwise`)."""
    pair = _config2_pair(1e-3)
    plan = make_plan(pair, True)
    assert (plan.K, plan.n_lo, plan.n_hi, plan.S) == (225, 128, 512, 5025)
    st = gpu_state(plan, pair, True)
    hist = plan.run(st, dev(pair.meas, True), 1)
    torch.cuda.synchronize()
    ref, rl4 = orc.step(pair.state, pair.meas, pair.oprob)
    e_psi, e_P = rel_l2(host(st.psi), ref.psi), rel_l2(host(st.P), ref.P)
    x_psi, x_P = elementwise(host(st.psi), ref.psi, True, True), elementwise(host(st.P), ref.P, True, True)
    el = np.abs(host(hist)[0] - rl4) / np.abs(rl4)
    print(f"config2 smoothed: psi {e_psi:.2e} P {e_P:.2e} elementwise {x_psi:.3f} {x_P:.3f} loss {el}")
    assert e_psi < 1e-5 and e_P < 1e-5
    assert x_psi <= 1.0 and x_P <= 1.0
    assert np.all(el < 1e-5)


def test_config2_full_size_literal_l1_at_the_librarys_decisions():
    """The benchmark's own mode (literal L1, l1_eps = 0) at full size.  The library's sign
    decisions at ties (features within FP32 rounding of zero) are inferred from its gradient
    at the state (`ties`); the oracle's gradient with those decisions must then match to
    1e-5 (rel-L2) and elementwise, and the state after one elfpie_run iteration must match
    the Eq. 19 step that the oracle's update functions take with that gradient, to 1e-5
    and elementwise.  The flip count is reported."""
    import ties
    pair = _config2_pair(0.0)
    plan = make_plan(pair, True)
    meas = dev(pair.meas, True)
    l4, g, gP = plan.grad(dev(pair.psi, True), dev(pair.P, True), meas)
    st = gpu_state(plan, pair, True)
    hist = plan.run(st, meas, 1)
    torch.cuda.synchronize()
    gh, gph = host(g), host(gP)
    T = ties.infer(pair, gh, gph)
    ref = ties.step_from(pair, T.g_psi, T.g_P)
    raw = orc.step(pair.state, pair.meas, pair.oprob)[0]
    eg, egp = rel_l2(gh, T.g_psi), rel_l2(gph, T.g_P)
    es, esp = rel_l2(host(st.psi), ref["psi"]), rel_l2(host(st.P), ref["P"])
    xs, xsp = ties.elementwise_excess(host(st.psi), ref["psi"]), ties.elementwise_excess(host(st.P), ref["P"])
    print(f"config2 literal L1: ties fid {T.n_fid} hess {T.n_hess}; flips fid {T.flips_fid} hess {T.flips_hess} "
          f"(max |c|/bound {T.max_abs_flipped:.3f}); gradient {eg:.2e} {egp:.2e} elementwise "
          f"{ties.elementwise_excess(gh, T.g_psi):.3f}; step psi {es:.2e} P {esp:.2e} elementwise {xs:.3f} {xsp:.3f}; "
          f"against the oracle's own decisions psi {rel_l2(host(st.psi), raw.psi):.2e}")
    assert eg < 1e-5 and egp < 1e-5
    assert ties.elementwise_excess(gh, T.g_psi) <= 1.0 and ties.elementwise_excess(gph, T.g_P) <= 1.0
    assert es < 1e-5 and esp < 1e-5 and xs <= 1.0 and xsp <= 1.0
    assert np.all(np.abs(host(hist)[0] - T.loss4) / np.abs(T.loss4) < 1e-5)
    assert np.all(np.abs(host(l4) - T.loss4) / np.abs(T.loss4) < 1e-5)


def test_config2_chained_run_equals_steps_and_tracks_oracle():
    """The launch sequence the benchmark times, at full size: elfpie_run(41) launches 41
    iterations directly (T1 carried over from each update launch to the next per-LED launch,
    the run's counters cleared by its opening row transforms).  In the benchmark's mode
    (literal L1) it must equal 41 elfpie_step calls bit for bit.  In the smoothed mode three chained iterations
    (graphs of 2 and 1) must match three oracle iterations to 1e-5."""
    for l1_eps in (0.0, 1e-3):
        pair = _config2_pair(l1_eps)
        plan = make_plan(pair, True)
        meas = dev(pair.meas, True)
        a = gpu_state(plan, pair, True)
        if l1_eps == 0.0:
            b = a.clone()
            h = plan.run(a, meas, 41)
            hs = [plan.step(b, meas) for _ in range(41)]
            torch.cuda.synchronize()
            for k in ("psi", "P", "mu_psi", "v_psi", "delta_psi", "mu_P", "v_P", "delta_P", "t"):
                assert torch.equal(getattr(a, k), getattr(b, k)), k
            assert torch.equal(h, torch.stack(hs))
            assert int(a.t.item()) == pair.state.t + 41
        else:
            h = plan.run(a, meas, 3)
            torch.cuda.synchronize()
            ref, rh = orc.run(pair.state, pair.meas, pair.oprob, 3)
            e_psi, e_P = rel_l2(host(a.psi), ref.psi), rel_l2(host(a.P), ref.P)
            eh = np.max(np.abs(host(h) - rh) / np.abs(rh))
            print(f"config2 smoothed, 3 chained iterations: psi {e_psi:.2e} P {e_P:.2e} loss {eh:.2e}")
            assert e_psi < 1e-5 and e_P < 1e-5 and eh < 1e-5


def test_run_with_a_kept_history_buffer_only_replays():
    """Repeated runs with the same state, stack and history buffer capture their graphs once."""
    pair = make_pair(32, 4, 5, f32=True)
    plan = make_plan(pair, True)
    meas = dev(pair.meas, True)
    st = gpu_state(plan, pair, True)
    hist = torch.empty((20, 4), dtype=torch.float64, device="cuda")
    plan.run(st, meas, 5, history=hist)
    c0 = plan.stats()["captures"]
    plan.run(st, meas, 20, history=hist)
    plan.run(st, meas, 7, history=hist)
    torch.cuda.synchronize()
    assert plan.stats()["captures"] == c0 > 0
    assert torch.isfinite(hist).all()


def test_checked_run_reports_nonfinite_loss():
    """checked = 1: a NaN in the measured stack makes the loss NaN; the run returns
    ELFPIE_E_NONFINITE after synchronising, and a clean stack returns OK."""
    e = E()
    pair = make_pair(32, 4, 5, f32=True)
    plan = make_plan(pair, True)
    st = gpu_state(plan, pair, True)
    meas = dev(pair.meas, True)
    plan.run(st, meas, 3, checked=True)
    bad = meas.clone()
    bad[2, 5, 7] = float("nan")
    st2 = gpu_state(plan, pair, True)
    with pytest.raises(e.ElfpieError) as ei:
        plan.run(st2, bad, 3, checked=True)
    assert ei.value.status == 6  # ELFPIE_E_NONFINITE
    plan.run(st, meas, 2, checked=True)  # the flag is cleared by the next run


def test_checked_run_of_the_fused_plan():
    """The same at the benchmark's size, where elfpie_run launches directly and its opening
    row transforms clear the counters: a NaN in one image gives ELFPIE_E_NONFINITE, the next
    clean run returns OK, and its history starts at row 0."""
    e = E()
    pair = _config2_pair(0.0)
    plan = make_plan(pair, True)
    assert plan.stats()["captures"] == 0
    meas = dev(pair.meas, True)
    bad = meas.clone()
    bad[100, 64, 64] = float("nan")
    st = gpu_state(plan, pair, True)
    with pytest.raises(e.ElfpieError) as ei:
        plan.run(st, bad, 2, checked=True)
    assert ei.value.status == 6  # ELFPIE_E_NONFINITE
    st = gpu_state(plan, pair, True)
    h = plan.run(st, meas, 3, checked=True)
    torch.cuda.synchronize()
    assert torch.isfinite(h).all()
    ref = plan.run(gpu_state(plan, pair, True), meas, 3)
    torch.cuda.synchronize()
    assert torch.equal(h, ref)
    assert plan.stats()["captures"] == 0  # direct launches: nothing captured


@pytest.mark.parametrize("n_lo,up", [(64, 8), (32, 16)])
def test_fp64_large_spectrum_matches_oracle(n_lo, up):
    """FP64 plans with n_hi above 256 take the tile-form object branch (line transforms,
    k_hessian on 16 x 16 tiles, tile-form update): gradient and one step against the
    oracle to 1e-12, and a 5-iteration run equal to 5 steps bit for bit."""
    pair = make_pair(n_lo, up, 3, f32=False)
    plan = make_plan(pair, False)
    assert plan.n_hi == n_lo * up > 256
    psi, P, meas = dev(pair.psi, False), dev(pair.P, False), dev(pair.meas, False)
    l4, g, gP = plan.grad(psi, P, meas)
    rl4, rg, rgP = orc.loss_and_grad(pair.psi, pair.P, pair.meas, pair.oprob)
    a = gpu_state(plan, pair, False)
    b = a.clone()
    plan.step(a, meas)
    torch.cuda.synchronize()
    ref, _ = orc.step(pair.state, pair.meas, pair.oprob)
    eg, egp, es = rel_l2(host(g), rg), rel_l2(host(gP), rgP), rel_l2(host(a.psi), ref.psi)
    print(f"f64 n_hi={plan.n_hi}: g_psi {eg:.2e} g_P {egp:.2e} step {es:.2e}")
    assert eg < 1e-11 and egp < 1e-11 and es < 1e-12 and rel_l2(host(a.P), ref.P) < 1e-12
    assert np.all(np.abs(host(l4) - rl4) / np.abs(rl4) < 1e-12)
    c = b.clone()
    plan.run(b, meas, 5)
    for _ in range(5):
        plan.step(c, meas)
    torch.cuda.synchronize()
    for k in ("psi", "P", "mu_psi", "v_psi", "t"):
        assert torch.equal(getattr(b, k), getattr(c, k)), k


# --- multiplexed illumination (Eq. 1 with M LEDs per image) ---

MUX_CASES = [(2, orc.FID_INTENSITY, orc.NORM_ANISO, 0.5, True), (3, orc.FID_AMPLITUDE, orc.NORM_ISO, 0.5, True),
             (2, orc.FID_GAMMA, orc.NORM_ANISO, 0.375, False), (3, orc.FID_INTENSITY, orc.NORM_ISO, 0.5, False),
             (2, orc.FID_LOG, orc.NORM_ANISO, 0.5, True)]


@pytest.mark.parametrize("mux,fidelity,norm,gamma,f32", MUX_CASES)
def test_multiplexed_forward_and_step_match_oracle(mux, fidelity, norm, gamma, f32):
    pair = make_pair(32, 4, 5, f32=f32, fidelity=fidelity, norm=norm, fid_gamma=gamma, mux=mux)
    plan = make_plan(pair, f32)
    assert plan.n_img == pair.oprob.K and plan.K == pair.oprob.n_led
    psi, P, meas = dev(pair.psi, f32), dev(pair.P, f32), dev(pair.meas, f32)
    out = plan.forward(psi, P, meas, fields=True, intens=True, loss=True)
    rl4, rg, rgP = orc.loss_and_grad(pair.psi, pair.P, pair.meas, pair.oprob)
    tol = TOL[f32]
    assert rel_l2(host(out["fields"]), orc.fields(pair.psi, pair.P, pair.oprob)) < tol["field"]
    assert rel_l2(host(out["intens"]), orc.intensities(pair.psi, pair.P, pair.oprob)) < tol["field"]
    assert np.all(np.abs(host(out["loss4"]) - rl4) / np.abs(rl4) < tol["loss"])
    l4, g, gP = plan.grad(psi, P, meas)
    eg, egp = rel_l2(host(g), rg), rel_l2(host(gP), rgP)
    _, g2, gP2 = plan.grad(psi, P, meas, fields=out["fields"])
    st = gpu_state(plan, pair, f32)
    plan.step(st, meas)
    torch.cuda.synchronize()
    ref, _ = orc.step(pair.state, pair.meas, pair.oprob)
    es = rel_l2(host(st.psi), ref.psi)
    print(f"mux={mux} fid={fidelity} f32={f32}: g_psi {eg:.2e} g_P {egp:.2e} step psi {es:.2e}")
    assert eg < tol["grad"] and egp < tol["grad"]
    assert torch.equal(g, g2) and torch.equal(gP, gP2)  # stored fields give the same bits
    assert es < tol["state"] and rel_l2(host(st.P), ref.P) < tol["state"]


def test_multiplexed_run_equals_repeated_steps():
    pair = make_pair(32, 4, 5, f32=False, mux=2)
    plan = make_plan(pair, False)
    meas = dev(pair.meas, False)
    a = gpu_state(plan, pair, False)
    b = a.clone()
    plan.run(a, meas, 9)
    for _ in range(9):
        plan.step(b, meas)
    torch.cuda.synchronize()
    for k in ("psi", "P", "mu_psi", "v_psi", "t"):
        assert torch.equal(getattr(a, k), getattr(b, k)), k
    ref, _ = orc.run(pair.state, pair.meas, pair.oprob, 9)
    assert rel_l2(host(a.psi), ref.psi) < 1e-11


def test_multiplexed_full_tile_gradient_matches_oracle():
    """The 128^2 tile of the multiplexed kernel (FP32, two LEDs per image)."""
    pair = make_pair(128, 4, 5, f32=True, mux=2, warm_steps=0)
    plan = make_plan(pair, True)
    l4, g, gP = plan.grad(dev(pair.psi, True), dev(pair.P, True), dev(pair.meas, True))
    torch.cuda.synchronize()
    rl4, rg, rgP = orc.loss_and_grad(pair.psi, pair.P, pair.meas, pair.oprob)
    eg, egp = rel_l2(host(g), rg), rel_l2(host(gP), rgP)
    print(f"mux=2 n_lo=128: g_psi {eg:.2e} g_P {egp:.2e}")
    assert eg < TOL[True]["grad"] and egp < TOL[True]["grad"]
    assert np.all(np.abs(host(l4) - rl4) / np.abs(rl4) < TOL[True]["loss"])



# --- the 256^2 tile (per-LED branch through HBM scratch) ---

BIG_CASES = [(2, orc.FID_INTENSITY, orc.NORM_ANISO, 0.5), (4, orc.FID_AMPLITUDE, orc.NORM_ISO, 0.5),
             (2, orc.FID_GAMMA, orc.NORM_ANISO, 0.375)]


@pytest.mark.parametrize("up,fidelity,norm,gamma", BIG_CASES)
def test_large_tile_matches_oracle(up, fidelity, norm, gamma):
    """n_lo = 256 (FP32): forward fields, images and loss, gradients, stored fields, one step."""
    pair = make_pair(256, up, 3, f32=True, fidelity=fidelity, norm=norm, fid_gamma=gamma)
    plan = make_plan(pair, True)
    psi, P, meas = dev(pair.psi, True), dev(pair.P, True), dev(pair.meas, True)
    out = plan.forward(psi, P, meas, fields=True, intens=True, loss=True)
    rl4, rg, rgP = orc.loss_and_grad(pair.psi, pair.P, pair.meas, pair.oprob)
    ef = rel_l2(host(out["fields"]), orc.fields(pair.psi, pair.P, pair.oprob))
    ei = rel_l2(host(out["intens"]), orc.intensities(pair.psi, pair.P, pair.oprob))
    el = np.abs(host(out["loss4"]) - rl4) / np.abs(rl4)
    l4, g, gP = plan.grad(psi, P, meas)
    eg, egp = rel_l2(host(g), rg), rel_l2(host(gP), rgP)
    _, g2, gP2 = plan.grad(psi, P, meas, fields=out["fields"])
    st = gpu_state(plan, pair, True)
    plan.step(st, meas)
    torch.cuda.synchronize()
    ref, _ = orc.step(pair.state, pair.meas, pair.oprob)
    es = rel_l2(host(st.psi), ref.psi)
    print(f"n_lo=256 up={up} fid={fidelity}: fields {ef:.2e} intens {ei:.2e} g_psi {eg:.2e} g_P {egp:.2e} "
          f"step {es:.2e}")
    assert ef < 1e-5 and ei < 1e-5 and np.all(el < 1e-5)
    assert eg < 1e-4 and egp < 1e-4
    assert torch.equal(g, g2) and torch.equal(gP, gP2)
    assert es < 1e-5 and rel_l2(host(st.P), ref.P) < 1e-5


def test_large_tile_init_state_matches_oracle():
    pair = make_pair(256, 4, 3, f32=True, warm_steps=0)
    plan = make_plan(pair, True)
    st = plan.init_state(dev(pair.meas, True))
    ref = orc.init_state(pair.meas, pair.oprob)
    assert rel_l2(host(st.psi), ref.psi) < 1e-6
    assert np.array_equal(host(st.P), ref.P)


def test_config5_full_size_step():
    """1024^2 high-res, K = 225, 256^2 low-res, FP32, noise-free with LED jitter: one step
    from an identical state, every element."""
    pair = _config2_pair(1e-3, config=5)
    plan = make_plan(pair, True)
    assert (plan.K, plan.n_lo, plan.n_hi) == (225, 256, 1024)
    st = gpu_state(plan, pair, True)
    hist = plan.run(st, dev(pair.meas, True), 1)
    torch.cuda.synchronize()
    ref, rl4 = orc.step(pair.state, pair.meas, pair.oprob)
    e_psi, e_P = rel_l2(host(st.psi), ref.psi), rel_l2(host(st.P), ref.P)
    el = np.abs(host(hist)[0] - rl4) / np.abs(rl4)
    print(f"config5: psi {e_psi:.2e} P {e_P:.2e} loss {el}")
    assert e_psi < 1e-5 and e_P < 1e-5
    assert np.all(el < 1e-5)


def test_large_tile_forward_without_measurements():
    """The forward model alone (no stack given) at n_lo = 256: images and fields only.
    Regression: the column kernel once read the stack in this mode."""
    pair = make_pair(256, 2, 3, f32=True, warm_steps=0)
    plan = make_plan(pair, True)
    out = plan.forward(dev(pair.psi, True), dev(pair.P, True), fields=True, intens=True)
    torch.cuda.synchronize()
    assert rel_l2(host(out["intens"]), orc.intensities(pair.psi, pair.P, pair.oprob)) < 1e-5
    assert rel_l2(host(out["fields"]), orc.fields(pair.psi, pair.P, pair.oprob)) < 1e-5


# --- sizes with a factor 3 (radix-3 / 6 / 12 passes): 96 and 192 low-res, 384 and 768 high-res ---

@pytest.mark.parametrize("n_lo,up,grid", [(96, 4, 5), (192, 2, 3), (192, 4, 3)])
def test_radix3_sizes_match_oracle(n_lo, up, grid):
    pair = make_pair(n_lo, up, grid, f32=True)
    plan = make_plan(pair, True)
    assert (plan.n_lo, plan.n_hi) == (n_lo, n_lo * up)
    psi, P, meas = dev(pair.psi, True), dev(pair.P, True), dev(pair.meas, True)
    out = plan.forward(psi, P, meas, fields=True, intens=True, loss=True)
    rl4, rg, rgP = orc.loss_and_grad(pair.psi, pair.P, pair.meas, pair.oprob)
    ef = rel_l2(host(out["fields"]), orc.fields(pair.psi, pair.P, pair.oprob))
    el = np.abs(host(out["loss4"]) - rl4) / np.abs(rl4)
    l4, g, gP = plan.grad(psi, P, meas)
    eg, egp = rel_l2(host(g), rg), rel_l2(host(gP), rgP)
    st = gpu_state(plan, pair, True)
    plan.step(st, meas)
    init = plan.init_state(meas)
    torch.cuda.synchronize()
    ref, _ = orc.step(pair.state, pair.meas, pair.oprob)
    es = rel_l2(host(st.psi), ref.psi)
    ei = rel_l2(host(init.psi), orc.init_state(pair.meas, pair.oprob).psi)
    print(f"n_lo={n_lo} n_hi={n_lo * up}: fields {ef:.2e} g_psi {eg:.2e} g_P {egp:.2e} step {es:.2e} init {ei:.2e}")
    assert ef < 1e-5 and np.all(el < 1e-5)
    assert eg < 1e-4 and egp < 1e-4
    assert es < 1e-5 and rel_l2(host(st.P), ref.P) < 1e-5
    assert ei < 1e-6


# --- the split-precision matrix-core form of the 256^2 row transforms ---

MFMA_TOL = dict(field=2e-5, grad=5e-4, state=1e-5)


@pytest.mark.parametrize("up,fidelity,norm", [(2, orc.FID_INTENSITY, orc.NORM_ANISO),
                                              (4, orc.FID_AMPLITUDE, orc.NORM_ISO)])
def test_mfma_rows_match_oracle(up, fidelity, norm):
    """ELFPIE_F32_MFMA_BF16X3 at n_lo = 256 (smoothed L1): the row transforms as DFT-matrix
    products on the matrix cores with BF16 hi + lo operands, three products accumulated in
    FP32, about 2^-16 relative error per product (FP32: 2^-24).  Stated bounds, from that
    error through two transform stages (fields ~4e-6 measured): fields and images 2e-5;
    gradients 5e-4 (the smoothed normaliser amplifies the fields' error as in FP32, whose
    gradients are held to 1e-4); the state after one step 1e-5; loss 1e-5.  Stored fields
    give the gradients bit for bit."""
    e = E()
    pair = make_pair(256, up, 3, f32=True, fidelity=fidelity, norm=norm)
    plan = e.Plan(e.Problem(precision=e.F32_MFMA_BF16X3, **pair.kw))
    psi, P, meas = dev(pair.psi, True), dev(pair.P, True), dev(pair.meas, True)
    out = plan.forward(psi, P, meas, fields=True, intens=True, loss=True)
    l4, g, gP = plan.grad(psi, P, meas)
    _, g2, gP2 = plan.grad(psi, P, meas, fields=out["fields"])
    st = gpu_state(plan, pair, True)
    plan.step(st, meas)
    torch.cuda.synchronize()
    rl4, rg, rgP = orc.loss_and_grad(pair.psi, pair.P, pair.meas, pair.oprob)
    ref, _ = orc.step(pair.state, pair.meas, pair.oprob)
    ef = rel_l2(host(out["fields"]), orc.fields(pair.psi, pair.P, pair.oprob))
    ei = rel_l2(host(out["intens"]), orc.intensities(pair.psi, pair.P, pair.oprob))
    eg, egp = rel_l2(host(g), rg), rel_l2(host(gP), rgP)
    es, esp = rel_l2(host(st.psi), ref.psi), rel_l2(host(st.P), ref.P)
    el = np.max(np.abs(host(l4) - rl4) / np.abs(rl4))
    print(f"mfma n_lo=256 up={up} fid={fidelity} norm={norm}: fields {ef:.2e} intens {ei:.2e} g_psi {eg:.2e} "
          f"g_P {egp:.2e} step psi {es:.2e} P {esp:.2e} loss {el:.2e}")
    assert ef < MFMA_TOL["field"] and ei < MFMA_TOL["field"]
    assert eg < MFMA_TOL["grad"] and egp < MFMA_TOL["grad"]
    assert es < MFMA_TOL["state"] and esp < MFMA_TOL["state"] and el < 1e-5
    assert torch.equal(g, g2) and torch.equal(gP, gP2)


def test_mfma_run_equals_steps_and_full_size_step():
    """The matrix-core form is deterministic (a 9-iteration run equals 9 steps bit for bit)
    and, at 1024^2 / K = 225 / 256^2 (smoothed L1), one step matches the oracle within the
    form's bound."""
    e = E()
    pair = make_pair(256, 2, 3, f32=True)
    plan = e.Plan(e.Problem(precision=e.F32_MFMA_BF16X3, **pair.kw))
    meas = dev(pair.meas, True)
    a = gpu_state(plan, pair, True)
    b = a.clone()
    plan.run(a, meas, 9)
    for _ in range(9):
        plan.step(b, meas)
    torch.cuda.synchronize()
    for k in ("psi", "P", "mu_psi", "v_psi", "delta_psi", "t"):
        assert torch.equal(getattr(a, k), getattr(b, k)), k
    pair = _config2_pair(1e-3, config=5)
    kw = dict(pair.kw)
    plan = e.Plan(e.Problem(precision=e.F32_MFMA_BF16X3, **kw))
    assert (plan.K, plan.n_lo, plan.n_hi) == (225, 256, 1024)
    st = gpu_state(plan, pair, True)
    hist = plan.run(st, dev(pair.meas, True), 1)
    torch.cuda.synchronize()
    ref, rl4 = orc.step(pair.state, pair.meas, pair.oprob)
    e_psi, e_P = rel_l2(host(st.psi), ref.psi), rel_l2(host(st.P), ref.P)
    el = np.max(np.abs(host(hist)[0] - rl4) / np.abs(rl4))
    print(f"mfma config5 step: psi {e_psi:.2e} P {e_P:.2e} loss {el:.2e}")
    assert e_psi < MFMA_TOL["state"] and e_P < MFMA_TOL["state"] and el < 1e-5
