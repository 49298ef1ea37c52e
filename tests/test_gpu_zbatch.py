"""Batches of independent fields of view (one graph replay = one iteration of every tile):
each tile's trajectory must equal that of its plan run alone, bit for bit, whatever the
branch count, and the oracle's to the usual bounds; tuning must leave the states untouched.
The tiles span every per-LED route: the LDS tile (32-128, FP32 and FP64) and the 192^2 and
256^2 tiles through HBM scratch."""
import numpy as np
import pytest

import oracle as orc
import synth
from helpers import rel_l2
from pairs import Pair, make_pair

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TILES = [(32, 4, 5, True, 0), (64, 4, 7, True, 1), (96, 4, 5, True, 2), (32, 4, 5, False, 3), (128, 4, 5, True, 4),
         (192, 2, 3, True, 5), (256, 2, 3, True, 6)]


def E():
    import paper_2209_14671_amd as E_
    return E_


def dev(x, f32):
    t = torch.from_numpy(np.ascontiguousarray(x))
    if np.iscomplexobj(x):
        return t.to(torch.complex64 if f32 else torch.complex128).cuda()
    return t.to(torch.float32 if f32 else torch.float64).cuda()


def build_tiles(with_pairs=False):
    """Tiles from the library's initial state, or (with_pairs) from the pairs' oracle
    states, so that the oracle can follow them."""
    e = E()
    out, pairs = [], []
    for n_lo, up, grid, f32, seed in TILES:
        pair = make_pair(n_lo, up, grid, f32=f32, seed=seed, warm_steps=1 if with_pairs else 0)
        plan = e.Plan(e.Problem(precision=e.F32 if f32 else e.F64, **pair.kw))
        if with_pairs:
            s = pair.state
            st = e.State(psi=dev(s.psi, f32), P=dev(s.P, f32), mu_psi=dev(s.mu_psi, f32),
                         v_psi=torch.from_numpy(s.v_psi.copy()).cuda(), delta_psi=dev(s.delta_psi, f32),
                         mu_P=dev(s.mu_P, f32), v_P=torch.from_numpy(s.v_P.copy()).cuda(),
                         delta_P=dev(s.delta_P, f32), t=torch.tensor([s.t], dtype=torch.int64).cuda())
        else:
            st = plan.init_state(dev(pair.meas, f32))
        out.append((plan, st, dev(pair.meas, f32)))
        pairs.append(pair)
    return (out, pairs) if with_pairs else out


def test_batch_tiles_match_the_oracle():
    """Two batched iterations of every tile against two oracle iterations from the same
    state: psi and P within 1e-5 (FP32) or 1e-12 (FP64), loss history likewise."""
    e = E()
    tiles, pairs = build_tiles(with_pairs=True)
    batch = e.Batch(tiles, n_branches=4)
    hist = batch.run(2)
    torch.cuda.synchronize()
    for (plan, st, _), pair, h, (n_lo, _, _, f32, _) in zip(tiles, pairs, hist, TILES):
        ref, rh = orc.run(pair.state, pair.meas, pair.oprob, 2)
        tol = 1e-5 if f32 else 1e-12
        ep = rel_l2(st.psi.cpu().numpy().astype(np.complex128), ref.psi)
        eP = rel_l2(st.P.cpu().numpy().astype(np.complex128), ref.P)
        eh = np.max(np.abs(h.cpu().numpy() - rh) / np.abs(rh))
        print(f"batch tile n_lo={n_lo} f32={f32}: psi {ep:.2e} P {eP:.2e} loss {eh:.2e}")
        assert ep < tol and eP < tol and eh < tol
        assert int(st.t.item()) == pair.state.t + 2
    batch.close()


def test_batch_follows_penalty_changes():
    """A plan's new Eq. 8 weights reach the replays of a batch captured before the change:
    batch.run(1), set_penalty, batch.run(1) equals the same on the plan alone, bit for bit."""
    e = E()
    tiles = build_tiles()[:3]
    alone = [(p, st.clone(), m) for p, st, m in tiles]
    batch = e.Batch(tiles, n_branches=2)
    batch.run(1, history=False)  # no history: the same (null) pointers on both calls
    torch.cuda.synchronize()
    for p, st, m in alone:
        p.run(st, m, 1)
    torch.cuda.synchronize()
    tiles[1][0].set_penalty(0.05, 0.02)
    batch.run(1, history=False)
    torch.cuda.synchronize()
    for p, st, m in alone:
        p.run(st, m, 1)
    torch.cuda.synchronize()
    for (p, sb, _), (_, sa, _) in zip(tiles, alone):
        assert torch.equal(sb.psi, sa.psi) and torch.equal(sb.P, sa.P), p.n_lo
    batch.close()


@pytest.mark.parametrize("branches", [1, 3, 8])
def test_batch_equals_tiles_run_alone(branches):
    e = E()
    tiles = build_tiles()
    alone = [(p, st.clone(), m) for p, st, m in tiles]
    batch = e.Batch([(p, st, m) for p, st, m in tiles], n_branches=branches)
    hb = batch.run(6)
    ha = [p.run(st, m, 6) for p, st, m in alone]
    torch.cuda.synchronize()
    for (p, sb, _), (_, sa, _), xb, xa in zip(tiles, alone, hb, ha):
        for k in ("psi", "P", "mu_psi", "v_psi", "delta_psi", "mu_P", "t"):
            assert torch.equal(getattr(sb, k), getattr(sa, k)), (p.n_lo, k)
        assert torch.equal(xb, xa)
    batch.close()


@pytest.mark.skip(reason="elfpie_batch_tune is switched off: one GPU run of this test ended in a host abort "
                         "(no device fault reported) whose cause reading the code has not found")
def test_batch_tuning_keeps_states_and_picks_a_count():
    e = E()
    tiles = build_tiles()
    before = [st.clone() for _, st, _ in tiles]
    batch = e.Batch(tiles, n_branches=2)
    ms = batch.tune(3)
    torch.cuda.synchronize()
    print("batch tuning (ms per replay by branch count):", ms)
    assert set(ms) <= {1, 2, 4, 8} and batch.n_branches in ms
    for (_, st, _), b in zip(tiles, before):
        assert torch.equal(st.psi, b.psi) and torch.equal(st.P, b.P) and torch.equal(st.t, b.t)
    h = batch.run(2)
    torch.cuda.synchronize()
    assert all(torch.isfinite(x).all() for x in h)
    batch.close()


def test_sweep_stacks_in_one_batch_match_the_oracle():
    """The robustness sweep's inputs (Eq. 20 with Table 1's second level of Gaussian,
    salt-and-pepper and Poisson noise, c = 0.25 and 0.75, LEDs shifted 0.5 mm) in one batch,
    literal L1 as the sweep runs it, from the oracle's state two iterations in: the next batched
    iteration of every tile against the oracle's step at the library's sign decisions
    (rel-L2 1e-5 and elementwise), then three more batched iterations equal to the same
    tile run alone, bit for bit."""
    import ties
    from paper_2209_14671_amd import metrics
    e = E()
    optics = synth.Optics(n_lo=32, upsample=4, led_grid=9)
    base = synth.make_case(optics, [8, 0], jitter_mm=0.5)
    sim = orc.problem_from_optics(optics, base.led_k_true, flags=orc.PUPIL_SUPPORT)
    clean = orc.intensities(orc.spectrum_from_object(base.obj), base.pupil, sim)
    dark = metrics.dark_field(base.led_k_true, optics.n_lo, optics.dx_lo_um, optics.wavelength_um, optics.na)
    flags = orc.LEARN_PUPIL | orc.PUPIL_SUPPORT | orc.PUPIL_FILTER
    oprob = orc.problem_from_optics(optics, base.led_k, flags=flags)
    kw = dict(n_lo=optics.n_lo, upsample=optics.upsample, led_k=base.led_k, wavelength_um=optics.wavelength_um,
              na=optics.na, dx_lo_um=optics.dx_lo_um, flags=flags)
    f = lambda a: a.astype(np.complex64).astype(np.complex128)  # noqa: E731
    tiles, pairs = [], []
    for ci, c in enumerate((0.25, 0.75)):
        for ni, noise in enumerate(("gaussian", "snp", "poisson")):
            noisy = synth.degrade(clean, synth.sweep_degradation(noise, 1, c), np.random.SeedSequence([8, ci, ni]),
                                  dark=dark)
            meas = noisy.astype(np.float32).astype(np.float64)
            s0 = orc.init_state(meas, oprob)
            for _ in range(2):  # off the initial state, whose object is real (all phase features tie)
                s0, _ = orc.step(s0, meas, oprob)
            r = lambda a: a.astype(np.float32).astype(np.float64)  # noqa: E731
            s0 = orc.State(f(s0.psi), f(s0.P), f(s0.mu_psi), s0.v_psi, r(s0.delta_psi), f(s0.mu_P), s0.v_P,
                           r(s0.delta_P), s0.t)
            pair = Pair(oprob, kw, s0.psi, s0.P, meas, s0)
            plan = e.Plan(e.Problem(precision=e.F32, **kw))
            st = e.State(psi=dev(s0.psi, True), P=dev(s0.P, True), mu_psi=dev(s0.mu_psi, True),
                         v_psi=torch.from_numpy(s0.v_psi.copy()).cuda(), delta_psi=dev(s0.delta_psi, True),
                         mu_P=dev(s0.mu_P, True), v_P=torch.from_numpy(s0.v_P.copy()).cuda(),
                         delta_P=dev(s0.delta_P, True), t=torch.tensor([s0.t], dtype=torch.int64).cuda())
            tiles.append((plan, st, dev(meas, True)))
            pairs.append((pair, noise, c))
    grads = []
    for (plan, _, m), (pair, _, _) in zip(tiles, pairs):
        _, g, gP = plan.grad(dev(pair.psi, True), dev(pair.P, True), m)
        grads.append((g.cpu().numpy().astype(np.complex128), gP.cpu().numpy().astype(np.complex128)))
    batch = e.Batch(tiles, n_branches=3)
    batch.run(1, history=False)
    torch.cuda.synchronize()
    for (plan, st, _), (pair, noise, c), (gh, gph) in zip(tiles, pairs, grads):
        T = ties.infer(pair, gh, gph)
        ref = ties.step_from(pair, T.g_psi, T.g_P)
        got, gotP = st.psi.cpu().numpy().astype(np.complex128), st.P.cpu().numpy().astype(np.complex128)
        es, esp = rel_l2(got, ref["psi"]), rel_l2(gotP, ref["P"])
        xs, xsp = ties.elementwise_excess(got, ref["psi"]), ties.elementwise_excess(gotP, ref["P"])
        print(f"sweep tile {noise} c={c}: ties {T.n_fid}/{T.n_hess}, flips {T.flips_fid}/{T.flips_hess}; "
              f"step psi {es:.2e} P {esp:.2e} elementwise {xs:.3f} {xsp:.3f}")
        assert es < 1e-5 and esp < 1e-5 and xs <= 1.0 and xsp <= 1.0
    alone = [(p, st.clone(), m) for p, st, m in tiles]
    batch.run(3, history=False)
    for p, st, m in alone:
        p.run(st, m, 3, history=False)
    torch.cuda.synchronize()
    for (p, sb, _), (_, sa, _) in zip(tiles, alone):
        assert torch.equal(sb.psi, sa.psi) and torch.equal(sb.P, sa.P)
    batch.close()
