"""Batches of independent fields of view (one graph replay = one iteration of every tile):
each tile's trajectory must equal that of its plan run alone, bit for bit, whatever the
branch count; tuning must leave the states untouched."""
import numpy as np
import pytest

from pairs import make_pair

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TILES = [(32, 4, 5, True, 0), (64, 4, 7, True, 1), (96, 4, 5, True, 2), (32, 4, 5, False, 3), (128, 4, 5, True, 4)]


def E():
    import paper_2209_14671_amd as E_
    return E_


def dev(x, f32):
    t = torch.from_numpy(np.ascontiguousarray(x))
    if np.iscomplexobj(x):
        return t.to(torch.complex64 if f32 else torch.complex128).cuda()
    return t.to(torch.float32 if f32 else torch.float64).cuda()


def build_tiles():
    e = E()
    out = []
    for n_lo, up, grid, f32, seed in TILES:
        pair = make_pair(n_lo, up, grid, f32=f32, seed=seed, warm_steps=0)
        plan = e.Plan(e.Problem(precision=e.F32 if f32 else e.F64, **pair.kw))
        st = plan.init_state(dev(pair.meas, f32))
        out.append((plan, st, dev(pair.meas, f32)))
    return out


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
