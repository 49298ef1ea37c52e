"""elfpie_grad_noalloc (no plan, no device workspace: the library's static scratch) against
elfpie_grad on a plan with its own workspace, through the C ABI: two calls in a row, the
second with a smaller problem (the scratch keeps the first call's contents), each equal
to elfpie_grad bit for bit and to the FP64 oracle within the gradient bounds."""
import numpy as np
import pytest

import oracle as orc
from helpers import rel_l2
from pairs import make_pair

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev(x, f32):
    t = torch.from_numpy(np.ascontiguousarray(x))
    if np.iscomplexobj(x):
        return t.to(torch.complex64 if f32 else torch.complex128).cuda()
    return t.to(torch.float32 if f32 else torch.float64).cuda()


def test_grad_noalloc_equals_grad_on_two_calls():
    import paper_2209_14671_amd as E
    cases = [(128, 4, 9, True), (32, 4, 3, False)]  # the second call is the smaller problem
    for n_lo, up, grid, f32 in cases:
        pair = make_pair(n_lo, up, grid, f32=f32)
        prob = E.Problem(precision=E.F32 if f32 else E.F64, **pair.kw)
        assert E.workspace_bytes(prob) <= 32 << 20
        psi, P, meas = dev(pair.psi, f32), dev(pair.P, f32), dev(pair.meas, f32)
        l4, g, gP = E.grad_noalloc(prob, psi, P, meas)
        torch.cuda.synchronize()
        plan = E.Plan(prob)
        rl4, rg, rgP = plan.grad(psi, P, meas)
        torch.cuda.synchronize()
        print(f"noalloc n_lo={n_lo} K={plan.K} f32={f32}: bitwise "
              f"{torch.equal(g, rg) and torch.equal(gP, rgP) and torch.equal(l4, rl4)}")
        assert torch.equal(g, rg) and torch.equal(gP, rgP) and torch.equal(l4, rl4)
        ol4, og, ogP = orc.loss_and_grad(pair.psi, pair.P, pair.meas, pair.oprob)
        tol = 1e-4 if f32 else 1e-11
        cg = np.complex128
        assert rel_l2(g.cpu().numpy().astype(cg), og) < tol and rel_l2(gP.cpu().numpy().astype(cg), ogP) < tol
        assert np.all(np.abs(l4.cpu().numpy() - ol4) / np.abs(ol4) < (1e-5 if f32 else 1e-12))
        plan.close()
