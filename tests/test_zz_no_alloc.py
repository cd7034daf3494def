"""The smoothed gradient without a caller workspace (bddmp_solver_smooth_grad_noalloc) against the
same run with one (bddmp_solver_smooth_run + bddmp_solver_smooth_grad): the same kernels in the same
order, so the gradient, the bound history and the final multipliers are bitwise equal. Two calls in
a row share the library's static scratch; the second has a smaller input and must not see the
first one's contents."""
import numpy as np
import pytest

from oracle import Oracle
from paper_2009_00481_amd import binding as B
from paper_2009_00481_amd import instances as I

pytestmark = pytest.mark.gpu


def _with_workspace(ilp, alpha, T):
    import torch

    plan = B.Plan(B.Problem.from_ilp(ilp), hist_cap=max(64, T + 4))
    s = B.Solver(plan)
    nb = B.bddmp_smooth_workspace_bytes(plan.h, T)
    ws = torch.empty(max(nb, 256), dtype=torch.uint8, device="cuda")
    g = torch.empty(max(ilp.n, 1), dtype=torch.float32, device="cuda")
    B.bddmp_solver_smooth_run(s.h, alpha, T, ws, nb)
    B.bddmp_solver_smooth_grad(s.h, alpha, T, ws, nb, 1.0, g)
    out = (g[:ilp.n].cpu().numpy(), s.lb_history(T + 1), s.get_lambda().cpu().numpy())
    torch.cuda.synchronize()
    return out


def _no_alloc(ilp, alpha, T):
    import torch

    plan = B.Plan(B.Problem.from_ilp(ilp), hist_cap=max(64, T + 4))
    s = B.Solver(plan)
    g = torch.empty(max(ilp.n, 1), dtype=torch.float32, device="cuda")
    B.bddmp_solver_smooth_grad_noalloc(s.h, alpha, T, 1.0, g)
    out = (g[:ilp.n].cpu().numpy(), s.lb_history(T + 1), s.get_lambda().cpu().numpy())
    torch.cuda.synchronize()
    return out


def test_no_alloc_gradient_equals_workspace_gradient_twice():
    cases = [(I.config("5sub"), 0.1, 20), (I.config(1), 1.0, 5)]  # the second call is smaller
    for k, (ilp, alpha, T) in enumerate(cases):
        print(f"[no-alloc] call {k}: {ilp.name} alpha={alpha} T={T}", flush=True)
        g_ref, h_ref, lam_ref = _with_workspace(ilp, alpha, T)
        g, h, lam = _no_alloc(ilp, alpha, T)
        assert np.array_equal(g, g_ref), k
        assert np.array_equal(h, h_ref), k
        assert np.array_equal(lam, lam_ref), k
        # and the oracle's fp64 adjoint at the forward bar
        g_or, lb_or = Oracle(ilp).smooth_grad(alpha, T)
        assert h[-1] == pytest.approx(lb_or, rel=1e-4, abs=1e-4)
        assert np.abs(g - g_or).max() / max(1.0, np.abs(g_or).max()) <= 1e-4


def test_no_alloc_rejects_a_workspace_beyond_the_scratch():
    ilp = I.config("5sub")
    plan = B.Plan(B.Problem.from_ilp(ilp))
    T = 1000
    assert B.bddmp_smooth_workspace_bytes(plan.h, T) > 64 << 20
    import torch

    s = B.Solver(plan)
    g = torch.empty(ilp.n, dtype=torch.float32, device="cuda")
    n_hist = len(s.lb_history())
    with pytest.raises(B.BddmpError) as e:
        B.bddmp_solver_smooth_grad_noalloc(s.h, 0.1, T, 1.0, g)
    assert e.value.code == -1
    assert len(s.lb_history()) == n_hist  # nothing ran
