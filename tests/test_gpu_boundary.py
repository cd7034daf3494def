"""GPU tests of the boundary's checks of device inputs and of the bound for any multipliers.

- Multipliers that break the dual constraint sum_j lambda^j_i = c_i (problem (D), Sec. 3.1), set
  through bddmp_solver_set_lambda: bound, residual and the App. A.1 bound valid for any lambda
  against the oracle given the same multipliers (dyadic values, so every sum is exact in fp32 and
  fp64 and the two sides agree to rounding of the fp64 sums).
- NaN and infinities injected through set_lambda, set_copy_duals and set_costs come back as
  NONFINITE (-8) with the solver's state unchanged; finite multipliers whose row minimum overflows
  fp32 give an infinite bound, which lower_bound reports as NONFINITE. Only values change: every
  kernel runs on the same sizes as in a good call.
"""
import numpy as np
import pytest

from oracle import Oracle
from paper_2009_00481_amd import binding as B
from paper_2009_00481_amd import instances as I

pytestmark = pytest.mark.gpu


def _solver(ilp, **kw):
    plan = B.Plan(B.Problem.from_ilp(ilp), **kw)
    return B.Solver(plan), plan


@pytest.mark.parametrize("name", ["cfg1", "rand", "tomo"])
def test_infeasible_multipliers_match_oracle(name):
    import torch

    ilp = {"cfg1": lambda: I.config(1), "rand": lambda: I.random_ilp(40, 30, kmax=8, cmax=3, seed=5),
           "tomo": lambda: I.tomography(6, seed=2, unary="normal")}[name]()
    print(f"[any-lambda] {name}", flush=True)
    s, plan = _solver(ilp)
    rng = np.random.default_rng(11)
    o = Oracle(ilp)
    o.init()
    for trial in range(3):
        lam = rng.integers(-20, 21, size=s.n_incidences).astype(np.float64) / 8.0
        s.set_lambda(torch.tensor(lam, dtype=torch.float32, device="cuda"))
        lb, resid, any_lb = s.lower_bound()
        o.set_lambda(lam)
        r_resid, r_any = o.residual()
        assert lb == pytest.approx(o.lower_bound(), rel=1e-12, abs=1e-9), trial
        assert resid == pytest.approx(r_resid, rel=1e-12, abs=1e-12), trial
        assert any_lb == pytest.approx(r_any, rel=1e-12, abs=1e-9), trial
        assert resid > 0 and any_lb < lb
    # the multipliers then iterate as the oracle's do from the same point
    s.iterate(5)
    tr = o.iterate(5)
    lb, resid, any_lb = s.lower_bound()
    r_resid, r_any = o.residual()
    assert lb == pytest.approx(tr[-1], rel=1e-4, abs=1e-4)
    assert any_lb == pytest.approx(r_any, rel=1e-4, abs=1e-4)
    torch.cuda.synchronize()


@pytest.mark.parametrize("bad", [float("nan"), float("inf"), float("-inf")])
def test_set_lambda_rejects_nonfinite(bad):
    import torch

    ilp = I.config(1)
    s, plan = _solver(ilp)
    s.iterate(4)
    before = s.get_lambda().clone()
    lb_before = s.lower_bound()[0]
    n_hist = len(s.lb_history())
    lam = before.clone()
    lam[int(lam.numel() // 3)] = bad
    with pytest.raises(B.BddmpError) as e:
        s.set_lambda(lam)
    assert e.value.code == -8
    assert torch.equal(s.get_lambda(), before)
    assert s.lower_bound()[0] == lb_before
    assert len(s.lb_history()) == n_hist
    # a good call afterwards works and resumes bitwise
    s.set_lambda(before)
    s.iterate(2)
    ref, _ = _solver(ilp)
    ref.iterate(4)
    ref.set_lambda(ref.get_lambda().clone())
    ref.iterate(2)
    assert torch.equal(s.get_lambda(), ref.get_lambda())
    torch.cuda.synchronize()


def test_set_copy_duals_rejects_nonfinite():
    import torch

    ilp = I.tomography(8, seed=3)
    s, plan = _solver(ilp, n_intervals=2)
    assert plan.stats.n_copy_pairs > 0
    s.iterate(3)
    state = [t.clone() for t in s.copy_duals()]
    for k in range(4):
        bad = [t.clone() for t in state]
        bad[k][0] = float("nan") if k % 2 == 0 else float("inf")
        with pytest.raises(B.BddmpError) as e:
            s.set_copy_duals(*bad)
        assert e.value.code == -8, k
        for a, b in zip(s.copy_duals(), state):
            assert torch.equal(a, b)
    s.set_copy_duals(*state)
    torch.cuda.synchronize()


def test_set_costs_rejects_nonfinite():
    import torch

    ilp = I.config(1)
    s, plan = _solver(ilp)
    c = torch.tensor(ilp.cost, dtype=torch.float64, device="cuda")
    c[7] = float("nan")
    with pytest.raises(B.BddmpError) as e:
        B.bddmp_solver_set_costs(s.h, c)
    assert e.value.code == -8
    # the plan's costs still hold: instance bounds are available
    s.instance_bounds()
    c[7] = float("-inf")
    with pytest.raises(B.BddmpError) as e:
        B.bddmp_solver_set_costs(s.h, c)
    assert e.value.code == -8
    torch.cuda.synchronize()


def test_overflowing_bound_is_nonfinite():
    """x0 + x1 = 2 forces both variables to 1, so E = lambda_0 + lambda_1, which overflows fp32 for
    multipliers of 3e38; lower_bound reports NONFINITE and still returns the value."""
    import torch

    ilp = I.from_rows(3, [1.0, 1.0, -0.5], [([0, 1], [1, 1], 0, 2), ([2], [1], 1, 1)])
    s, plan = _solver(ilp)
    lb, _, _ = s.lower_bound()
    assert lb == pytest.approx(1.5)
    s.set_lambda(torch.tensor([3e38, 3e38, -0.5], dtype=torch.float32, device="cuda"))
    with pytest.raises(B.BddmpError) as e:
        s.lower_bound()
    assert e.value.code == -8
    out = np.zeros(1)
    rc = B.lib().bddmp_solver_lower_bound(s.h, out.ctypes.data_as(B.C.POINTER(B.C.c_double)), None, None)
    assert rc == -8 and out[0] == np.inf
    torch.cuda.synchronize()
