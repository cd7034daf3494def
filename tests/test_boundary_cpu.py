"""Status codes of the C-ABI that the host half decides (no device calls): every code the problem
and plan calls can return, input validation of costs and row magnitudes, and the real-valued row
entry point's integrality rule (integer rows, Sec. 3 Example "ILP"; partial sums of Sec. 5.2)."""
import numpy as np
import pytest

from paper_2009_00481_amd import binding as B
from paper_2009_00481_amd import instances as I


def _code(fn, *a, **kw):
    with pytest.raises(B.BddmpError) as e:
        fn(*a, **kw)
    return e.value.code


@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf])
def test_nonfinite_cost_is_rejected(bad):
    c = np.array([0.5, bad, -1.0])
    assert _code(B.Problem, 3, c) == -8


def test_row_magnitude_limit():
    p = B.Problem(3, np.zeros(3))
    big = 1 << 62
    # one coefficient at 2^62, the rhs at 2^62, and sums crossing it
    assert _code(p.add_rows, [0, 1], [0], [big], [1], [0]) == -1
    assert _code(p.add_rows, [0, 1], [0], [1], [1], [big]) == -1
    assert _code(p.add_rows, [0, 1], [0], [1], [1], [-big]) == -1
    assert _code(p.add_rows, [0, 2], [0, 1], [1 << 61, 1 << 61], [1], [0]) == -1
    assert _code(p.add_rows, [0, 2], [0, 1], [1 << 61, -(1 << 60)], [1], [1 << 60]) == -1
    assert _code(p.add_rows, [0, 1], [0], [-(2 ** 63)], [1], [0]) == -1
    # nothing of a rejected call is kept; just below the limit is accepted and builds
    p.add_rows([0, 2], [0, 1], [(1 << 61) - 1, -(1 << 60)], [1], [1 << 60])
    pl = B.Plan(p)
    assert pl.stats.n_bdds == 1 and pl.stats.n_incidences == 2


def test_real_rows_need_integers():
    p = B.Problem(3, np.zeros(3))
    assert _code(B.bddmp_problem_add_rows_real, p.h, [0, 2], [0, 1], [1.0, 0.5], [1], [1.0]) == -4
    assert _code(B.bddmp_problem_add_rows_real, p.h, [0, 2], [0, 1], [1.0, 1.0], [1], [1.5]) == -4
    assert _code(B.bddmp_problem_add_rows_real, p.h, [0, 1], [0], [2.0 ** 53], [1], [0.0]) == -4
    assert _code(B.bddmp_problem_add_rows_real, p.h, [0, 1], [0], [np.nan], [1], [0.0]) == -4
    assert _code(B.bddmp_problem_add_rows_real, p.h, [0, 1], [0], [1.0], [1], [np.inf]) == -4
    # other argument errors pass through to the integer call
    assert _code(B.bddmp_problem_add_rows_real, p.h, [0, 1], [7], [1.0], [1], [1.0]) == -1
    assert _code(B.bddmp_problem_add_rows_real, p.h, [0, 1], [0], [1.0], [3], [1.0]) == -1


@pytest.mark.parametrize("seed", range(4))
def test_real_rows_build_the_integer_plan(seed):
    ilp = I.random_ilp(30, 20, kmax=6, cmax=3, seed=seed)
    a = B.Problem(ilp.n, ilp.cost)
    a.add_rows(ilp.row_ptr, ilp.col, ilp.coef, ilp.sense, ilp.rhs)
    a.set_order(ilp.order)
    b = B.Problem(ilp.n, ilp.cost)
    # a CSR whose row_ptr starts inside a larger array
    pad = 3
    rp = ilp.row_ptr + pad
    col = np.concatenate([np.zeros(pad, np.int32), ilp.col])
    coef = np.concatenate([np.full(pad, 0.25), ilp.coef.astype(np.float64)])
    B.bddmp_problem_add_rows_real(b.h, rp, col, coef, ilp.sense, ilp.rhs.astype(np.float64))
    b.set_order(ilp.order)
    pa, pb = B.Plan(a), B.Plan(b)
    for x, y in zip(pa.structure(), pb.structure()):
        assert np.array_equal(x, y)
    assert pa.stats.as_dict() == pb.stats.as_dict()


def test_every_plan_status_code():
    """The codes bddmp_problem_* and bddmp_plan_* return, each from the condition that defines it."""
    z = np.zeros(3)
    # -1 INVALID_ARG: column out of range, bad sense, repeated column, bad permutation, bad tiling
    assert _code(B.Problem(3, z).add_rows, [0, 1], [5], [1], [0], [1]) == -1
    assert _code(B.Problem(3, z).add_rows, [0, 1], [1], [1], [3], [1]) == -1
    assert _code(lambda: B.Plan(B.Problem.from_ilp(I.from_rows(3, z, [([0, 0], [1, 1], 0, 1)])))) == -1
    assert _code(B.Problem(3, z).set_order, [0, 0, 1]) == -1
    assert _code(lambda: B.Plan(B.Problem.from_ilp(I.config(1)), tiling="3,0,0,0")) == -1
    # -2 ROW_INFEASIBLE: x0 + x1 = 3 has no 0/1 point; a row without variables that fails
    assert _code(lambda: B.Plan(B.Problem.from_ilp(I.from_rows(3, z, [([0, 1], [1, 1], 0, 3)])))) == -2
    assert _code(lambda: B.Plan(B.Problem.from_ilp(I.from_rows(3, z, [([], [], 1, -1)])))) == -2
    # -3 BDD_TOO_LARGE: node budget
    assert _code(lambda: B.Plan(B.Problem.from_ilp(I.config(1)), node_budget=1000)) == -3
    # -4 NOT_INTEGER: real-valued rows
    assert _code(B.bddmp_problem_add_rows_real, B.Problem(3, z).h, [0, 1], [0], [0.5], [1], [1.0]) == -4
    # -5 CONFLICT: one row forces x0 = 1, another x0 = 0
    assert _code(lambda: B.Plan(B.Problem.from_ilp(
        I.from_rows(2, np.ones(2), [([0, 1], [1, 1], 0, 2), ([0], [1], 1, 0)])))) == -5
    # -7 BAD_STATE: a solver call without a bound solver
    assert _code(B.bddmp_solver_iterate, None, 1) == -7
    assert _code(B.bddmp_solver_lower_bound, None) == -7
    # -8 NONFINITE: a cost that is not finite
    assert _code(B.Problem, 2, np.array([1.0, np.nan])) == -8
