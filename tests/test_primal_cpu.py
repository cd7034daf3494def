"""CPU tests of the primal heuristic (Sec. 4; App. "Primal heuristic", "Variable fixations").

Pins: the restricted diagram of Fig. "bdd-restricted" (fixture), restrictions against enumeration
of each row's feasible set, the library search against the enumeration-based oracle of the same
algorithm on the same total differences, and feasibility of every solution it reports.
"""
import json
import os

import numpy as np
import pytest

from oracle import Oracle
from oracle.primal import primal_heuristic
from paper_2009_00481_amd import binding as B
from paper_2009_00481_amd import instances as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _holds(ilp, x):
    for j in range(ilp.m):
        cols, coefs, sense, rhs = ilp.row(j)
        s = int(np.dot(coefs, x[cols]))
        if not ((sense == 0 and s == rhs) or (sense == 1 and s <= rhs) or (sense == 2 and s >= rhs)):
            return False
    return True


def test_restricted_diagram_of_the_figure():
    g = json.load(open(os.path.join(GOLDEN, "fig_bdd_restricted.json")))
    ilp = I.from_rows(3, [0.0, 0.0, 0.0], [([0, 1, 2], g["row"]["coefs"], 0, g["row"]["rhs"])])
    plan = B.Plan(B.Problem.from_ilp(ilp))
    alive, lo, hi, feas = B.bddmp_plan_restrict_row(plan.h, 0, int(plan.stats.n_nodes), [g["fix"]["level"]],
                                                    [g["fix"]["value"]])
    assert feas
    assert alive.astype(int).tolist() == g["alive"]
    for u, v in g["lo"].items():
        assert lo[int(u)] == v
    for u, v in g["hi"].items():
        assert hi[int(u)] == v


def _paths(level_width, lo, hi, alive):
    """Root-to-TRUE paths of a (restricted) diagram as 0/1 tuples."""
    first = np.concatenate([[0], np.cumsum(level_width)])
    out = []

    def walk(l, u, x):
        if not alive[first[l] + u]:
            return
        for b, ch in ((0, lo[first[l] + u]), (1, hi[first[l] + u])):
            if ch == -2:
                out.append(tuple(x + [b]))
            elif ch >= 0:
                walk(l + 1, ch, x + [b])

    walk(0, 0, [])
    return sorted(out)


@pytest.mark.parametrize("seed", range(8))
def test_restrictions_equal_enumeration(seed):
    rng = np.random.default_rng(seed)
    ilp = I.random_ilp(12, 6, kmin=3, kmax=8, cmax=3, seed=seed, shuffle_order=False)
    plan = B.Plan(B.Problem.from_ilp(ilp))
    w, var, lo, hi = plan.structure()
    inc = 0
    node = 0
    for j in range(ilp.m):
        cols, coefs, sense, rhs = ilp.row(j)
        k = int(np.count_nonzero(coefs))
        lw = w[inc:inc + k]
        nn = int(lw.sum())
        vars_ = var[inc:inc + k]
        fix_vars = rng.choice(vars_, size=min(2, k), replace=False)
        fix_vals = rng.integers(0, 2, size=fix_vars.shape[0]).astype(np.int8)
        alive, rlo, rhi, feas = B.bddmp_plan_restrict_row(plan.h, j, nn, fix_vars, fix_vals)
        # enumeration of the row's solutions in level order, restricted
        coef_of = {int(c): int(a) for c, a in zip(cols, coefs)}
        want = []
        import itertools
        for x in itertools.product((0, 1), repeat=k):
            s = sum(coef_of[int(v)] * xi for v, xi in zip(vars_, x))
            ok = (sense == 0 and s == rhs) or (sense == 1 and s <= rhs) or (sense == 2 and s >= rhs)
            if ok and all(x[list(vars_).index(fv)] == fb for fv, fb in zip(fix_vars, fix_vals)):
                want.append(x)
        assert feas == bool(want), (seed, j)
        if want:
            assert _paths(lw, rlo, rhi, alive) == sorted(want), (seed, j)
            # every remaining node lies on a root-to-TRUE path (both removal rules applied)
            first = np.concatenate([[0], np.cumsum(lw)])
            on_path = np.zeros(nn, bool)
            for x in want:
                u = 0
                for l, b in enumerate(x):
                    on_path[first[l] + u] = True
                    ch = rlo[first[l] + u] if b == 0 else rhi[first[l] + u]
                    u = ch
            assert np.array_equal(alive, on_path), (seed, j)
        inc += k
        node += nn


def _instances():
    yield I.config(1)
    yield I.random_ilp(30, 22, kmax=6, cmax=2, seed=1)
    yield I.random_ilp(40, 30, kmax=7, cmax=3, seed=7)
    yield I.graph_matching(25, 25, 4, 30, seed=2)
    yield I.tracking(150, seed=4)
    yield I.tomography(4, seed=3, unary="normal")


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_search_equals_oracle_and_is_feasible(mode):
    for ilp in _instances():
        o = Oracle(ilp)
        o.init()
        o.iterate(15)
        M, _, _, _ = o.round()
        plan = B.Plan(B.Problem.from_ilp(ilp))
        x, obj, feas, implied = plan.primal_search(M.astype(np.float32), mode)
        xr, objr, feasr = primal_heuristic(ilp, M, mode)
        assert feas == feasr, ilp.name
        assert np.array_equal(x, xr), ilp.name
        assert obj == pytest.approx(objr, abs=1e-9)
        if feas:
            assert _holds(ilp, x.astype(np.int64)), ilp.name
            assert implied >= 0


def test_search_improves_on_sign_rounding_for_potts():
    ilp = I.potts_grid(12, 12, 4, seed=5)
    o = Oracle(ilp)
    o.init()
    o.iterate(30)
    M, xr, objr, nviol = o.round()
    plan = B.Plan(B.Problem.from_ilp(ilp))
    x, obj, feas, _ = plan.primal_search(M.astype(np.float32), 0)
    assert feas and _holds(ilp, x.astype(np.int64))
    # the bound after 30 iterations is below any feasible objective
    assert obj >= o.lower_bound() - 1e-9


def test_search_errors():
    plan = B.Plan(B.Problem.from_ilp(I.config(1)))
    with pytest.raises(B.BddmpError) as e:
        plan.primal_search(np.zeros(plan.n, np.float32), 3)
    assert e.value.code == -1
    with pytest.raises(B.BddmpError) as e:
        B.bddmp_plan_restrict_row(plan.h, plan.stats.n_bdds, 4, [0], [1])
    assert e.value.code == -1


@pytest.mark.parametrize("seed,mode", [(7, 1), (27, 0), (41, 0), (42, 2), (53, 2)])
def test_search_backtracks_past_dead_ends(seed, mode):
    """Instances where the dive with one-value retries dead-ends (no solution with a budget of 0
    dead ends) while the depth-first search finds one; library and oracle agree on both."""
    ilp = I.random_ilp(24, 18, kmin=2, kmax=6, cmax=2, seed=seed)
    o = Oracle(ilp)
    o.init()
    o.iterate(3)
    M, _, _, _ = o.round()
    plan = B.Plan(B.Problem.from_ilp(ilp))
    for budget in (0, 100000):
        x, obj, feas, _ = plan.primal_search(M.astype(np.float32), mode, max_dead_ends=budget)
        xr, objr, feasr = primal_heuristic(ilp, M, mode, max_dead_ends=budget)
        assert feas == feasr and np.array_equal(x, xr), budget
        assert feas == (budget > 0)
        if feas:
            assert _holds(ilp, x.astype(np.int64))
