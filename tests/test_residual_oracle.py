"""Pins of the oracle's dual-feasibility residual and of its bound valid for any multipliers (no GPU).

The dual (D) of Sec. 3.1 asks sum_{j in J_i} lambda^j_i = c_i. For multipliers that break it, App. A.1
still gives a lower bound: relax the coupling by giving every row its own copy x^j of the variables and
keeping one free copy y in {0,1}^n that carries what the rows do not, c_i - sum_j lambda^j_i. The
minimum of sum_j <lambda^j, x^j> + <c - sum_j lambda^j, y> over x^j in X_j and y in {0,1}^n is at most
the ILP optimum (every feasible x gives x^j = x, y = x the value c^T x), and it splits into
sum_j E^j(lambda^j) plus the minimum over y of the free part.

The tests compute that relaxation by enumerating each row's feasible set and every y, in exact
rational arithmetic, and compare the oracle's bound with it; the residual max_i |c_i - sum_j
lambda^j_i| is recomputed in rationals too. Multipliers are dyadic rationals (multiples of 1/8 with
small numerators), so fp64 holds them and their sums exactly.
"""
import itertools
from fractions import Fraction

import numpy as np
import pytest

import bruteforce as bf
from oracle import Oracle
from paper_2009_00481_amd import instances as I


def _incidences(ilp):
    """(row, variable) per canonical incidence: rows in input order, a row's variables by rank."""
    rank = np.empty(ilp.n, np.int64)
    rank[np.asarray(ilp.order)] = np.arange(ilp.n)
    out = []
    for j in range(ilp.m):
        cols, coefs, _, _ = ilp.row(j)
        vs = sorted((int(v) for v, c in zip(cols, coefs) if c != 0), key=lambda v: rank[v])
        out.extend((j, v) for v in vs)
    return out


def _dyadic_costs(ilp, rng):
    """The same ILP with costs k/8, k in [-24, 24] (exact in binary floating point)."""
    c = rng.integers(-24, 25, size=ilp.n).astype(np.float64) / 8.0
    return I.ILP(ilp.n, c, ilp.row_ptr, ilp.col, ilp.coef, ilp.sense, ilp.rhs, ilp.order, name=ilp.name)


def _relaxation(ilp, inc, lam):
    """min over x^j in X_j and y in {0,1}^n of sum_j <lambda^j, x^j> + <c - sum_j lambda^j, y>, exact."""
    lamq = [Fraction(float(v)) for v in lam]
    total = Fraction(0)
    by_row = {}
    for q, (j, v) in enumerate(inc):
        by_row.setdefault(j, []).append((v, lamq[q]))
    for j in range(ilp.m):
        cols, coefs, s, b = ilp.row(j)
        coef_of = {int(v): int(c) for v, c in zip(cols, coefs)}
        pairs = by_row.get(j, [])
        if not pairs:
            continue
        best = None
        for x in itertools.product((0, 1), repeat=len(pairs)):
            if not bf.row_ok(s, sum(coef_of[v] * xv for (v, _), xv in zip(pairs, x)), b):
                continue
            val = sum((lv for (_, lv), xv in zip(pairs, x) if xv), Fraction(0))
            best = val if best is None or val < best else best
        assert best is not None, "row without a feasible point"
        total += best
    g = [Fraction(float(c)) for c in ilp.cost]
    for q, (j, v) in enumerate(inc):
        g[v] -= lamq[q]
    # the free copy y: enumerate {0,1}^n
    best_y = min(sum((gi for gi, yi in zip(g, y) if yi), Fraction(0)) for y in itertools.product((0, 1), repeat=ilp.n))
    return total + best_y, g


def _residual_exact(ilp, inc, g):
    has_row = {v for _, v in inc}
    return max((abs(g[v]) for v in range(ilp.n) if v in has_row), default=Fraction(0))


def _cases():
    for seed in range(14):
        rng = np.random.default_rng(700 + seed)
        n = int(rng.integers(3, 11))
        ilp = I.random_ilp(n, int(rng.integers(1, 7)), kmin=1, kmax=int(rng.integers(2, 6)),
                           cmax=int(rng.integers(1, 4)), seed=1700 + seed, cover_all=bool(seed % 3))
        yield seed, _dyadic_costs(ilp, rng), rng


@pytest.mark.parametrize("seed,ilp,rng", list(_cases()))
def test_any_lambda_bound_is_the_relaxation_with_a_free_copy(seed, ilp, rng):
    """Infeasible multipliers (sum_j lambda^j_i != c_i): the oracle's bound equals the enumerated
    relaxation exactly, lies below the ILP optimum, and the residual is the largest violation."""
    inc = _incidences(ilp)
    o = Oracle(ilp)
    o.init()
    for trial in range(4):
        lam = rng.integers(-20, 21, size=len(inc)).astype(np.float64) / 8.0
        o.set_lambda(lam)
        want, g = _relaxation(ilp, inc, lam)
        resid, any_lb = o.residual()
        assert any_lb == pytest.approx(float(want), abs=1e-12), (seed, trial)
        assert resid == float(_residual_exact(ilp, inc, g)), (seed, trial)
        opt = bf.ilp_optimum(ilp)
        if opt is not None:
            assert any_lb <= opt + 1e-12, (seed, trial, any_lb, opt)
        # the plain bound (sum_j E^j plus min(0, c_i) of the variables in no row) lacks the free copy's
        # part of the variables with rows: the two differ by exactly that part's minimum
        with_rows = {v for _, v in inc}
        free = sum((min(Fraction(0), g[v]) for v in with_rows), Fraction(0))
        assert o.lower_bound() - any_lb == pytest.approx(-float(free), abs=1e-12)


@pytest.mark.parametrize("seed,ilp,rng", list(_cases()))
def test_feasible_multipliers_give_zero_residual_and_the_plain_bound(seed, ilp, rng):
    """Multipliers with sum_j lambda^j_i = c_i exactly: residual 0, the any-lambda bound equals LB,
    and both equal the enumerated relaxation, also after iterations."""
    inc = _incidences(ilp)
    rows_of = {}
    for q, (j, v) in enumerate(inc):
        rows_of.setdefault(v, []).append(q)
    lam = np.zeros(len(inc))
    for v, qs in rows_of.items():
        part = rng.integers(-12, 13, size=len(qs) - 1).astype(np.float64) / 8.0
        lam[qs[:-1]] = part
        lam[qs[-1]] = ilp.cost[v] - part.sum()
    o = Oracle(ilp)
    o.init()
    o.set_lambda(lam)
    want, _ = _relaxation(ilp, inc, lam)
    resid, any_lb = o.residual()
    assert resid == 0.0
    assert any_lb == o.lower_bound()
    assert any_lb == pytest.approx(float(want), abs=1e-12)
    o.iterate(3)
    resid, any_lb = o.residual()
    opt = bf.ilp_optimum(ilp)
    # the updates keep sum_j lambda^j_i = c_i up to rounding (eq. "mma-update" moves mass between rows)
    assert resid <= 1e-12 * max(1.0, np.abs(ilp.cost).max())
    assert any_lb <= o.lower_bound() + 1e-15
    assert o.lower_bound() - any_lb <= ilp.n * resid + 1e-15
    if opt is not None:
        assert o.lower_bound() <= opt + 1e-9


def test_rows_free_variables_and_tightness():
    """Special cases with a known value: variables in no row contribute min(0, c_i) to both bounds;
    a single row with lambda = c and one variable per row attains the ILP optimum."""
    # x0 + x1 + x2 = 1 over three variables; x3, x4 in no row
    ilp = I.from_rows(5, [0.5, -0.25, 0.75, -1.5, 2.0], [([0, 1, 2], [1, 1, 1], 0, 1)])
    o = Oracle(ilp)
    o.init()
    resid, any_lb = o.residual()
    assert resid == 0.0
    assert any_lb == o.lower_bound() == -0.25 - 1.5
    assert any_lb == bf.ilp_optimum(ilp)
    # multipliers 1 above the costs on every incidence: E^j = -0.25 + 1 = 0.75, the free copy takes
    # each violated variable at -1, the no-row variables at min(0, c_i)
    o.set_lambda(np.array([1.5, 0.75, 1.75]))
    resid, any_lb = o.residual()
    assert resid == 1.0
    assert o.lower_bound() == pytest.approx(0.75 - 1.5)
    assert any_lb == pytest.approx(0.75 - 3.0 - 1.5)
    assert any_lb <= bf.ilp_optimum(ilp)
