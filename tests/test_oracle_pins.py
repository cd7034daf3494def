"""Pins of the CPU oracle against what the paper and the mathematics fix (no GPU).

Each test compares the oracle with something other than itself: the paper's
worked example (Fig. "bdd"), closed forms, brute-force enumeration, exact
rational arithmetic, weak duality and the propositions of Sec. 3 and 5.
"""
import json
import os

import numpy as np
import pytest

import bruteforce as bf
from oracle import ORC_CHECK_ALL, Oracle, OracleError, build_row
from paper_2009_00481_amd import instances as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_fig1_worked_example():
    g = json.load(open(os.path.join(GOLDEN, "fig1_bdd.json")))
    w, lo, hi = build_row(g["row"]["coefs"], 0, g["row"]["rhs"])
    assert w.tolist() == g["level_width"]
    assert lo.tolist() == g["lo"]
    assert hi.tolist() == g["hi"]
    # the green path x1=0, x3=1, x7=0 visits 3a then 7b and ends in TOP
    first = np.concatenate([[0], np.cumsum(w)])
    node = 0
    for lvl, x in enumerate(g["green_path"]["x"]):
        assert [lvl, node] == g["green_path"]["nodes"][lvl]
        c = (hi if x else lo)[first[lvl] + node]
        node = c
    assert node == -2


def _random_row(rng):
    k = int(rng.integers(1, 13))
    a = rng.integers(1, 4, size=k) * rng.choice([-1, 1], size=k)
    lo_, hi_ = int(a[a < 0].sum()), int(a[a > 0].sum())
    b = int(rng.integers(lo_ - 1, hi_ + 2))
    return a.astype(np.int64), int(rng.integers(0, 3)), b


def test_builder_equals_truth_table_bdd():
    rng = np.random.default_rng(1234)
    n_inf = 0
    for _ in range(400):
        a, s, b = _random_row(rng)
        ref = bf.truth_table_bdd(a.tolist(), s, b)
        if ref is None:
            with pytest.raises(OracleError) as e:
                build_row(a, s, b)
            assert e.value.code == -2
            n_inf += 1
            continue
        w, lo, hi = build_row(a, s, b)
        assert w.tolist() == ref[0], (a, s, b)
        assert lo.tolist() == ref[1], (a, s, b)
        assert hi.tolist() == ref[2], (a, s, b)
    assert 0 < n_inf < 200


def _live(lo, hi):
    return int((lo != -1).sum() + (hi != -1).sum())


@pytest.mark.parametrize("k", range(2, 13))
def test_closed_form_sizes(k):
    # simplex sum x = 1: 2k-1 nodes, 3k-2 live arcs
    w, lo, hi = build_row([1] * k, 0, 1)
    assert w.sum() == 2 * k - 1 and _live(lo, hi) == 3 * k - 2
    # at most one: 2k-1 nodes, 3k-1 live arcs
    w, lo, hi = build_row([1] * k, 1, 1)
    assert w.sum() == 2 * k - 1 and _live(lo, hi) == 3 * k - 1
    # marginalisation x_u - sum_k y_k = 0 with the unary first: 2L+1 nodes, 3L+1 live arcs
    L = k
    w, lo, hi = build_row([1] + [-1] * L, 0, 0)
    assert w.sum() == 2 * L + 1 and _live(lo, hi) == 3 * L + 1


def test_closed_form_small_rows():
    assert build_row([-1, 1], 1, 0)[0].sum() == 3      # y <= x_a, order (x_a, y)
    assert build_row([1, -1], 1, 0)[0].sum() == 3      # y <= x_a, order (y, x_a)
    assert build_row([1, 1, -1], 1, 1)[0].sum() == 5   # x_a + x_b - y <= 1


def test_solution_counts_closed_forms():
    # counting algebra (Table "algebras"): |X| of simplex k = k, at-most-one k = k+1, marginalisation = L+1
    rows = []
    for k in range(1, 9):
        rows.append((list(range(k)), [1] * k, 0, 1))
    for k in range(1, 9):
        rows.append((list(range(k)), [1] * k, 1, 1))
    for L in range(1, 9):
        rows.append((list(range(L + 1)), [1] + [-1] * L, 0, 0))
    ilp = I.from_rows(10, np.zeros(10), rows)
    o = Oracle(ilp)
    cnt = o.count_solutions()
    want = [k for k in range(1, 9)] + [k + 1 for k in range(1, 9)] + [L + 1 for L in range(1, 9)]
    assert cnt.tolist() == want


def _tiny_ilps():
    out = []
    for s in range(8):
        out.append(I.random_ilp(10, 7, kmax=4, seed=s))
    for s in range(3):
        out.append(I.random_ilp(12, 9, kmax=5, cmax=1, seed=100 + s))
    out.append(I.potts_grid(2, 3, 2, unary="normal", weight=(0.2, 1.0), seed=7))
    out.append(I.potts_grid(3, 3, 2, unary="uniform", weight=0.5, seed=3))
    # rows that force variables: 2a + 3b = 5 forces a = b = 1; c + d <= 0 forces c = d = 0
    out.append(I.from_rows(6, [0.3, -0.7, 0.2, 0.9, -0.4, 0.25], [
        ([0, 1], [2, 3], 0, 5), ([2, 3], [1, 1], 1, 0), ([0, 2, 4], [1, 1, 1], 1, 2),
        ([1, 3, 5], [1, -1, 1], 2, 1), ([4, 5], [1, 1], 0, 1)], order=[3, 1, 5, 0, 2, 4]))
    return out


@pytest.mark.parametrize("idx", range(14))
def test_oracle_equals_exact_enumeration_dbca(idx):
    """The oracle's bound trace and multipliers equal Alg. "Min-marginal averaging" run with
    min-marginals taken by enumeration in exact rationals."""
    ilp = _tiny_ilps()[idx]
    o = Oracle(ilp)
    lb0 = o.init()
    b = bf.BruteDBCA(ilp)
    assert lb0 == pytest.approx(float(b.lb()), rel=1e-12, abs=1e-12)
    tr = o.iterate(4)
    ref = [float(v) for v in b.iterate(4)]
    np.testing.assert_allclose(tr, ref, rtol=1e-10, atol=1e-10)
    lam = o.lam()
    np.testing.assert_allclose(lam, [float(v) for v in b.lam_canonical()], rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("idx", range(14))
def test_oracle_self_checks_propositions(idx):
    """Per update: incremental min-marginals equal from-scratch ones (Prop. "correctness"), the bound
    gain equals Prop. 1, all differences equal their mean afterwards (proof of Prop. 1) and
    sum_j lambda^j_i = c_i (constraint of (D))."""
    ilp = _tiny_ilps()[idx]
    o = Oracle(ilp)
    o.init(ORC_CHECK_ALL)
    o.iterate(3)
    chk = o.checks()
    assert np.all(chk <= 1e-9), chk


@pytest.mark.parametrize("idx", range(14))
def test_fresh_min_marginals_equal_enumeration(idx):
    ilp = _tiny_ilps()[idx]
    o = Oracle(ilp)
    o.init()
    o.iterate(2)
    lam = o.lam()
    m0, m1 = o.min_marginals()
    b = bf.BruteDBCA(ilp)
    q = 0
    for j, (vs, X) in enumerate(b.rows):
        for t, v in enumerate(vs):
            lamj = lam[q - t: q - t + len(vs)]
            for beta, got in ((0, m0[q]), (1, m1[q])):
                vals = [float(np.dot(lamj, x)) for x in X if x[t] == beta]
                want = min(vals) if vals else np.inf
                if np.isinf(want):
                    assert np.isinf(got) and got > 0
                else:
                    assert got == pytest.approx(want, rel=1e-12, abs=1e-12)
            q += 1


@pytest.mark.parametrize("seed", range(6))
def test_weak_duality_and_monotone(seed):
    ilp = I.random_ilp(14, 10, kmax=5, seed=50 + seed)
    opt = bf.ilp_optimum(ilp)
    o = Oracle(ilp)
    lb0 = o.init()
    tr = np.concatenate([[lb0], o.iterate(20)])
    scale = 1e-12 * (np.abs(ilp.cost).sum() + 1)
    assert np.all(np.diff(tr) >= -scale)
    assert tr[-1] <= opt + 1e-9


def test_lp_bound_for_unimodular_rows():
    """With coefficients in {0, +-1} one row plus the box is an integral polytope, so the dual
    optimum is the LP optimum and every bound must stay below it."""
    from scipy.optimize import linprog
    for ilp in (I.potts_grid(4, 4, 3, unary="normal", weight=(0.2, 1.0), seed=1),
                I.random_ilp(16, 12, kmax=5, cmax=1, seed=9)):
        A = np.zeros((ilp.m, ilp.n))
        for j in range(ilp.m):
            c, a, _, _ = ilp.row(j)
            A[j, c] = a
        eq = ilp.sense == 0
        le = ilp.sense == 1
        ge = ilp.sense == 2
        A_ub = np.vstack([A[le], -A[ge]])
        b_ub = np.concatenate([ilp.rhs[le], -ilp.rhs[ge]]).astype(float)
        res = linprog(ilp.cost, A_ub=A_ub if A_ub.size else None, b_ub=b_ub if A_ub.size else None,
                      A_eq=A[eq] if eq.any() else None, b_eq=ilp.rhs[eq].astype(float) if eq.any() else None,
                      bounds=[(0, 1)] * ilp.n, method="highs")
        assert res.status == 0
        o = Oracle(ilp)
        o.init()
        tr = o.iterate(60)
        assert tr[-1] <= res.fun + 1e-7
        assert tr[-1] >= tr[0] - 1e-12


def test_disjoint_rows_bound_is_constant():
    """Every variable in one row: the bound is sum_j min over X_j of c^T x from the start."""
    rows = [([0, 1, 2], [1, 1, 1], 0, 1), ([3, 4], [2, -1], 1, 1), ([5, 6, 7, 8], [1, -1, 1, 1], 2, 1)]
    cost = np.array([0.5, -0.25, 0.75, -1.0, 0.5, 0.1, -0.2, 0.3, -0.4])
    ilp = I.from_rows(9, cost, rows)
    want = 0.0
    for vs, cs, s, b in rows:
        X = bf.feasible_set(cs, s, b)
        want += min(float(np.dot(cost[vs], x)) for x in X)
    o = Oracle(ilp)
    assert o.init() == pytest.approx(want, abs=1e-12)
    np.testing.assert_allclose(o.iterate(5), want, atol=1e-12)


def test_single_row_bound_is_optimum():
    rows = [([0, 1, 2, 3, 4], [2, -1, 3, 1, -2], 1, 1)]
    cost = np.array([-0.5, 0.4, -0.9, -0.1, 0.7])
    ilp = I.from_rows(5, cost, rows)
    o = Oracle(ilp)
    assert o.init() == pytest.approx(bf.ilp_optimum(ilp), abs=1e-12)


def test_unconstrained_variables_and_rounding():
    rows = [([0, 1], [1, 1], 1, 1), ([1, 2], [1, -1], 0, 0)]
    cost = np.array([-1.0, -2.0, 0.5, -3.0, 4.0])  # variables 3 and 4 are in no row
    ilp = I.from_rows(5, cost, rows)
    o = Oracle(ilp)
    o.init()
    tr = o.iterate(10)
    assert tr[-1] <= bf.ilp_optimum(ilp) + 1e-12
    M, x, obj, nviol = o.round()
    assert x[3] == 1 and x[4] == 0
    assert obj == pytest.approx(float(cost @ x))


@pytest.mark.parametrize("idx", [0, 3, 12, 13])
def test_round_consistency(idx):
    ilp = _tiny_ilps()[idx]
    o = Oracle(ilp)
    o.init()
    o.iterate(5)
    M, x, obj, nviol = o.round()
    assert np.array_equal(x, (M <= 0).astype(np.int8))
    assert obj == pytest.approx(float(ilp.cost @ x), abs=1e-12)
    bad = 0
    for j in range(ilp.m):
        c, a, s, b = ilp.row(j)
        bad += not bf.row_ok(s, int(a @ x[c]), b)
    assert bad == nviol
    m0, m1 = o.min_marginals()
    # M_i = sum over the variable's rows of m1 - m0
    w, var, _, _ = o.structure()
    Mi = np.zeros(ilp.n)
    np.add.at(Mi, var, m1 - m0)
    np.testing.assert_allclose(M, Mi, atol=1e-12)


def test_consensus_certifies_optimum():
    """Sec. 3.1: if the subproblem optima agree the consensus solves the problem, so when the rounded
    point is feasible and its cost meets the bound, it is the optimum."""
    found = 0
    for s in range(20):
        ilp = I.random_ilp(12, 8, kmax=4, seed=300 + s)
        o = Oracle(ilp)
        o.init()
        lb = o.iterate(30)[-1]
        M, x, obj, nviol = o.round()
        if nviol == 0 and abs(obj - lb) < 1e-9:
            assert bf.ilp_optimum(ilp) == pytest.approx(obj, abs=1e-9)
            found += 1
    assert found > 0


def test_errors():
    with pytest.raises(OracleError) as e:
        Oracle(I.from_rows(3, np.zeros(3), [([0, 1], [1, 1], 0, 3)]))
    assert e.value.code == -2
    with pytest.raises(OracleError) as e:
        Oracle(I.from_rows(3, np.zeros(3), [([0, 0], [1, 1], 0, 1)]))
    assert e.value.code == -1
    ilp = I.from_rows(3, np.zeros(3), [([0, 1], [1, 1], 0, 1)])
    ilp.order = np.array([0, 0, 1], np.int32)
    with pytest.raises(OracleError):
        Oracle(ilp)
    # rows forcing x0 to 1 and to 0
    with pytest.raises(OracleError) as e:
        o = Oracle(I.from_rows(2, np.ones(2), [([0, 1], [1, 1], 0, 2), ([0], [1], 1, 0)]))
        o.init()
        o.iterate(1)
    assert e.value.code == -5


def test_config1_sizes_and_fp32_mirror():
    ilp = I.config(1)
    c = I.potts_counts(8, 8, 3)
    o = Oracle(ilp)
    assert (o.n, o.m, o.n_incidences, o.n_nodes) == (c["n"], c["m"], c["incidences"], c["nodes"])
    assert o.n_live_arcs == 7168
    o.init()
    t64 = o.iterate(30)
    o32 = Oracle(ilp, precision="f32")
    o32.init()
    t32 = o32.iterate(30)
    np.testing.assert_allclose(t32, t64, rtol=1e-5)
