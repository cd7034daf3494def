"""Pins of the oracle's smoothed variant (App. "Smoothing") and of its reverse-mode derivative.

What fixes the values independently of the oracle's own code:
- log-sum-exp marginals and energies by enumeration of each row's feasible set;
- Prop. "Approximation guarantees": E^j >= E^j_alpha >= E^j - alpha log |X_j|;
- alpha -> 0 gives the min-plus iterates;
- the smoothed bound is a coordinate ascent: non-decreasing;
- the derivative against central finite differences of the oracle's own smoothed bound, and at
  T = 0 against the closed form sum_j P_j(x_i = 1) / |J_i| (P_j the Gibbs distribution of row j,
  by enumeration), whose alpha -> 0 limit is the argmin indicator.
"""
import numpy as np
import pytest

import bruteforce as bf
from oracle import Oracle
from paper_2009_00481_amd import instances as I


def _lse_min(vals, alpha):
    vals = np.asarray(vals, np.float64)
    if vals.size == 0:
        return np.inf
    m = vals.min()
    return m - alpha * np.log(np.exp(-(vals - m) / alpha).sum())


def _small_cases():
    yield "rand", I.random_ilp(9, 6, kmax=4, cmax=3, seed=3)
    yield "forced", I.from_rows(8, [0.3, -0.7, 0.2, 0.9, -0.4, 0.25, 0.5, -0.1],
                                [([0, 1], [2, 3], 0, 5), ([2, 3], [1, 1], 1, 0), ([0, 2, 4], [1, 1, 1], 1, 2),
                                 ([1, 3, 5], [1, -1, 1], 2, 1), ([4, 5], [1, 1], 0, 1), ([4, 6, 7], [1, 1, 1], 0, 1)],
                                order=[3, 1, 5, 0, 2, 4, 7, 6])
    yield "potts", I.potts_grid(2, 3, 3, seed=1)
    yield "free", I.from_rows(5, [0.4, -0.3, 0.8, -1.2, 0.05], [([0, 1, 2], [1, 1, 1], 1, 1)])


def _row_lams(ilp, lam_canon, o):
    """lambda of each row's levels in level order, with the level variables."""
    w, var, _, _ = o.structure()
    out, q = [], 0
    for j in range(ilp.m):
        cols, coefs, _, _ = ilp.row(j)
        k = int(np.count_nonzero(coefs))
        out.append((var[q:q + k], lam_canon[q:q + k]))
        q += k
    return out


def _row_feasible(ilp, j, levels_vars):
    cols, coefs, sense, rhs = ilp.row(j)
    pos = {int(c): t for t, c in enumerate(cols)}
    order = [pos[int(v)] for v in levels_vars]
    X = bf.feasible_set(np.asarray(coefs)[order], sense, rhs)
    return np.asarray(X, np.float64).reshape(-1, len(order))


@pytest.mark.parametrize("alpha", [1.0, 0.1])
def test_marginals_and_energies_equal_enumeration(alpha):
    for name, ilp in _small_cases():
        o = Oracle(ilp)
        o.smooth_init(alpha)
        m0, m1 = o.smooth_marginals(alpha)
        e, ea = o.row_energies(alpha)
        lam = o.lam()
        q = 0
        for j, (vars_, lj) in enumerate(_row_lams(ilp, lam, o)):
            X = _row_feasible(ilp, j, vars_)
            costs = X @ lj
            assert ea[j] == pytest.approx(_lse_min(costs, alpha), abs=1e-12), (name, j)
            assert e[j] == pytest.approx(costs.min(), abs=1e-12)
            for t in range(len(vars_)):
                for beta, got in ((0, m0[q + t]), (1, m1[q + t])):
                    want = _lse_min(costs[X[:, t] == beta], alpha)
                    if np.isinf(want):
                        assert np.isinf(got) and got > 0
                    else:
                        assert got == pytest.approx(want, abs=1e-12), (name, j, t, beta)
            q += len(vars_)


@pytest.mark.parametrize("alpha", [1.0, 0.3, 0.01])
def test_approximation_sandwich(alpha):
    ilp = I.random_ilp(30, 20, kmax=6, cmax=3, seed=8)
    o = Oracle(ilp)
    o.smooth_init(alpha)
    o.smooth_iterate(alpha, 3)
    e, ea = o.row_energies(alpha)
    cnt = o.count_solutions()
    assert np.all(e >= ea - 1e-12)
    assert np.all(ea >= e - alpha * np.log(cnt) - 1e-12)
    # strict where a row has more than one solution (while the other solutions' weight exp(-gap /
    # alpha) is representable in double precision)
    if alpha >= 0.3:
        assert np.all((e > ea)[cnt > 1])


def test_small_alpha_recovers_min_plus():
    """Instances without forced variables (there the smoothed forced-row rule differs from the
    min-plus one; see the next test)."""
    for ilp in (I.config(1), I.potts_grid(4, 5, 3, seed=3), I.graph_matching(30, 30, 4, 40, seed=1)):
        o = Oracle(ilp)
        lb0 = o.init()
        tr = o.iterate(10)
        s = Oracle(ilp)
        sl0 = s.smooth_init(1e-9)
        st = s.smooth_iterate(1e-9, 10)
        np.testing.assert_allclose(st, tr, rtol=0, atol=1e-6)
        assert sl0 == pytest.approx(lb0, abs=1e-6)
        np.testing.assert_allclose(s.lam(), o.lam(), rtol=0, atol=1e-6)


@pytest.mark.parametrize("alpha", [1.0, 0.1, 0.01])
def test_smoothed_bound_is_monotone(alpha):
    for ilp in (I.config("5sub"), I.random_ilp(60, 45, kmax=7, seed=5), I.tomography(6, seed=2, unary="normal")):
        o = Oracle(ilp)
        lb0 = o.smooth_init(alpha)
        tr = np.concatenate([[lb0], o.smooth_iterate(alpha, 15)])
        assert np.all(np.diff(tr) >= -1e-10 * (1 + np.abs(tr[1:]))), (ilp.name, np.diff(tr).min())


def test_forced_rows_keep_the_smoothed_bound_monotone_and_match_min_plus_bound():
    """With forced variables (tomography lines with right-hand side 0, random rows) the smoothed
    rule moves only rows whose move raises the bound, so the smoothed bound is monotone; the
    starting bounds agree as alpha -> 0 (later iterates differ: the min-plus rule also moves rows
    that change no energy, which changes what later variables see)."""
    for ilp in (I.random_ilp(40, 30, kmax=6, seed=2), I.tomography(5, seed=1, unary="normal")):
        o = Oracle(ilp)
        tr = np.concatenate([[o.init()], o.iterate(10)])
        s = Oracle(ilp)
        st = np.concatenate([[s.smooth_init(1e-9)], s.smooth_iterate(1e-9, 10)])
        assert np.all(np.diff(st) >= -1e-9)
        assert st[0] == pytest.approx(tr[0], abs=1e-6)
        assert st[-1] > st[0]


def _fd(ilp, alpha, T, idx, h=1e-6):
    out = []
    for i in idx:
        vals = []
        for sgn in (1, -1):
            c = ilp.cost.copy()
            c[i] += sgn * h
            q = I.ILP(ilp.n, c, ilp.row_ptr, ilp.col, ilp.coef, ilp.sense, ilp.rhs, ilp.order)
            o = Oracle(q)
            o.smooth_init(alpha)
            tr = o.smooth_iterate(alpha, T)
            vals.append(tr[-1] if T else o.lower_bound())
        out.append((vals[0] - vals[1]) / (2 * h))
    return np.array(out)


@pytest.mark.parametrize("alpha", [1.0, 0.1])
@pytest.mark.parametrize("T", [0, 1, 3])
def test_gradient_equals_finite_differences(alpha, T):
    for name, ilp in _small_cases():
        o = Oracle(ilp)
        g, lb = o.smooth_grad(alpha, T)
        s = Oracle(ilp)
        s.smooth_init(alpha)
        tr = s.smooth_iterate(alpha, T)
        assert lb == pytest.approx(tr[-1] if T else s.lower_bound(), abs=1e-12)
        fd = _fd(ilp, alpha, T, range(ilp.n))
        np.testing.assert_allclose(g, fd, rtol=1e-5, atol=2e-6, err_msg=f"{name} alpha={alpha} T={T}")


def test_gradient_on_a_potts_subgrid_sampled():
    ilp = I.potts_grid(6, 6, 4, seed=4)
    alpha, T = 0.1, 4
    g, _ = Oracle(ilp).smooth_grad(alpha, T)
    idx = np.random.default_rng(0).choice(ilp.n, size=25, replace=False)
    fd = _fd(ilp, alpha, T, idx)
    np.testing.assert_allclose(g[idx], fd, rtol=1e-5, atol=2e-6)


@pytest.mark.parametrize("alpha", [1.0, 0.2])
def test_gradient_at_t0_is_mean_marginal_probability(alpha):
    for name, ilp in _small_cases():
        o = Oracle(ilp)
        g, _ = o.smooth_grad(alpha, 0)
        s = Oracle(ilp)
        s.smooth_init(alpha)
        lam = s.lam()
        want = np.zeros(ilp.n)
        nj = np.zeros(ilp.n)
        for j, (vars_, lj) in enumerate(_row_lams(ilp, lam, s)):
            X = _row_feasible(ilp, j, vars_)
            costs = X @ lj
            p = np.exp(-(costs - costs.min()) / alpha)
            p /= p.sum()
            for t, v in enumerate(vars_):
                want[v] += float(p @ X[:, t])
                nj[v] += 1
        free = nj == 0
        want[~free] /= nj[~free]
        c = ilp.cost[free]
        want[free] = 1.0 / (1.0 + np.exp(c / alpha))
        np.testing.assert_allclose(g, want, rtol=1e-9, atol=1e-12, err_msg=name)


def test_gradient_at_t0_tends_to_argmin_indicator():
    # rows with unique minimisers at lambda = c / |J_i|
    rows = [([0, 1, 2], [1, 1, 1], 0, 1), ([1, 2, 3], [1, 1, 1], 1, 2), ([3, 4], [1, -1], 2, 0)]
    ilp = I.from_rows(5, [0.9, -0.6, 0.2, -0.3, 0.5], rows)
    o = Oracle(ilp)
    g, _ = o.smooth_grad(1e-3, 0)
    s = Oracle(ilp)
    s.init()
    lam = s.lam()
    want = np.zeros(ilp.n)
    nj = np.zeros(ilp.n)
    for j, (vars_, lj) in enumerate(_row_lams(ilp, lam, s)):
        X = _row_feasible(ilp, j, vars_)
        costs = X @ lj
        best = np.argsort(costs)
        assert costs[best[1]] - costs[best[0]] > 0.05
        for t, v in enumerate(vars_):
            want[v] += X[best[0], t]
            nj[v] += 1
    want /= nj
    np.testing.assert_allclose(g, want, atol=1e-6)
