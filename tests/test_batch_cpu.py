"""CPU tests of the batched workload: the tomography and tracking generators, the oracle on them
(weak duality, LP bound, monotone bound), and the batched plan against the instances' own plans."""
import numpy as np
import pytest

from oracle import Oracle
from paper_2009_00481_amd import binding as B
from paper_2009_00481_amd import instances as I


def _dense(ilp):
    A = np.zeros((ilp.m, ilp.n))
    for j in range(ilp.m):
        c, a, _, _ = ilp.row(j)
        A[j, c] = a
    return A


def _row_values(ilp, x):
    return _dense(ilp) @ x.astype(np.float64)


def _holds(ilp, x):
    v = _row_values(ilp, x)
    s, b = ilp.sense, ilp.rhs
    return np.where(s == 0, v == b, np.where(s == 1, v <= b, v >= b))


@pytest.mark.parametrize("P", [3, 5, 8])
def test_tomography_sizes_and_truth_point(P):
    ilp = I.tomography(P, seed=P)
    nE = 2 * P * (P - 1)
    n_lines = P + P + 2 * (2 * P - 1)
    assert ilp.n == 3 * P * P + 9 * nE
    assert ilp.m == P * P + 6 * nE + n_lines
    assert ilp.meta["n_lines"] == n_lines
    # projection rows: coefficients 1 and 2 on labels 1 and 2 of the line's pixels, right-hand side
    # the line's sum of the ground truth
    img = ilp.meta["truth"].reshape(-1)
    for k, ln in enumerate(I.tomography_lines(P)):
        cols, coefs, sense, rhs = ilp.row(ilp.m - n_lines + k)
        assert sense == 0 and rhs == int(img[ln].sum())
        assert sorted(cols.tolist()) == sorted((np.concatenate([ln * 3 + 1, ln * 3 + 2])).tolist())
        assert set(coefs.tolist()) <= {1, 2}
    x = I.tomography_truth_point(ilp)
    assert _holds(ilp, x).all()
    assert sorted(ilp.order.tolist()) == list(range(ilp.n))


def test_tomography_truth_has_both_labels_somewhere():
    labs = set()
    for s in range(6):
        labs |= set(np.unique(I.tomography_truth(32, s)).tolist())
    assert labs == {0, 1, 2}


@pytest.mark.parametrize("D", [60, 250, 777])
def test_tracking_structure(D):
    ilp = I.tracking(D, seed=D)
    F = (D + 99) // 100
    assert ilp.m == D and ilp.meta["frames"] == F
    lens = np.diff(ilp.row_ptr)
    assert lens.min() >= 2 and lens.max() <= 2 + 2 + 30
    A = _dense(ilp)
    # appear +1 and disappear -1 in their own detection's row only
    for d in range(D):
        assert A[d, 2 * d] == 1 and A[d, 2 * d + 1] == -1
        assert np.count_nonzero(A[:, 2 * d]) == 1 and np.count_nonzero(A[:, 2 * d + 1]) == 1
    # each link: -1 in its source row, +1 in its target row, nowhere else
    L = A[:, 2 * D:]
    assert np.all(np.count_nonzero(L, axis=0) == 2)
    assert np.all(L.sum(axis=0) == 0)
    assert _holds(ilp, np.zeros(ilp.n, np.int8)).all()
    if F > 1:
        assert ilp.meta["links"] >= _detections_with_out_links(D, F)


def _detections_with_out_links(D, F):
    """Detections outside the last frame (each has at least one out-link)."""
    return (F - 1) * D // F


def test_tomography_zero_unaries_fixed_point():
    """With zero unary costs every min-marginal difference of a unary variable is 0 (its cheapest
    completion in a marginalisation row uses the zero-cost diagonal pair, and projection rows hold
    zero multipliers), so all multipliers on unary incidences stay 0 and the bound stays 0 although
    the ground truth costs more: a fixed point of the coordinate ascent, not the dual optimum."""
    ilp = I.tomography(6, seed=3)
    o = Oracle(ilp)
    tr = np.concatenate([[o.init()], o.iterate(30)])
    assert np.all(tr == 0.0)
    w, var, _, _ = o.structure()
    unary = var < 3 * 36
    assert np.all(o.lam()[unary] == 0.0)
    assert float(ilp.cost @ I.tomography_truth_point(ilp)) > 0


def test_oracle_on_tomography_weak_duality():
    from scipy.optimize import Bounds, LinearConstraint, milp

    ilp = I.tomography(4, seed=3, unary="normal")
    A = _dense(ilp)
    lo = np.where(ilp.sense == 2, ilp.rhs, -np.inf).astype(float)
    hi = np.where(ilp.sense == 1, ilp.rhs, np.inf).astype(float)
    eq = ilp.sense == 0
    lo[eq] = hi[eq] = ilp.rhs[eq]
    res = milp(ilp.cost, constraints=LinearConstraint(A, lo, hi), integrality=np.ones(ilp.n),
               bounds=Bounds(0, 1))
    assert res.status == 0
    x_truth = I.tomography_truth_point(ilp)
    o = Oracle(ilp)
    tr = np.concatenate([[o.init()], o.iterate(40)])
    assert np.all(np.diff(tr) >= -1e-12 * (1 + np.abs(tr[1:])))
    assert tr[-1] <= res.fun + 1e-9
    assert res.fun <= float(ilp.cost @ x_truth) + 1e-9
    assert tr[-1] > tr[0]


def test_oracle_on_tracking_lp_bound():
    """Conservation rows have coefficients +-1: one row plus the box is integral, so every bound
    stays below the LP optimum."""
    from scipy.optimize import linprog

    ilp = I.tracking(220, seed=5)
    A = _dense(ilp)
    res = linprog(ilp.cost, A_eq=A, b_eq=ilp.rhs.astype(float), bounds=[(0, 1)] * ilp.n, method="highs")
    assert res.status == 0
    o = Oracle(ilp)
    tr = np.concatenate([[o.init()], o.iterate(80)])
    assert np.all(np.diff(tr) >= -1e-12 * (1 + np.abs(tr[1:])))
    assert tr[-1] <= res.fun + 1e-7
    assert tr[-1] > tr[0]


def _small_batch():
    return [I.tomography(5, seed=0, unary="normal"), I.tracking(150, seed=1), I.tomography(7, seed=2),
            I.config(1), I.random_ilp(30, 20, kmax=6, seed=4), I.tracking(330, seed=5)]


@pytest.mark.parametrize("order_mode", [0, 1])
def test_batched_plan_is_the_concatenation(order_mode):
    insts = _small_batch()
    probs = [B.Problem.from_ilp(q) for q in insts]
    bp = B.Plan(probs, order_mode=order_mode)
    st = bp.stats
    assert st.n_instances == len(insts)
    plans = [B.Plan(B.Problem.from_ilp(q), order_mode=order_mode) for q in insts]
    sts = [p.stats for p in plans]
    for f in ("n_vars", "n_bdds", "n_nodes", "n_arcs_live", "n_arcs_bot", "n_incidences"):
        assert getattr(st, f) == sum(getattr(s, f) for s in sts), f
    assert st.waves_fwd == max(s.waves_fwd for s in sts)
    assert st.waves_bwd == max(s.waves_bwd for s in sts)
    var_off, row_off, inc_off = bp.instances()
    assert var_off.tolist() == np.cumsum([0] + [q.n for q in insts]).tolist()
    assert row_off.tolist() == np.cumsum([0] + [q.m for q in insts]).tolist()
    assert inc_off.tolist() == np.cumsum([0] + [s.n_incidences for s in sts]).tolist()
    # structure, waves and order: each instance's own, shifted
    w, v, lo, hi = bp.structure()
    wf, wb = bp.waves()
    order = bp.order()
    node_off = np.cumsum([0] + [s.n_nodes for s in sts])
    for k, p in enumerate(plans):
        pw, pv, plo, phi = p.structure()
        a, b = inc_off[k], inc_off[k + 1]
        assert np.array_equal(w[a:b], pw)
        assert np.array_equal(v[a:b], pv + var_off[k])
        assert np.array_equal(lo[node_off[k]:node_off[k + 1]], plo)
        assert np.array_equal(hi[node_off[k]:node_off[k + 1]], phi)
        pf, pb = p.waves()
        assert np.array_equal(wf[var_off[k]:var_off[k + 1]], pf)
        assert np.array_equal(wb[var_off[k]:var_off[k + 1]], pb)
        mine = order[(order >= var_off[k]) & (order < var_off[k + 1])] - var_off[k]
        assert np.array_equal(mine, p.order())


def test_single_plan_has_one_instance():
    p = B.Plan(B.Problem.from_ilp(I.config(1)))
    assert p.stats.n_instances == 1
    v, r, c = p.instances()
    assert v.tolist() == [0, p.stats.n_vars] and r.tolist() == [0, p.stats.n_bdds]
    assert c.tolist() == [0, p.stats.n_incidences]


def test_batch_errors():
    with pytest.raises(B.BddmpError) as e:
        B.bddmp_plan_create_batch([], None)
    assert e.value.code == -1
    with pytest.raises(B.BddmpError) as e:
        B.bddmp_plan_create_batch([None], None)
    assert e.value.code == -1
    # an infeasible row in one instance fails the whole batch with that row's error
    bad = I.from_rows(2, [1.0, 1.0], [([0, 1], [1, 1], 0, 3)])
    with pytest.raises(B.BddmpError) as e:
        B.Plan([B.Problem.from_ilp(I.config(1)), B.Problem.from_ilp(bad)])
    assert e.value.code == -2


def test_batch_config_mix():
    insts = I.batch_config(6, p_range=(4, 9), d_range=(120, 260))
    kinds = [q.meta["kind"] for q in insts]
    assert kinds == ["tomography", "tracking"] * 3
    assert all(4 <= q.meta["P"] <= 9 for q in insts[::2])
    assert all(120 <= q.meta["D"] <= 260 for q in insts[1::2])
    again = I.batch_config(6, p_range=(4, 9), d_range=(120, 260))
    for a, b in zip(insts, again):
        assert np.array_equal(a.col, b.col) and np.array_equal(a.cost, b.cost)


def test_tiling_option():
    q = I.tomography(6, seed=0)
    for good in ("4,16,64,64", "1,1,1,1", "64,32,2,8", "0,0,0,0", "0,16,0,64"):
        B.Plan(B.Problem.from_ilp(q), tiling=good)
    for bad in ("3,16,64,64", "4,16,64", "4,16,64,64,1", "4,16,128,64", "a,b,c,d", "4,16,64,64x", "", "-1,0,0,0"):
        with pytest.raises(B.BddmpError) as e:
            B.Plan(B.Problem.from_ilp(q), tiling=bad)
        assert e.value.code == -1, bad
