"""Pins of the oracle's sub-BDD split (Sec. 6, Alg. "Parallel min-marginal averaging").

What fixes the values independently of the oracle's code:
- the whole algorithm by enumeration in exact rationals (``BruteSplitDBCA``: sub-BDDs as path lists
  of truth-table diagrams): bounds, multipliers, copy duals and min-marginals per iteration;
- Prop. "correctness-parallel": the bound never decreases, and the copy duals stay feasible
  (mu + mu_bar <= 0 per pair);
- the bound stays below the ILP optimum (enumeration of {0,1}^n);
- one row split into pieces, with gamma = 1/2, climbs to the row's minimum (its multipliers are
  fixed, so the copy duals alone close the gap between the pieces); the split bound with all duals
  0 is the sum of the pieces' minima;
- K = 1 is the unsplit algorithm.
"""
from fractions import Fraction

import numpy as np
import pytest

import bruteforce as bf
from oracle import Oracle
from paper_2009_00481_amd import binding as B
from paper_2009_00481_amd import instances as I


def _small(seed):
    return I.random_ilp(10, 7, kmin=2, kmax=6, cmax=3, seed=seed)


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("K", [2, 3, 5])
def test_oracle_equals_enumeration(seed, K):
    ilp = _small(seed)
    br = bf.BruteSplitDBCA(ilp, K)
    o = Oracle(ilp, split=K)
    assert o.init() == pytest.approx(float(br.lb()), abs=1e-12)
    for _ in range(3):
        tr = o.iterate(2)
        tb = br.iterate(2)
        np.testing.assert_allclose(tr, [float(v) for v in tb], rtol=0, atol=1e-12)
    np.testing.assert_allclose(o.lam(), [float(v) for v in br.base.lam_canonical()], rtol=0, atol=1e-12)
    cd = o.copy_duals()
    for q in range(len(cd["mu"])):
        key = (int(cd["row"][q]), int(cd["level"][q]), int(cd["node"][q]), int(cd["label"][q]))
        assert cd["mu"][q] == pytest.approx(float(br.mue[key]), abs=1e-12)
        assert cd["mu_bar"][q] == pytest.approx(float(br.mux[key]), abs=1e-12)
    assert len(cd["mu"]) == len(br.mue)
    m0, m1 = o.min_marginals()
    q = 0
    for j, (vs, _) in enumerate(br.base.rows):
        for v in vs:
            for beta, got in ((0, m0[q]), (1, m1[q])):
                want = br.mm(j, v, beta)
                assert (np.isinf(got) and want == bf.INF) or got == pytest.approx(float(want), abs=1e-12)
            q += 1


def test_intervals_follow_node_counts():
    for ilp in (I.config(1), I.random_ilp(40, 30, kmax=7, seed=3), I.tomography(6, seed=1, unary="normal")):
        o = Oracle(ilp)
        w, var, _, _ = o.structure()
        cnt = np.bincount(var, weights=w, minlength=ilp.n)
        for K in (2, 3, 7):
            s = Oracle(ilp, split=K)
            k, ncut, npair, intv = s.split_info()
            assert k == K
            seq = intv[np.asarray(ilp.order)]
            assert np.all(np.diff(seq) >= 0) and seq.min() >= 0 and seq.max() < K
            # interval p holds the variables whose preceding node count lies in [p N / K, (p+1) N / K)
            before = np.concatenate([[0], np.cumsum(cnt[np.asarray(ilp.order)])[:-1]])
            N = cnt.sum()
            assert np.all(before * K >= seq * N) and np.all(before * K < (seq + 1) * N)
            # the library cuts the same levels
            plan = B.Plan(B.Problem.from_ilp(ilp), n_intervals=K)
            assert (plan.stats.n_cuts, plan.stats.n_copy_pairs) == (ncut, npair)
            assert plan.stats.waves_fwd <= B.Plan(B.Problem.from_ilp(ilp)).stats.waves_fwd


def test_k1_is_the_unsplit_algorithm():
    ilp = I.config(1)
    a, b = Oracle(ilp), Oracle(ilp, split=1)
    assert a.init() == b.init()
    assert np.array_equal(a.iterate(10), b.iterate(10))
    assert np.array_equal(a.lam(), b.lam())


@pytest.mark.parametrize("K", [2, 3, 4, 6])
def test_one_row_climbs_to_its_minimum(K):
    rng = np.random.default_rng(K)
    for _ in range(12):
        k = int(rng.integers(5, 11))
        coefs = rng.integers(-3, 4, size=k)
        coefs[coefs == 0] = 1
        rhs, sense = int(rng.integers(-2, 4)), int(rng.integers(0, 3))
        X = bf.feasible_set(list(coefs), sense, rhs)
        if not X:
            continue
        c = rng.standard_normal(k)
        best = min(float(np.dot(c, x)) for x in X)
        ilp = I.from_rows(k, c, [(list(range(k)), list(coefs), sense, rhs)])
        o = Oracle(ilp, split=K, gamma=0.5)
        tr = np.concatenate([[o.init()], o.iterate(300)])
        assert np.all(np.diff(tr) >= -1e-12)
        assert tr.max() <= best + 1e-12
        assert tr[-1] == pytest.approx(best, abs=1e-9)


@pytest.mark.parametrize("gamma", [0.5, 1.0, 0.25])
def test_bound_is_monotone_and_duals_feasible(gamma):
    """Prop. "correctness-parallel": non-decreasing bound; mu + mu_bar <= 0 for every pair."""
    cases = [I.config(1), I.random_ilp(40, 30, kmax=7, cmax=3, seed=5), I.graph_matching(25, 25, 4, 30, seed=2),
             I.tracking(150, seed=4), I.tomography(6, seed=2, unary="normal")]
    for ilp in cases:
        for K in (2, 4):
            o = Oracle(ilp, split=K, gamma=gamma)
            prev = o.init()
            for _ in range(12):
                lb = o.iterate(1)[0]
                assert lb >= prev - 1e-10 * (1 + abs(lb)), (ilp.name, K)
                prev = lb
                cd = o.copy_duals()
                assert np.all(cd["mu"] + cd["mu_bar"] <= 1e-12), (ilp.name, K)


def test_bound_stays_below_the_ilp_optimum():
    for seed in range(8):
        ilp = I.random_ilp(14, 9, kmin=2, kmax=6, cmax=3, seed=seed)
        opt = bf.ilp_optimum(ilp)
        if opt is None:
            continue
        for K in (2, 3):
            o = Oracle(ilp, split=K)
            tr = np.concatenate([[o.init()], o.iterate(40)])
            assert tr.max() <= opt + 1e-9


def test_float_mirror_tracks_fp64():
    ilp = I.config(1)
    a, b = Oracle(ilp, split=3), Oracle(ilp, precision="f32", split=3)
    ta = np.concatenate([[a.init()], a.iterate(30)])
    tb = np.concatenate([[b.init()], b.iterate(30)])
    np.testing.assert_allclose(tb, ta, rtol=1e-4)


def test_split_rejects_smoothing_and_bad_arguments():
    from oracle import OracleError

    o = Oracle(I.config(1), split=2)
    with pytest.raises(OracleError):
        o.smooth_init(0.5)
    with pytest.raises(OracleError):
        Oracle(I.config(1), split=2, gamma=1.5)
    for bad in (dict(n_intervals=-1), dict(n_intervals=2, split_gamma=1.5), dict(n_intervals=2, split_gamma=-0.5)):
        with pytest.raises(B.BddmpError) as e:
            B.Plan(B.Problem.from_ilp(I.config(1)), **bad)
        assert e.value.code == -1


def test_split_of_the_figure():
    """Fig. "split-bdd": the diagram of x1 + x3 + x7 = 1 (Fig. "bdd") with x1, x3 in one interval and
    x7 in the next: three copy-arc pairs, the first piece's paths end with the copy-arcs of
    (x1, x3) = (0, 0), (0, 1), (1, 0) and the second piece's paths start with the matching arcs,
    followed by x7 = 1, 0, 0. Level 1 numbers the node after x1 = 0 first (breadth-first order)."""
    ilp = I.from_rows(3, [0.2, -0.4, 0.7], [([0, 1, 2], [1, 1, 1], 0, 1)])
    # node counts 1, 2, 2: with K = 2 the variables before 2 and 6/5 split as (x1, x3 | x7)
    o = Oracle(ilp, split=2)
    k, ncut, npair, intv = o.split_info()
    assert (ncut, npair) == (1, 3) and list(intv) == [0, 0, 1]
    cd = o.copy_duals()
    assert list(zip(cd["row"], cd["level"], cd["node"], cd["label"])) == [(0, 1, 0, 0), (0, 1, 0, 1), (0, 1, 1, 0)]
    br = bf.BruteSplitDBCA(ilp, 2)
    (_, _, pa), (_, _, pb) = br.segs[0]
    assert sorted(pa) == [(None, [0, 0], (1, 0, 0)), (None, [0, 1], (1, 0, 1)), (None, [1, 0], (1, 1, 0))]
    assert sorted(pb) == [((1, 0, 0), [1], None), ((1, 0, 1), [0], None), ((1, 1, 0), [0], None)]
    plan = B.Plan(B.Problem.from_ilp(ilp), n_intervals=2)
    assert (plan.stats.n_cuts, plan.stats.n_copy_pairs) == (1, 3)
    # with every dual 0 the bound is the sum of the pieces' minima: min(0, -0.4, 0.2) + min(0.7, 0, 0)
    assert o.init() == pytest.approx(-0.4)
    # here the pieces' minima already agree with the row's minimum (x3 = 1), so the bound stays there
    assert o.iterate(50)[-1] == pytest.approx(-0.4, abs=1e-9)
