"""Host half of the library on the CPU: symbols, BDD structure against the oracle (bit-exact), the
dependency waves, the processing order and the error codes. No device calls."""
import os
import re

import numpy as np
import pytest

from oracle import Oracle
from paper_2009_00481_amd import binding as B
from paper_2009_00481_amd import instances as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _plan(ilp, **kw):
    prob = B.Problem.from_ilp(ilp)
    return B.Plan(prob, **kw)


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "bddmp.h")).read()
    declared = set(re.findall(r"\b(bddmp_[a-z_]+)\s*\(", hdr))
    assert declared == set(B.SIGNATURES), declared ^ set(B.SIGNATURES)
    L = B.lib()
    for name in declared:
        assert hasattr(L, name), name
    assert B.bddmp_version() >= 10000


def _same_structure(ilp, **kw):
    pl = _plan(ilp, **kw)
    o = Oracle(ilp)
    st = pl.stats
    assert (st.n_vars, st.n_bdds, st.n_nodes, st.n_incidences, st.n_arcs_live) == \
        (o.n, o.m, o.n_nodes, o.n_incidences, o.n_live_arcs)
    got = pl.structure()
    want = o.structure()
    for g, w, name in zip(got, want, ("level_width", "level_var", "lo", "hi")):
        assert np.array_equal(g, w), name
    return pl


@pytest.mark.parametrize("seed", range(40))
def test_structure_bit_exact_random(seed):
    ilp = I.random_ilp(30, 25, kmin=1, kmax=12, cmax=3, seed=seed)
    _same_structure(ilp)


def test_structure_bit_exact_configs():
    _same_structure(I.config(1))
    _same_structure(I.config("5sub"))
    _same_structure(I.graph_matching(300, 300, 10, 3000, seed=1))
    _same_structure(I.potts_grid(5, 7, 6, seed=2))


def test_structure_wide_rows():
    # long rows with coefficients up to 3: wide levels (the tomography-like regime)
    rng = np.random.default_rng(7)
    rows = []
    for j in range(6):
        k = 40
        vs = rng.choice(60, size=k, replace=False)
        cs = rng.integers(1, 4, size=k)
        rows.append((vs, cs, j % 3, int(cs.sum() // 2)))
    ilp = I.from_rows(60, rng.standard_normal(60), rows, order=rng.permutation(60))
    pl = _same_structure(ilp)
    assert pl.stats.max_width > 4


def test_potts_closed_forms():
    for (H, W, L) in ((8, 8, 3), (16, 16, 4), (5, 9, 8)):
        c = I.potts_counts(H, W, L)
        pl = _plan(I.potts_grid(H, W, L, seed=0))
        st = pl.stats
        nV, m_edge = H * W, c["n_edges"] * 2 * L
        assert (st.n_vars, st.n_bdds, st.n_incidences, st.n_nodes) == (c["n"], c["m"], c["incidences"], c["nodes"])
        assert st.n_arcs_live == nV * (3 * L - 2) + m_edge * (3 * L + 1)
        # unary x[u,l] runs in wave l+1, pairwise y[e,l,k] in wave l+k+2: 2L waves per pass
        assert st.waves_fwd == 2 * L and st.waves_bwd == 2 * L
        assert st.bwd_contiguous == 1
        assert st.n_shapes == 2


def _check_waves(ilp, pl):
    order = pl.order()
    rank = np.empty(ilp.n, np.int64)
    rank[order] = np.arange(ilp.n)
    wf, wb = pl.waves()
    rows = []
    for j in range(ilp.m):
        c, a, _, _ = ilp.row(j)
        vs = [int(v) for v in c[a != 0]]
        vs.sort(key=lambda v: rank[v])
        rows.append(vs)
    need_f = np.zeros(ilp.n, np.int64)
    need_b = np.zeros(ilp.n, np.int64)
    inrow = np.zeros(ilp.n, bool)
    for vs in rows:
        for t, v in enumerate(vs):
            inrow[v] = True
            if t > 0:
                need_f[v] = max(need_f[v], wf[vs[t - 1]])
            if t + 1 < len(vs):
                need_b[v] = max(need_b[v], wb[vs[t + 1]])
        # one row never has two variables in one wave
        assert len({wf[v] for v in vs}) == len(vs)
        assert len({wb[v] for v in vs}) == len(vs)
    assert np.array_equal(wf[inrow], need_f[inrow] + 1)
    assert np.array_equal(wb[inrow], need_b[inrow] + 1)
    assert np.all(wf[~inrow] == 0) and np.all(wb[~inrow] == 0)
    assert pl.stats.waves_fwd == (wf.max() if ilp.n else 0)


@pytest.mark.parametrize("seed", range(10))
def test_waves_are_the_dependency_levels(seed):
    ilp = I.random_ilp(40, 30, kmax=6, seed=seed)
    _check_waves(ilp, _plan(ilp))


def _check_latest_waves(ilp, asap, alap):
    """The latest waves (wave_align 1) against the earliest ones of the same problem: forward wave
    D + 1 - (earliest backward wave) and backward wave D + 1 - (earliest forward wave), every
    variable after each of its row predecessors (forward) or successors (backward), each row's
    variables in distinct waves."""
    wf0, wb0 = asap.waves()
    wf1, wb1 = alap.waves()
    D = asap.stats.waves_fwd
    assert alap.stats.waves_fwd == D and alap.stats.waves_bwd == D
    inrow = wf0 > 0
    assert np.array_equal(wf1[inrow], D + 1 - wb0[inrow]) and np.array_equal(wb1[inrow], D + 1 - wf0[inrow])
    assert np.all(wf1[~inrow] == 0) and np.all(wb1[~inrow] == 0)
    order = asap.order()
    rank = np.empty(ilp.n, np.int64)
    rank[order] = np.arange(ilp.n)
    for j in range(ilp.m):
        c, a, _, _ = ilp.row(j)
        vs = sorted((int(v) for v in c[a != 0]), key=lambda v: rank[v])
        for t in range(1, len(vs)):
            assert wf1[vs[t]] > wf1[vs[t - 1]] and wb1[vs[t - 1]] > wb1[vs[t]]
    # no wave is empty
    assert set(wf1[inrow].tolist()) == set(range(1, D + 1)) and set(wb1[inrow].tolist()) == set(range(1, D + 1))


@pytest.mark.parametrize("seed", range(5))
def test_latest_waves_random(seed):
    ilp = I.random_ilp(40, 30, kmax=6, seed=seed)
    _check_latest_waves(ilp, _plan(ilp), _plan(ilp, wave_align=1))


def test_latest_waves_batch_start_shorter_instances_late():
    """In a batch, an instance with a shorter longest chain than the batch's has its first
    variables in a later forward wave than 1; the deepest instance keeps wave 1."""
    qs = [I.tracking(250, seed=1), I.config(1), I.tomography(6, seed=0)]
    asap = B.Plan([B.Problem.from_ilp(q) for q in qs])
    alap = B.Plan([B.Problem.from_ilp(q) for q in qs], wave_align=1)
    _check_latest_waves(I.concat(qs), asap, alap)
    voff, _, _ = alap.instances()
    wf1, _ = alap.waves()
    first = [int(wf1[voff[k]:voff[k + 1]][wf1[voff[k]:voff[k + 1]] > 0].min()) for k in range(len(qs))]
    assert min(first) == 1 and max(first) > 1


def test_waves_configs():
    for ilp in (I.config(1), I.graph_matching(300, 300, 10, 3000, seed=1)):
        _check_waves(ilp, _plan(ilp))


def test_turnaround_fusion():
    """A variable of the last forward wave is last in each of its rows, so it is in the first
    backward wave; the plan runs the two waves as one launch only when the two sets are equal (and
    there is no split). Potts grids have this shape, graph matching and split plans do not."""
    for ilp in [I.config(1), I.config(5), I.graph_matching(300, 300, 10, 3000, seed=1)] + \
            [I.random_ilp(40, 30, kmax=6, seed=s) for s in range(6)]:
        pl = _plan(ilp)
        wf, wb = pl.waves()
        last_f = set(np.flatnonzero(wf == pl.stats.waves_fwd).tolist())
        first_b = set(np.flatnonzero(wb == 1).tolist())
        assert last_f <= first_b
        if pl.stats.fused_turn:
            assert last_f == first_b
        # mirror image: a variable of the first forward wave is first in its rows, so in the last
        # backward wave; the wrap-around launch needs the two sets equal
        first_f = set(np.flatnonzero(wf == 1).tolist())
        last_b = set(np.flatnonzero(wb == pl.stats.waves_bwd).tolist())
        assert last_b <= first_f or pl.stats.waves_bwd == 0
        if pl.stats.fused_wrap:
            assert first_f == last_b and pl.stats.waves_fwd > 1
    for c in (1, 5):
        st = _plan(I.config(c)).stats
        assert st.fused_turn == 1 and st.fused_wrap == 1
    st = _plan(I.graph_matching(300, 300, 10, 3000, seed=1)).stats
    assert st.fused_turn == 0 and st.fused_wrap == 0
    st = B.Plan(B.Problem.from_ilp(I.config(1)), n_intervals=2).stats
    assert st.fused_turn == 0 and st.fused_wrap == 0


def test_greedy_colour_order_matches_generator():
    ilp = I.graph_matching(200, 200, 10, 2000, seed=3)
    prob = B.Problem.from_ilp(ilp, order=False)
    pl = B.Plan(prob, order_mode=1)
    assert np.array_equal(pl.order(), ilp.order)
    # the colour order makes the waves about as many as the colours
    assert pl.stats.waves_fwd <= 60


def test_given_order_is_used():
    ilp = I.random_ilp(20, 10, seed=1)
    pl = _plan(ilp)
    assert np.array_equal(pl.order(), ilp.order)


def test_errors():
    with pytest.raises(B.BddmpError) as e:
        _plan(I.from_rows(3, np.zeros(3), [([0, 1], [1, 1], 0, 3)]))
    assert e.value.code == -2
    with pytest.raises(B.BddmpError) as e:
        _plan(I.from_rows(3, np.zeros(3), [([0, 0], [1, 1], 0, 1)]))
    assert e.value.code == -1
    with pytest.raises(B.BddmpError) as e:
        _plan(I.from_rows(2, np.ones(2), [([0, 1], [1, 1], 0, 2), ([0], [1], 1, 0)]))
    assert e.value.code == -5
    with pytest.raises(B.BddmpError) as e:
        _plan(I.config(1), node_budget=1000)
    assert e.value.code == -3
    for bad in (-1, 2):
        with pytest.raises(B.BddmpError) as e:
            _plan(I.config(1), wave_align=bad)
        assert e.value.code == -1
    p = B.Problem(3, np.zeros(3))
    with pytest.raises(B.BddmpError) as e:
        p.set_order([0, 0, 1])
    assert e.value.code == -1
    with pytest.raises(B.BddmpError) as e:
        p.add_rows([0, 1], [5], [1], [0], [1])
    assert e.value.code == -1
    with pytest.raises(B.BddmpError) as e:
        p.add_rows([0, 1], [1], [1], [3], [1])
    assert e.value.code == -1


def test_empty_and_degenerate_plans():
    # no rows at all
    pl = _plan(I.from_rows(4, np.array([1.0, -2.0, 0.5, -0.5]), []))
    assert pl.stats.n_incidences == 0 and pl.stats.waves_fwd == 0
    # a row without variables that holds is kept as an empty diagram
    pl = _plan(I.from_rows(2, np.zeros(2), [([], [], 1, 0), ([0, 1], [1, 1], 1, 1)]))
    assert pl.stats.n_bdds == 2 and pl.stats.n_incidences == 2
    # zero coefficients are dropped from I_j
    pl = _plan(I.from_rows(3, np.zeros(3), [([0, 1, 2], [1, 0, 1], 0, 1)]))
    assert pl.stats.n_incidences == 2


def test_plan_digest_is_reproducible():
    """The planner fills the layers' arcs and meta words and checks the layout on several host
    threads over layer ranges; the same problems and options must give the same plan bytes on every
    build (a batch with general levels, large enough for several threads), other options other
    bytes."""
    probs = [B.Problem.from_ilp(q) for q in I.batch_config(4, p_range=(40, 64), d_range=(200, 600))]
    plan = B.Plan(probs, wave_align=1)
    assert plan.stats.n_incidences > 4 * 65536 and plan.stats.max_width > 2
    d = plan.digest()
    for _ in range(3):
        assert B.Plan(probs, wave_align=1).digest() == d
    assert B.Plan(probs, wave_align=0).digest() != d
    assert B.Plan(probs[:3], wave_align=1).digest() != d


def test_plan_digest_arguments():
    with pytest.raises(B.BddmpError) as e:
        B._check(B.lib().bddmp_plan_digest(None, None))
    assert e.value.code == -1
