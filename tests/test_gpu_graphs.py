"""GPU tests of graph replay: iterate replays one captured iteration; the results must equal host
launches bitwise, over several replays with the program's own eager work and synchronisations in
between, and after a change of the general-layer path (which re-captures)."""
import numpy as np
import pytest

from paper_2009_00481_amd import binding as B
from paper_2009_00481_amd import instances as I

pytestmark = pytest.mark.gpu


def _trace(ilp, graphs: bool, switch_groups: bool = False):
    import torch

    s = B.Solver(B.Plan(B.Problem.from_ilp(ilp), hist_cap=64))
    s.set_graphs(graphs)
    lams, lbs = [], []
    for rep in range(5):
        s.iterate(3)
        # eager work between replays: a bound read (syncs), multipliers out, a torch op on them
        lbs.append(s.lower_bound()[0])
        lam = s.get_lambda()
        lams.append((lam * 1.0).cpu().numpy())
        torch.cuda.synchronize()
        if switch_groups and rep == 2:
            s.set_groups([16, 0, 64, 4])
    m0, m1 = s.min_marginals()
    hist = s.lb_history(64)
    M, x, obj, nv = s.round_primal()
    return lams, lbs, hist, m0.cpu().numpy(), m1.cpu().numpy(), x


@pytest.mark.parametrize("name", ["cfg1", "tomo", "batch"])
def test_graph_replay_equals_host_launches(name):
    if name == "cfg1":
        ilp = I.config(1)
        # runs of iterations here use the wrap-around launch; host launches never do
        assert B.Plan(B.Problem.from_ilp(ilp)).stats.fused_wrap == 1
    elif name == "tomo":
        ilp = I.tomography(14, seed=1, unary="normal")
    else:
        ilp = I.concat([I.tomography(9, seed=2, unary="normal"), I.tracking(260, seed=3), I.config(1)])
    print(f"[graphs] {name}", flush=True)
    a = _trace(ilp, False)
    b = _trace(ilp, True)
    c = _trace(ilp, True, switch_groups=True)
    for r in (b, c):
        for la, lb in zip(a[0], r[0]):
            assert np.array_equal(la, lb)
        assert a[1] == r[1]
        assert np.array_equal(a[2], r[2])
        assert np.array_equal(a[3], r[3]) and np.array_equal(a[4], r[4])
        assert np.array_equal(a[5], r[5])
    # 1 initial bound + 15 iterations recorded in order
    assert a[2].shape == (16,)


def test_history_ring_wraps_with_graphs():
    import torch

    ilp = I.config(1)
    s = B.Solver(B.Plan(B.Problem.from_ilp(ilp), hist_cap=8))
    s.iterate(20)
    h = s.lb_history(8)
    t = B.Solver(B.Plan(B.Problem.from_ilp(ilp), hist_cap=64))
    t.set_graphs(False)
    t.iterate(20)
    ref = t.lb_history(64)
    torch.cuda.synchronize()
    assert np.array_equal(h, ref[-8:])


def test_full_size_replays_equal_host_launches():
    """The benchmark's Potts 256x256x8 workload as bench.py runs it (graph replays, so the
    wrap-around launch inside each run of iterations) against host launches: bitwise equal
    multipliers, bounds and fresh min-marginals after two runs of 10 iterations."""
    import torch

    ilp = I.config(2)
    plan = B.Plan(B.Problem.from_ilp(ilp), hist_cap=64)
    assert plan.stats.fused_turn == 1 and plan.stats.fused_wrap == 1
    out = []
    for graphs in (False, True):
        print(f"[graphs] cfg2 graphs={graphs}", flush=True)
        s = B.Solver(plan)
        s.set_graphs(graphs)
        s.iterate(10)
        s.iterate(10)
        lam = s.get_lambda().cpu().numpy()
        m0, m1 = s.min_marginals()
        hist = s.lb_history(64)
        torch.cuda.synchronize()
        out.append((lam, hist, m0.cpu().numpy(), m1.cpu().numpy()))
        del s
        torch.cuda.empty_cache()
    a, b = out
    assert a[1].shape == (21,)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
