"""GPU tests of the wave-group launches (bddmp_solver_set_launch modes 3 and 4): several consecutive
waves of a pass per launch, one workgroup per tile (mode 3) or per two consecutive tiles (mode 4,
plans whose layers are all narrow), a later wave's tiles waiting only for the flags of the tiles
they read from. Each tile runs the same operations as with one launch per wave, after every tile it
reads from, so every output must be bitwise equal to the wave launches: multipliers, bounds,
min-marginals, rounded primal, per-instance bounds; with graph replay and eager launches; narrow,
wide, list, batched and split plans; 2, 3 and 8 waves per launch and every wave of a pass in one
launch; pairs of tiles inside one wave and across a wave boundary (the second tile reading from
the first); switching launch forms between calls. A wait that exceeds its bound is forced from the
host (a spin limit of zero) and must come back as DEVICE from the next bound read, every kernel
exiting normally."""
import numpy as np
import pytest

from paper_2009_00481_amd import binding as B
from paper_2009_00481_amd import instances as I
from test_gpu_dataflow import _cases, _run, _same

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", list(_cases()))
def test_wave_groups_equal_wave_launches_bitwise(name):
    insts = _cases()[name]()
    T = 4
    print(f"[wave groups] {name}", flush=True)
    plan, ref = _run(insts, 0, 0, True, T)
    for graphs, g in ((True, 2), (True, 3), (False, 8), (True, 4096)):
        _, got = _run(insts, 3, g, graphs, T)
        _same(ref, got, (name, graphs, g))


def _narrow_cases():
    c = _cases()
    return {"cfg1": c["cfg1"], "5sub": c["5sub"], "gm_list": c["gm"],
            "narrow_batch": lambda: [I.config(1), I.graph_matching(40, 40, 4, 200, seed=5), I.config("5sub")]}


@pytest.mark.parametrize("name", list(_narrow_cases()))
def test_two_tile_wave_groups_equal_wave_launches_bitwise(name):
    """Mode 4 on plans whose layers are all narrow (contiguous and listed backward waves, a batch),
    earliest and latest waves: small waves make many pairs straddle a wave boundary, so both the
    paired path and the one-after-the-other path run."""
    insts = _narrow_cases()[name]()
    T = 4
    print(f"[two-tile wave groups] {name}", flush=True)
    plan, ref = _run(insts, 0, 0, True, T)
    assert plan.stats.max_width <= 2
    for align, graphs, g in ((0, True, 2), (0, True, 3), (0, False, 8), (0, True, 4096), (1, True, 4096)):
        _, got = _run(insts, 4, g, graphs, T, wave_align=align)
        _same(ref, got, (name, align, graphs, g))


def test_two_tile_wave_groups_reject_general_plans():
    import torch

    plan = B.Plan(B.Problem.from_ilp(I.tomography(9, seed=2, unary="normal")))
    assert plan.stats.max_width > 2
    s = B.Solver(plan)
    with pytest.raises(B.BddmpError) as e:
        s.set_launch(4, 8)
    assert e.value.code == -1
    assert s.launch()[0] == 0
    torch.cuda.synchronize()


def test_latest_waves_equal_earliest_waves_bitwise():
    """A batch planned with every variable in its latest wave (wave_align 1), with one launch per
    wave and with wave groups, against the default plan's wave launches: the same multipliers,
    bounds, min-marginals, rounded primal and instance bounds."""
    insts = _cases()["batch"]()
    _, ref = _run(insts, 0, 0, True, 4)
    for mode, g in ((0, 0), (3, 4), (3, 256), (3, 4096)):
        _, got = _run(insts, mode, g, True, 4, wave_align=1)
        _same(ref, got, ("latest waves", mode, g))


def test_wave_groups_split_plan_bitwise():
    insts = [I.tomography(10, seed=5, unary="normal"), I.tracking(300, seed=9)]
    plan, ref = _run(insts, 0, 0, True, 3, split=3)
    assert plan.stats.n_cuts > 0
    _, got = _run(insts, 3, 4, True, 3, split=3)
    _same(ref, got, "split")


def test_wave_groups_full_size_mrf_bitwise():
    """The 256x256x8 Potts benchmark workload with 2, 4 and 8 waves per launch and with every wave of
    a pass in one launch, one and two tiles per workgroup: multipliers and bounds after 3 iterations
    bitwise those of the wave launches."""
    import torch

    plan = B.Plan(B.Problem.from_ilp(I.config(2)))
    res = []
    for mode, g in ((0, 0), (3, 2), (3, 4), (3, 8), (3, 4096), (4, 2), (4, 8), (4, 4096)):
        print(f"[wave groups full] mode {mode} waves {g}", flush=True)
        s = B.Solver(plan)
        s.set_launch(mode, g)
        s.iterate(3)
        res.append((s.get_lambda().cpu().numpy(), s.lb_history(4)))
        del s
        torch.cuda.empty_cache()
    for lam, hist in res[1:]:
        assert np.array_equal(lam, res[0][0])
        assert np.array_equal(hist, res[0][1])


def test_wave_groups_switching_and_arguments():
    import torch

    plan = B.Plan(B.Problem.from_ilp(I.config("5sub")))
    a, b = B.Solver(plan), B.Solver(plan)
    for mode, g in ((3, 2), (1, 1), (4, 3), (3, 4), (0, 0), (2, 0), (4, 0), (3, 0)):
        b.set_launch(mode, g)
        assert b.launch()[0] == mode
        if mode in (3, 4):
            assert b.launch()[1] == (g or 4)
        a.iterate(3)
        b.iterate(3)
        assert np.array_equal(a.get_lambda().cpu().numpy(), b.get_lambda().cpu().numpy()), (mode, g)
    assert np.array_equal(a.lb_history(19), b.lb_history(19))
    for mode, g in ((3, 4097), (4, 4097), (5, 0), (-1, 0)):
        with pytest.raises(B.BddmpError) as e:
            b.set_launch(mode, g)
        assert e.value.code == -1
    torch.cuda.synchronize()


@pytest.mark.parametrize("mode", [3, 4])
def test_wave_groups_wait_bound_reports_device_error(monkeypatch, mode):
    """A spin limit of zero makes every wait that finds its dependency unfinished give up at once:
    the kernel still exits, the error word is set, and lower_bound reports DEVICE (or, if no wait
    found its dependency unfinished, the results are exact); a reset clears it."""
    import torch

    monkeypatch.setenv("BDDMP_PASS_SPIN_LIMIT", "0")
    plan = B.Plan(B.Problem.from_ilp(I.config(5)))
    s = B.Solver(plan)
    s.set_launch(mode, 8)
    s.iterate(10)
    ref = B.Solver(plan)
    ref.iterate(10)
    try:
        lb = s.lower_bound()[0]
        gave_up = False
        assert lb == ref.lower_bound()[0]
    except B.BddmpError as e:
        assert e.code == -6
        gave_up = True
    print(f"[wave groups] mode {mode}: a wait gave up: {gave_up}", flush=True)
    monkeypatch.delenv("BDDMP_PASS_SPIN_LIMIT")
    s.set_launch(mode, 8)
    s.reset()
    ref.reset()
    s.iterate(5)
    ref.iterate(5)
    assert np.array_equal(s.get_lambda().cpu().numpy(), ref.get_lambda().cpu().numpy())
    assert s.lower_bound()[0] == ref.lower_bound()[0]
    torch.cuda.synchronize()


@pytest.mark.parametrize("case", ["no_rows", "degenerate_rows", "one_row", "one_variable"])
def test_launch_forms_on_degenerate_plans(case):
    """Plans with no rows, with empty and single-level rows and a variable in no row, with one row,
    and with one variable: every launch form (waves, dataflow, two-branch, wave groups, and latest
    waves) runs and gives the wave launches' multipliers and bounds bitwise."""
    import torch

    ilps = {
        "no_rows": lambda: I.from_rows(4, np.array([1.0, -2.0, 0.5, -0.25]), []),
        "degenerate_rows": lambda: I.from_rows(
            5, np.array([-1.0, -0.5, 0.75, 0.25, -3.0]),
            [([], [], 1, 0), ([0, 1], [1, 1], 1, 1), ([2], [1], 1, 0), ([3], [2], 2, 1), ([1, 3], [1, -1], 1, 0)]),
        "one_row": lambda: I.from_rows(3, np.array([0.5, -1.0, 0.25]), [([0, 1, 2], [1, 1, 1], 0, 1)]),
        "one_variable": lambda: I.from_rows(1, np.array([-0.5]), [([0], [1], 1, 1)]),
    }
    ilp = ilps[case]()
    res = []
    for align, mode, g in ((0, 0, 0), (0, 1, 1), (0, 2, 0), (0, 3, 2), (1, 3, 8), (1, 0, 0), (0, 4, 2), (1, 4, 8)):
        plan = B.Plan(B.Problem.from_ilp(ilp), wave_align=align)
        s = B.Solver(plan)
        if mode == 4 and plan.stats.max_width > 2:
            continue
        if mode:
            s.set_launch(mode, g)
        for graphs in (True, False):
            s.set_graphs(graphs)
            s.iterate(3)
        res.append((s.get_lambda().cpu().numpy(), s.lb_history(7), s.lower_bound()[0]))
        torch.cuda.synchronize()
    for lam, hist, lb in res[1:]:
        assert np.array_equal(lam, res[0][0]) and np.array_equal(hist, res[0][1]) and lb == res[0][2], case
