"""GPU tests of the two-branch wave launches (bddmp_solver_set_launch mode 2): every wave split in
an A part, launched in order on the solver's stream, and a B part, launched in order on a second
stream after the A part of the latest wave it reads from. Each tile runs the same operations as
with one launch per wave, after every tile it reads from, so every output must be bitwise equal to
the wave launches: multipliers, bounds, min-marginals, rounded primal, per-instance bounds; with
graph replay (the two chains as parallel graph branches) and with eager launches; narrow-only,
wide, list, batched and split plans; switching launch forms between calls."""
import numpy as np
import pytest

from paper_2009_00481_amd import binding as B
from paper_2009_00481_amd import instances as I
from test_gpu_dataflow import _cases, _run, _same

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", list(_cases()))
def test_two_branch_equals_wave_launches_bitwise(name):
    insts = _cases()[name]()
    T = 4
    print(f"[two-branch] {name}", flush=True)
    plan, ref = _run(insts, 0, 0, True, T)
    for graphs in (True, False):
        _, got = _run(insts, 2, 0, graphs, T)
        _same(ref, got, (name, graphs))


def test_two_branch_split_plan_bitwise():
    insts = [I.tomography(10, seed=5, unary="normal"), I.tracking(300, seed=9)]
    plan, ref = _run(insts, 0, 0, True, 3, split=3)
    assert plan.stats.n_cuts > 0
    _, got = _run(insts, 2, 0, True, 3, split=3)
    _same(ref, got, "split")


def test_two_branch_switching_forms_between_calls():
    """Iterations in mode 2, then 0, then 1, then 2 again continue one run: the same state as
    mode 0 throughout (graphs are re-captured at each switch)."""
    import torch

    plan = B.Plan(B.Problem.from_ilp(I.config("5sub")))
    a, b = B.Solver(plan), B.Solver(plan)
    for mode in (2, 0, 1, 2):
        b.set_launch(mode, 0)
        assert b.launch()[0] == mode
        a.iterate(3)
        b.iterate(3)
        assert np.array_equal(a.get_lambda().cpu().numpy(), b.get_lambda().cpu().numpy()), mode
    assert np.array_equal(a.lb_history(13), b.lb_history(13))
    torch.cuda.synchronize()


def test_two_branch_kernel_timing_entry_point():
    """The timing call runs 2 eager two-branch iterations bracketed by events on the solver's
    stream (counting the launched parts), then 2 replayed ones; the state advances by 4."""
    plan = B.Plan(B.Problem.from_ilp(I.config(5)))
    s, ref = B.Solver(plan), B.Solver(plan)
    s.set_launch(2, 0)
    kt = s.time_kernels(2)
    beg, mid, _ = plan.wave_split(0)
    parts = int(np.sum(mid > beg[:-1]) + np.sum(beg[1:] > mid))
    assert kt["fwd_launches"] == 2 * parts
    assert kt["fwd_ms"] > 0 and kt["bwd_ms"] > 0
    ref.iterate(4)
    assert np.array_equal(s.get_lambda().cpu().numpy(), ref.get_lambda().cpu().numpy())
