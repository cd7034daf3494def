"""GPU tests of the dataflow launch of the update passes (bddmp_solver_set_launch mode 1): one
launch per pass whose workgroups take tiles by ticket and wait only for the tiles that write what
they read. Every layer runs the same operations in the same order as with one launch per wave, so
every output must be bitwise equal to the wave launches: multipliers, bounds, min-marginals,
rounded primal, per-instance bounds; with graph replay and without; for narrow-only plans, plans
with wide levels, backward waves through the index list, batched plans and split plans; several
chunk sizes. A wait that exceeds its bound is forced from the host (a spin limit of zero) and must
come back as DEVICE from the next bound read, every kernel exiting normally."""
import numpy as np
import pytest

from paper_2009_00481_amd import binding as B
from paper_2009_00481_amd import instances as I

pytestmark = pytest.mark.gpu


def _cases():
    return {
        "cfg1": lambda: [I.config(1)],
        "5sub": lambda: [I.config("5sub")],
        "tomo": lambda: [I.tomography(9, seed=2, unary="normal")],
        "rand_list": lambda: [I.random_ilp(60, 45, kmax=9, cmax=3, seed=7)],
        "batch": lambda: [I.tomography(6, seed=0, unary="normal"), I.tracking(250, seed=1), I.tomography(11, seed=2),
                          I.tracking(180, seed=3), I.config(1), I.random_ilp(40, 30, kmax=8, seed=4)],
        "gm": lambda: [I.graph_matching(60, 60, 5, 400, seed=3)],
    }


def _run(insts, mode, chunk, graphs, T, split=0, wave_align=0):
    import torch

    probs = [B.Problem.from_ilp(q) for q in insts]
    plan = B.Plan(probs if len(probs) > 1 else probs[0], hist_cap=max(64, T + 8), n_intervals=split,
                  wave_align=wave_align)
    s = B.Solver(plan)
    s.set_graphs(graphs)
    s.set_launch(mode, chunk)
    out = {}
    for k in range(3):
        s.iterate(T)
        out[f"lam{k}"] = s.get_lambda().cpu().numpy()
        out[f"lb{k}"] = s.lower_bound()[0]
    out["hist"] = s.lb_history(3 * T + 1)
    m0, m1 = s.min_marginals()
    M, x, obj, nv = s.round_primal()
    out.update(m0=m0.cpu().numpy(), m1=m1.cpu().numpy(), M=M.cpu().numpy(), x=x, obj=obj, nv=nv,
               inst=s.instance_bounds())
    if split:
        out["copy"] = [t.cpu().numpy() for t in s.copy_duals()]
    torch.cuda.synchronize()
    return plan, out


def _same(a, b, what):
    for key in a:
        if key == "copy":
            for x, y in zip(a[key], b[key]):
                assert np.array_equal(x, y), (what, key)
            continue
        assert np.array_equal(np.asarray(a[key]), np.asarray(b[key])), (what, key)


@pytest.mark.parametrize("name", list(_cases()))
def test_dataflow_equals_wave_launches_bitwise(name):
    insts = _cases()[name]()
    T = 4
    print(f"[dataflow] {name}", flush=True)
    plan, ref = _run(insts, 0, 0, True, T)
    assert plan.stats.dataflow == 1
    for graphs in (True, False):
        for chunk in (1, 3):
            _, got = _run(insts, 1, chunk, graphs, T)
            _same(ref, got, (name, graphs, chunk))


def test_dataflow_split_plan_bitwise():
    insts = [I.tomography(10, seed=5, unary="normal"), I.tracking(300, seed=9)]
    plan, ref = _run(insts, 0, 0, True, 3, split=3)
    assert plan.stats.n_cuts > 0
    _, got = _run(insts, 1, 2, True, 3, split=3)
    _same(ref, got, "split")


def test_dataflow_full_size_mrf_bitwise():
    """The 256x256x8 Potts benchmark workload (16 + 16 waves, 75,684 tiles per pass): a few
    iterations with each launch form (waves, dataflow, two-branch waves), graph replay, multipliers
    and bounds bitwise equal."""
    import torch

    ilp = I.config(2)
    plan = B.Plan(B.Problem.from_ilp(ilp))
    print(f"[dataflow full] tiles {plan.stats.fwd_tiles}+{plan.stats.bwd_tiles}", flush=True)
    res = []
    for mode, chunk in ((0, 0), (1, 1), (1, 4), (2, 0)):
        s = B.Solver(plan)
        s.set_launch(mode, chunk)
        s.iterate(3)
        res.append((s.get_lambda().cpu().numpy(), s.lb_history(4)))
        del s
        torch.cuda.empty_cache()
    for lam, hist in res[1:]:
        assert np.array_equal(lam, res[0][0])
        assert np.array_equal(hist, res[0][1])


def test_dataflow_launch_arguments():
    s = B.Solver(B.Plan(B.Problem.from_ilp(I.config(1))))
    for bad in ((5, 0), (-1, 0), (1, -1), (1, 5000)):
        with pytest.raises(B.BddmpError) as e:
            s.set_launch(*bad)
        assert e.value.code == -1
    s.set_launch(1, 2)
    assert s.launch() == (1, 2)
    s.set_launch(0, 0)
    assert s.launch()[0] == 0
    # a variable in more than 256 rows has no dataflow launch
    rows = [([0, k], [1, 1], 1, 1) for k in range(1, 301)]
    big = B.Solver(B.Plan(B.Problem.from_ilp(I.from_rows(301, np.ones(301), rows))))
    assert big.plan.stats.dataflow == 0
    for mode in (1, 2, 3, 4):
        with pytest.raises(B.BddmpError) as e:
            big.set_launch(mode, 0)
        assert e.value.code == -1


def test_dataflow_wait_bound_reports_device_error(monkeypatch):
    """A spin limit of zero makes every wait that finds its dependency unfinished give up at once:
    the kernel still exits, the error word is set, and lower_bound reports DEVICE; a reset clears
    it and a normal launch afterwards matches the wave launches again."""
    import torch

    monkeypatch.setenv("BDDMP_PASS_SPIN_LIMIT", "0")
    ilp = I.config("5sub")
    plan = B.Plan(B.Problem.from_ilp(ilp))
    s = B.Solver(plan)
    s.set_launch(1, 1)
    s.iterate(20)
    try:
        s.lower_bound()
        gave_up = False
    except B.BddmpError as e:
        assert e.code == -6
        gave_up = True
    print(f"[dataflow] a wait gave up: {gave_up}", flush=True)
    monkeypatch.delenv("BDDMP_PASS_SPIN_LIMIT")
    s.set_launch(1, 1)
    s.reset()
    s.iterate(5)
    lam = s.get_lambda().cpu().numpy()
    ref = B.Solver(plan)
    ref.iterate(5)
    assert np.array_equal(lam, ref.get_lambda().cpu().numpy())
    assert s.lower_bound()[0] == ref.lower_bound()[0]
    torch.cuda.synchronize()
