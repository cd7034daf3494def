"""GPU tests of the batched plan: one schedule for several independent instances must give each
instance bitwise the results of its own plan, and those results must match the oracle run on the
instance alone."""
import numpy as np
import pytest

from parity import assert_incidence_close, incidence_scale
from oracle import Oracle
from paper_2009_00481_amd import binding as B
from paper_2009_00481_amd import instances as I

pytestmark = pytest.mark.gpu


def _batch():
    return [I.tomography(6, seed=0, unary="normal"), I.tracking(250, seed=1), I.tomography(11, seed=2),
            I.tracking(180, seed=3), I.config(1), I.random_ilp(40, 30, kmax=8, seed=4),
            I.tomography(9, seed=6)]


def _outputs(s):
    import torch

    lam = s.get_lambda().cpu().numpy()
    m0, m1 = s.min_marginals()
    M, x, obj, nviol = s.round_primal()
    inst = s.instance_bounds()
    torch.cuda.synchronize()
    return dict(lam=lam, m0=m0.cpu().numpy(), m1=m1.cpu().numpy(), M=M.cpu().numpy(), x=x, inst=inst)


@pytest.mark.parametrize("order_mode", [0, 1])
def test_batched_equals_each_plain_plan_bitwise(order_mode):
    insts = _batch()
    T = 25
    print(f"[batch] order_mode={order_mode} instances={len(insts)} T={T}", flush=True)
    bp = B.Plan([B.Problem.from_ilp(q) for q in insts], order_mode=order_mode)
    bs = B.Solver(bp)
    bs.iterate(T)
    got = _outputs(bs)
    hist = bs.lb_history(T + 1)
    var_off, row_off, inc_off = bp.instances()
    total = np.zeros(T + 1)
    for k, q in enumerate(insts):
        plan = B.Plan(B.Problem.from_ilp(q), order_mode=order_mode)
        s = B.Solver(plan)
        s.iterate(T)
        ref = _outputs(s)
        total += s.lb_history(T + 1)
        a, b = inc_off[k], inc_off[k + 1]
        va, vb = var_off[k], var_off[k + 1]
        assert np.array_equal(got["lam"][a:b], ref["lam"]), k
        assert np.array_equal(got["m0"][a:b], ref["m0"]), k
        assert np.array_equal(got["m1"][a:b], ref["m1"]), k
        assert np.array_equal(got["M"][va:vb], ref["M"]), k
        assert np.array_equal(got["x"][va:vb], ref["x"]), k
        assert got["inst"][k] == ref["inst"][0], k
    # the batch's bound is the sum of the instances' bounds (fp64 sums in another order)
    np.testing.assert_allclose(hist, total, rtol=1e-12, atol=1e-9)


def test_batched_against_oracle_per_instance():
    insts = _batch()
    T = 20
    bp = B.Plan([B.Problem.from_ilp(q) for q in insts])
    bs = B.Solver(bp)
    bs.iterate(T)
    got = _outputs(bs)
    var_off, row_off, inc_off = bp.instances()
    for k, q in enumerate(insts):
        print(f"[batch-oracle] instance {k} {q.name}", flush=True)
        o = Oracle(q)
        o.init()
        tr = o.iterate(T)
        lam_ref = o.lam()
        r0, r1 = o.min_marginals()
        a, b = inc_off[k], inc_off[k + 1]
        assert got["inst"][k] == pytest.approx(tr[-1], rel=1e-4, abs=1e-4)
        scale = incidence_scale(q, lam_ref)
        assert_incidence_close(got["lam"][a:b], lam_ref, scale, what=f"lambda {k}")
        assert_incidence_close(got["m0"][a:b], r0, scale, what=f"m0 {k}")
        assert_incidence_close(got["m1"][a:b], r1, scale, what=f"m1 {k}")
        # the oracle's float mirror: bitwise
        f = Oracle(q, precision="f32")
        f.init()
        f.iterate(T)
        assert np.array_equal(got["lam"][a:b].astype(np.float64), f.lam()), k


def test_instance_bound_of_a_single_plan_is_the_bound():
    ilp = I.config(1)
    s = B.Solver(B.Plan(B.Problem.from_ilp(ilp)))
    s.iterate(7)
    lb = s.lower_bound()[0]
    (inst,) = s.instance_bounds()
    assert inst == pytest.approx(lb, rel=1e-12, abs=1e-12)
    with pytest.raises(B.BddmpError) as e:
        B.bddmp_solver_instance_bounds(s.h, 2)
    assert e.value.code == -1


def test_full_size_batched_workload():
    """The 256-instance batched workload at its full size, in the launch configuration the benchmark
    times (graph replay): bound finite and non-decreasing, the instance bounds add up to it, sampled
    instances bitwise equal to their own plans, and the smallest tomography instance against the fp64
    oracle."""
    import torch

    insts = I.batch_config(256)
    T = 8
    bp = B.Plan([B.Problem.from_ilp(q) for q in insts])
    print(f"[batch full] nodes={bp.stats.n_nodes} waves={bp.stats.waves_fwd}", flush=True)
    bs = B.Solver(bp)
    bs.iterate(T)
    hist = bs.lb_history(T + 1)
    lam = bs.get_lambda().cpu().numpy()
    inst = bs.instance_bounds()
    torch.cuda.synchronize()
    assert np.all(np.isfinite(hist))
    assert np.all(np.diff(hist) >= -1e-6 * np.maximum(np.abs(hist[1:]), 1.0))
    assert inst.sum() == pytest.approx(hist[-1], rel=1e-12, abs=1e-6)
    var_off, row_off, inc_off = bp.instances()
    del bs
    torch.cuda.empty_cache()
    sizes = [q.n for q in insts]
    tomo = [k for k, q in enumerate(insts) if q.name.startswith("tomo")]
    small = min(tomo, key=lambda k: sizes[k])
    for k in sorted({0, 1, small, len(insts) - 2, len(insts) - 1}):
        print(f"[batch full] instance {k} {insts[k].name}", flush=True)
        s = B.Solver(B.Plan(B.Problem.from_ilp(insts[k])))
        s.iterate(T)
        assert np.array_equal(lam[inc_off[k]:inc_off[k + 1]], s.get_lambda().cpu().numpy()), k
        del s
    q = insts[small]
    o = Oracle(q)
    o.init()
    tr = o.iterate(T)
    assert inst[small] == pytest.approx(tr[-1], rel=1e-4, abs=1e-4)
    lam_ref = o.lam()
    assert_incidence_close(lam[inc_off[small]:inc_off[small + 1]], lam_ref, incidence_scale(q, lam_ref),
                           what="lambda (smallest tomography instance)")
