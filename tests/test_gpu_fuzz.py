"""Randomised GPU parity: many small random 0-1 ILPs of varied shape (row lengths, coefficient
ranges, senses, variable orders, forced variables, wide levels, splits into intervals), each run on
the GPU and through the oracle's float mirror with the same steps: multipliers, min-marginals and
total differences bitwise equal, bounds to 1e-12 (fp64 sums in another order). A second pass packs
the same instances into batched plans and checks each against its own plan bitwise."""
import numpy as np
import pytest

from oracle import Oracle, OracleError
from paper_2009_00481_amd import binding as B
from paper_2009_00481_amd import instances as I

pytestmark = pytest.mark.gpu


def _draw(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(6, 70))
    m = int(rng.integers(3, 50))
    kmax = int(rng.integers(2, 14))
    cmax = int(rng.integers(1, 5))
    ilp = I.random_ilp(n, m, kmin=1, kmax=kmax, cmax=cmax, seed=seed, cover_all=bool(rng.integers(0, 2)))
    return ilp, int(rng.integers(0, 2)), int(rng.choice([0, 0, 2, 3, 5])), int(rng.integers(1, 12))


def _gpu(ilp, order_mode, K, T):
    import torch

    plan = B.Plan(B.Problem.from_ilp(ilp), order_mode=order_mode, n_intervals=K)
    s = B.Solver(plan)
    s.iterate(T)
    out = dict(plan=plan, hist=s.lb_history(T + 1), lam=s.get_lambda().cpu().numpy().astype(np.float64))
    m0, m1 = s.min_marginals()
    M, x, obj, nv = s.round_primal()
    torch.cuda.synchronize()
    out.update(m0=m0.cpu().numpy().astype(np.float64), m1=m1.cpu().numpy().astype(np.float64),
               M=M.cpu().numpy().astype(np.float64), x=x, nviol=nv)
    return out


@pytest.mark.parametrize("block", range(4))
def test_random_instances_bitwise_against_float_mirror(block):
    checked = 0
    for seed in range(block * 40, block * 40 + 40):
        ilp, om, K, T = _draw(seed)
        try:
            g = _gpu(ilp, om, K, T)
        except B.BddmpError as e:
            # the oracle must reject the same instance (forced conflicts)
            with pytest.raises(OracleError):
                o = Oracle(ilp, precision="f32", split=K)
                o.init()
                o.iterate(T)
            assert e.code == -5, (seed, e)
            continue
        q = I.ILP(ilp.n, ilp.cost, ilp.row_ptr, ilp.col, ilp.coef, ilp.sense, ilp.rhs, g["plan"].order())
        o = Oracle(q, precision="f32", split=K)
        tr = np.concatenate([[o.init()], o.iterate(T)])
        m0, m1 = o.min_marginals()
        M, x, _, nv = o.round()
        ctx = (seed, om, K, T)
        assert np.array_equal(g["lam"], o.lam()), ctx
        assert np.array_equal(g["m0"], m0) and np.array_equal(g["m1"], m1), ctx
        assert np.array_equal(g["M"], M) and np.array_equal(g["x"], x) and g["nviol"] == nv, ctx
        np.testing.assert_allclose(g["hist"], tr, rtol=1e-12, atol=1e-9, err_msg=str(ctx))
        checked += 1
    print(f"[fuzz] block {block}: {checked} instances bitwise equal", flush=True)
    assert checked >= 30


def test_random_batches_equal_their_instances():
    import torch

    rng = np.random.default_rng(7)
    for trial in range(6):
        seeds = rng.choice(10000, size=int(rng.integers(2, 9)), replace=False)
        ilps = []
        for sd in seeds:
            ilp, _, _, _ = _draw(int(sd))
            try:
                B.Plan(B.Problem.from_ilp(ilp))
            except B.BddmpError:
                continue
            ilps.append(ilp)
        K = int(rng.choice([0, 2, 4]))
        om = int(rng.integers(0, 2))
        probs = [B.Problem.from_ilp(q) for q in ilps]
        bp = B.Plan(probs, order_mode=om, n_intervals=K)
        bs = B.Solver(bp)
        bs.iterate(5)
        lam = bs.get_lambda().cpu().numpy()
        inst = bs.instance_bounds()
        _, _, inc = bp.instances()
        for k, pr in enumerate(probs):
            s = B.Solver(B.Plan(pr, order_mode=om, n_intervals=K))
            s.iterate(5)
            assert np.array_equal(lam[inc[k]:inc[k + 1]], s.get_lambda().cpu().numpy()), (trial, k)
            assert inst[k] == s.instance_bounds()[0], (trial, k)
        torch.cuda.synchronize()


@pytest.mark.parametrize("block", range(2))
def test_random_wide_rows_any_general_path(block):
    """Long rows with large coefficients (levels of tens to hundreds of nodes, the general-layer
    paths), a random choice of lanes per width class: bitwise equal to the float mirror."""
    import torch

    checked = 0
    for seed in range(block * 12, block * 12 + 12):
        rng = np.random.default_rng(5000 + seed)
        n = int(rng.integers(20, 120))
        ilp = I.random_ilp(n, int(rng.integers(4, 30)), kmin=2, kmax=int(rng.integers(8, 40)),
                           cmax=int(rng.integers(2, 7)), seed=7000 + seed)
        om, K, T = int(rng.integers(0, 2)), int(rng.choice([0, 0, 3])), int(rng.integers(2, 8))
        try:
            plan = B.Plan(B.Problem.from_ilp(ilp), order_mode=om, n_intervals=K, node_budget=2_000_000)
        except B.BddmpError:
            continue
        s = B.Solver(plan)
        lanes = [int(rng.choice([0, 1, 2, 4, 8, 16, 32, 64])) for _ in range(4)]
        s.set_groups(lanes)
        s.iterate(T)
        lam = s.get_lambda().cpu().numpy().astype(np.float64)
        m0, m1 = (t.cpu().numpy().astype(np.float64) for t in s.min_marginals())
        torch.cuda.synchronize()
        q = I.ILP(ilp.n, ilp.cost, ilp.row_ptr, ilp.col, ilp.coef, ilp.sense, ilp.rhs, plan.order())
        o = Oracle(q, precision="f32", split=K)
        o.init()
        o.iterate(T)
        r0, r1 = o.min_marginals()
        ctx = (seed, om, K, T, lanes, plan.stats.max_width)
        assert np.array_equal(lam, o.lam()), ctx
        assert np.array_equal(m0, r0) and np.array_equal(m1, r1), ctx
        checked += 1
    print(f"[fuzz wide] block {block}: {checked} instances", flush=True)
    assert checked >= 8
