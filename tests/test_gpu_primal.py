"""The primal heuristic fed by the GPU path: total min-marginal differences M from the device
(bitwise those of the oracle's float mirror), then the search; the result equals the oracle's search
on the same M and satisfies every row."""
import numpy as np
import pytest

from oracle import Oracle
from oracle.primal import primal_heuristic
from paper_2009_00481_amd import binding as B
from paper_2009_00481_amd import instances as I

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["cfg1", "5sub", "gm", "track"])
def test_search_from_device_marginals(name):
    import torch

    ilp = {"cfg1": lambda: I.config(1), "5sub": lambda: I.config("5sub"),
           "gm": lambda: I.graph_matching(40, 40, 5, 60, seed=3), "track": lambda: I.tracking(300, seed=2)}[name]()
    plan = B.Plan(B.Problem.from_ilp(ilp))
    s = B.Solver(plan)
    s.iterate(20)
    M, x_round, obj_round, nviol = s.round_primal()
    M = M.cpu().numpy()
    torch.cuda.synchronize()
    f = Oracle(ilp, precision="f32")
    f.init()
    f.iterate(20)
    Mf, _, _, _ = f.round()
    assert np.array_equal(M.astype(np.float64), Mf)
    for mode in (0, 1, 2):
        x, obj, feas, _ = plan.primal_search(M, mode)
        xr, objr, feasr = primal_heuristic(ilp, M, mode)
        assert feas == feasr and np.array_equal(x, xr), (name, mode)
        if feas:
            for j in range(ilp.m):
                cols, coefs, sense, rhs = ilp.row(j)
                v = int(np.dot(coefs, x[cols].astype(np.int64)))
                assert (sense == 0 and v == rhs) or (sense == 1 and v <= rhs) or (sense == 2 and v >= rhs)
