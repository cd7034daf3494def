"""The stored oracle bound trajectories (tests/golden/oracle_bounds.json, written by
make_oracle_bounds.py) are what the oracle computes now: the small workloads are re-run in full, the
larger ones over their first iterations, and every trajectory rises (Alg. "Min-marginal averaging"
never lowers the bound of problem (D))."""
import json
import os

import numpy as np
import pytest

from oracle import Oracle
from paper_2009_00481_amd import instances as I

PATH = os.path.join(os.path.dirname(__file__), "golden", "oracle_bounds.json")


def _stored():
    with open(PATH) as f:
        return json.load(f)["workloads"]


def test_stored_workloads_and_lengths():
    w = _stored()
    want = {"potts8x8_L3": (1, 100), "potts128x128_L4": (5, 50), "gm5000x5000": (3, 200),
            "potts256x256_L8": (2, 500)}
    for name, (cfg, T) in want.items():
        assert w[name]["config"] == cfg and w[name]["iterations"] == T
        lb = np.asarray(w[name]["lb"])
        assert lb.shape == (T + 1,) and np.all(np.isfinite(lb))
        assert np.all(np.diff(lb) >= -1e-9 * np.abs(lb[1:])), name
        assert lb[-1] > lb[0]


@pytest.mark.parametrize("name,iters", [("potts8x8_L3", 100), ("potts128x128_L4", 3), ("gm5000x5000", 2)])
def test_oracle_reproduces_stored_bounds(name, iters):
    w = _stored()[name]
    ilp = I.config(w["config"])
    assert (ilp.n, ilp.m) == (w["n_vars"], w["n_rows"])
    o = Oracle(ilp)
    got = np.concatenate([[o.init()], o.iterate(iters)])
    ref = np.asarray(w["lb"][:iters + 1])
    assert np.allclose(got, ref, rtol=1e-12, atol=0.0), np.abs(got - ref).max()
