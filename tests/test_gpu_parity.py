"""GPU parity: the HIP path through the C-ABI against the CPU oracle, element by element.

Bars (the FP32 GPU against the FP64 oracle): every bound of the trace within relative 1e-4;
multipliers and fresh min-marginals within 1e-4 of max(|ref|, S_j, 1) with S_j the row's sum of
|lambda|; infinities identical. Against the oracle's float mirror (same precision, same order of
every sum) multipliers, min-marginals and total differences must be bitwise equal, so the rounded
primal is decided identically.
"""
import numpy as np
import pytest

from parity import (REL, assert_incidence_close, assert_trace_close, incidence_scale, run_gpu,
                    run_oracle)
from paper_2009_00481_amd import instances as I

pytestmark = pytest.mark.gpu


def _case(name):
    if name == "cfg1":
        return I.config(1), 100
    if name == "cfg5sub":
        return I.config("5sub"), 50
    if name == "gm_small":
        return I.graph_matching(300, 300, 10, 3000, seed=1), 40
    if name == "potts_5x7_L6":
        return I.potts_grid(5, 7, 6, seed=2), 30
    if name.startswith("rand"):
        seed = int(name[4:])
        return I.random_ilp(40, 30, kmin=1, kmax=10, cmax=3, seed=seed), 25
    if name == "wide":
        rng = np.random.default_rng(7)
        rows = []
        for j in range(8):
            vs = rng.choice(60, size=40, replace=False)
            cs = rng.integers(1, 4, size=40)
            rows.append((vs, cs, j % 3, int(cs.sum() // 2)))
        for v in range(60):
            rows.append(([v, (v + 1) % 60], [1, 1], 1, 1))
        return I.from_rows(60, rng.standard_normal(60).astype(np.float32), rows, order=rng.permutation(60)), 20
    if name == "bigvar":
        # variable 0 sits in 300 rows x0 + x_k <= 1 (a tile of its own); more rows tie the rest
        rows = [([0, k], [1, 1], 1, 1) for k in range(1, 301)]
        rows += [([k, k + 1, k + 2], [1, 1, 1], 2, 1) for k in range(1, 299, 3)]
        rng = np.random.default_rng(3)
        cost = rng.standard_normal(301).astype(np.float32)
        cost[0] = -5.0
        return I.from_rows(301, cost, rows, order=rng.permutation(301)), 15
    if name == "forced":
        rows = [([0, 1], [2, 3], 0, 5), ([2, 3], [1, 1], 1, 0), ([0, 2, 4], [1, 1, 1], 1, 2),
                ([1, 3, 5], [1, -1, 1], 2, 1), ([4, 5], [1, 1], 0, 1), ([4, 6, 7], [1, 1, 1], 0, 1)]
        return I.from_rows(8, [0.3, -0.7, 0.2, 0.9, -0.4, 0.25, 0.5, -0.1], rows, order=[3, 1, 5, 0, 2, 4, 7, 6]), 20
    raise ValueError(name)


CASES = ["cfg1", "cfg5sub", "gm_small", "potts_5x7_L6", "rand0", "rand1", "rand2", "rand3", "wide",
         "bigvar", "forced"]


@pytest.mark.parametrize("name", CASES)
def test_parity_against_fp64_oracle(name):
    ilp, iters = _case(name)
    print(f"[parity fp64] {name}: n={ilp.n} m={ilp.m} iters={iters}", flush=True)
    g = run_gpu(ilp, iters)
    r = run_oracle(ilp, iters, "f64")
    assert_trace_close(g["hist"], r["hist"])
    scale = incidence_scale(ilp, r["lam"])
    assert_incidence_close(g["lam"], r["lam"], scale, what="lambda")
    assert_incidence_close(g["m0"], r["m0"], scale, what="m0")
    assert_incidence_close(g["m1"], r["m1"], scale, what="m1")
    # rounded primal: identical wherever the total difference is decided beyond the tolerance
    decided = np.abs(r["M"]) > 1e-3 * np.maximum(1.0, np.abs(r["M"]))
    assert np.array_equal(g["x"][decided], r["x"][decided])
    assert g["obj"] == pytest.approx(float(ilp.cost @ g["x"]), abs=1e-9)
    # dual feasibility is kept up to float rounding: each update of variable i rounds |J_i| terms
    # three times (lambda - d, the share, their sum), 2 passes per iteration, each rounding at most
    # half an ulp of the largest multiplier (2^-24 relative)
    maxJ = g["plan"].stats.max_rows_per_var
    big = max(float(np.abs(r["lam"]).max()), float(np.abs(ilp.cost).max()), 1.0)
    assert g["resid"] <= 6 * iters * maxJ * 2.0 ** -24 * big, g["resid"]


@pytest.mark.parametrize("name", CASES)
def test_bitwise_against_fp32_mirror(name):
    ilp, iters = _case(name)
    print(f"[parity fp32] {name}: n={ilp.n} m={ilp.m} iters={iters}", flush=True)
    g = run_gpu(ilp, iters)
    r = run_oracle(ilp, iters, "f32")
    assert np.array_equal(g["lam"], r["lam"]), np.max(np.abs(g["lam"] - r["lam"]))
    assert np.array_equal(g["m0"], r["m0"])
    assert np.array_equal(g["m1"], r["m1"])
    assert np.array_equal(g["M"], r["M"])
    assert np.array_equal(g["x"], r["x"])
    assert g["nviol"] == r["nviol"]
    assert g["obj"] == pytest.approx(r["obj"], rel=1e-12, abs=1e-12)
    np.testing.assert_allclose(g["hist"], r["hist"], rtol=1e-12, atol=1e-9)
    # same multipliers, same fp64 per-variable sums: the residual and any-lambda bound agree
    assert g["resid"] == pytest.approx(r["resid"], rel=1e-12, abs=1e-15)
    assert g["any_lb"] == pytest.approx(r["any_lb"], rel=1e-12, abs=1e-9)
