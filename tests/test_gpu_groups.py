"""GPU tests of the lane groups that run general layers (a level or its next level wider than 2):
every group size and the autotuner's choice give bitwise the same iterates (every minimum is
exact), and wide workloads match the oracle."""
import numpy as np
import pytest

from parity import assert_incidence_close, assert_trace_close, incidence_scale
from oracle import Oracle
from paper_2009_00481_amd import binding as B
from paper_2009_00481_amd import instances as I

pytestmark = pytest.mark.gpu


def _run(ilp, T, lanes=None, tiling=None):
    import torch

    s = B.Solver(B.Plan(B.Problem.from_ilp(ilp), tiling=tiling))
    if lanes is not None:
        s.set_groups(lanes)
    s.iterate(T)
    lam = s.get_lambda().cpu().numpy()
    m0, m1 = s.min_marginals()
    hist = s.lb_history(T + 1)
    torch.cuda.synchronize()
    return s, lam, m0.cpu().numpy(), m1.cpu().numpy(), hist


def _wide_rows():
    rng = np.random.default_rng(11)
    rows = []
    for j in range(6):
        vs = rng.choice(90, size=70, replace=False)
        cs = rng.integers(1, 5, size=70)
        rows.append((vs, cs, j % 3, int(cs.sum() // 2)))
    for v in range(90):
        rows.append(([v, (v + 3) % 90], [1, 1], 1, 1))
    return I.from_rows(90, rng.standard_normal(90).astype(np.float32), rows, order=rng.permutation(90))


@pytest.mark.parametrize("name", ["tomo", "wide"])
def test_every_group_size_gives_the_same_iterates(name):
    ilp = I.tomography(12, seed=4, unary="normal") if name == "tomo" else _wide_rows()
    T = 12
    print(f"[groups] {name}", flush=True)
    _, lam, m0, m1, hist = _run(ilp, T, lanes=[1, 1, 1, 1])
    for g in (0, 2, 4, 8, 16, 32, 64):
        _, lam2, m02, m12, hist2 = _run(ilp, T, lanes=[g, g, g, g])
        assert np.array_equal(lam, lam2), g
        assert np.array_equal(m0, m02) and np.array_equal(m1, m12), g
        assert np.array_equal(hist, hist2), g
    _, lam3, _, _, _ = _run(ilp, T, tiling="64,8,2,32")
    assert np.array_equal(lam, lam3)
    _, lam4, _, _, _ = _run(ilp, T, tiling="0,8,0,32")
    assert np.array_equal(lam, lam4)


def test_autotune_then_reset_gives_the_same_iterates():
    import torch

    ilp = I.tomography(16, seed=5, unary="normal")
    T = 10
    _, lam, m0, m1, hist = _run(ilp, T)
    s = B.Solver(B.Plan(B.Problem.from_ilp(ilp)))
    lanes = s.autotune(2)
    assert all(int(v) in (0, 1, 2, 4, 8, 16, 32, 64) for v in lanes)
    assert np.array_equal(s.groups(), lanes)
    s.reset()
    s.iterate(T)
    lam2 = s.get_lambda().cpu().numpy()
    torch.cuda.synchronize()
    assert np.array_equal(lam, lam2)
    with pytest.raises(B.BddmpError) as e:
        s.set_groups([3, 4, 4, 4])
    assert e.value.code == -1


@pytest.mark.parametrize("P", [10, 24])
def test_tomography_against_oracle(P):
    ilp = I.tomography(P, seed=P, unary="normal")
    T = 15
    _, lam, m0, m1, hist = _run(ilp, T)
    o = Oracle(ilp)
    lb0 = o.init()
    tr = o.iterate(T)
    assert_trace_close(hist, np.concatenate([[lb0], tr]))
    lam_ref = o.lam()
    r0, r1 = o.min_marginals()
    scale = incidence_scale(ilp, lam_ref)
    assert_incidence_close(lam, lam_ref, scale, what="lambda")
    assert_incidence_close(m0, r0, scale, what="m0")
    assert_incidence_close(m1, r1, scale, what="m1")
    f = Oracle(ilp, precision="f32")
    f.init()
    f.iterate(T)
    assert np.array_equal(lam.astype(np.float64), f.lam())
    f0, f1 = f.min_marginals()
    assert np.array_equal(m0.astype(np.float64), f0) and np.array_equal(m1.astype(np.float64), f1)
