"""Shared helpers of the GPU parity tests: run a problem through the C-ABI and through the oracle."""
from __future__ import annotations

import numpy as np

from oracle import Oracle
from paper_2009_00481_amd import binding as B

# Tolerance of the FP32 GPU path against the FP64 oracle: relative 1e-4, the precision at which the
# benchmark's time to bound is defined
REL = 1e-4


def run_gpu(ilp, iters: int, *, order_mode: int = 0, stages=None, split: int = 0, gamma: float = 0.0):
    """Bind, iterate, read every output. stages: iterations after which the bound is read.
    split / gamma: variable intervals and copy-arc step size of Sec. 6 (0: no split)."""
    import torch

    prob = B.Problem.from_ilp(ilp)
    plan = B.Plan(prob, order_mode=order_mode, hist_cap=max(4096, iters + 8), n_intervals=split, split_gamma=gamma)
    s = B.Solver(plan)
    s.iterate(iters)
    lb, resid, any_lb = s.lower_bound()
    hist = s.lb_history(iters + 1)
    lam = s.get_lambda().cpu().numpy().astype(np.float64)
    m0, m1 = s.min_marginals()
    M, x, obj, nviol = s.round_primal()
    torch.cuda.synchronize()
    return dict(plan=plan, solver=s, lb=lb, resid=resid, any_lb=any_lb, hist=hist, lam=lam,
                m0=m0.cpu().numpy().astype(np.float64), m1=m1.cpu().numpy().astype(np.float64),
                M=M.cpu().numpy().astype(np.float64), x=x, obj=obj, nviol=nviol)


def run_oracle(ilp, iters: int, precision: str = "f64", split: int = 0, gamma: float = 0.5):
    o = Oracle(ilp, precision=precision, split=split, gamma=gamma)
    lb0 = o.init()
    tr = o.iterate(iters)
    m0, m1 = o.min_marginals()
    M, x, obj, nviol = o.round()
    resid, any_lb = o.residual()
    w, var, _, _ = o.structure()
    return dict(o=o, hist=np.concatenate([[lb0], tr]), lam=o.lam(), m0=m0, m1=m1, M=M, x=x, obj=obj,
                nviol=nviol, resid=resid, any_lb=any_lb, level_var=var, cost=ilp.cost)


def incidence_scale(ilp, lam_ref):
    """S_j per canonical incidence: sum of |lambda_ref| over the row's incidences."""
    nz = np.asarray(ilp.coef) != 0
    row_of_nnz = np.repeat(np.arange(ilp.m), np.diff(ilp.row_ptr))
    lens = np.bincount(row_of_nnz[nz], minlength=ilp.m)
    row_of = np.repeat(np.arange(ilp.m), lens)
    s = np.zeros(ilp.m)
    np.add.at(s, row_of, np.abs(lam_ref))
    return s[row_of]


def assert_incidence_close(got, ref, scale, rel=REL, what=""):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    inf_ref = np.isinf(ref)
    assert np.array_equal(np.isinf(got), inf_ref), f"{what}: infinities differ"
    assert np.array_equal(np.sign(got[inf_ref]), np.sign(ref[inf_ref])), f"{what}: infinity signs differ"
    fin = ~inf_ref
    tol = rel * np.maximum(np.maximum(np.abs(ref[fin]), scale[fin]), 1.0)
    err = np.abs(got[fin] - ref[fin])
    bad = err > tol
    assert not bad.any(), f"{what}: {bad.sum()} of {fin.sum()} beyond tolerance, worst {np.max(err / tol):.3g}x"


def assert_trace_close(got, ref, rel=REL, what="bound"):
    got = np.asarray(got)
    ref = np.asarray(ref)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    tol = rel * np.maximum(np.abs(ref), 1.0)
    bad = np.abs(got - ref) > tol
    assert not bad.any(), f"{what}: first bad t={np.argmax(bad)} got {got[bad][0]} ref {ref[bad][0]}"
