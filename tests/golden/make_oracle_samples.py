"""Writes seeded samples of the fp64 oracle's per-element results at the benchmark workloads' full
size, for the GPU tests that compare the end of a full benchmark run element by element.

- potts256x256_L8.npz: after 500 iterations of Alg. "Min-marginal averaging" (Sec. 3.2) on the
  256x256, 8-label Potts workload: the multipliers lambda^j_i and the fresh min-marginals m0, m1
  (eq. "min-marginals") at 100,000 canonical incidences drawn without replacement (seed 0), with
  each incidence's row scale S_j = sum over the row of |lambda|, the scale of the per-incidence bar.
- potts128x128_L4_grad.npz: the smoothed bound after 50 smoothed iterations at alpha = 0.1 (App.
  "Smoothing") on the 128x128, 4-label Potts workload and its gradient d LB_alpha / d c (the
  oracle's fp64 reverse accumulation) at 1,000 variables drawn without replacement (seed 0).

Only the seeded input generators and the oracle are called. Run from the repository root:

    python tests/golden/make_oracle_samples.py [potts256x256_L8] [potts128x128_L4_grad]

The first takes about 15 minutes on one host core, the second a few minutes.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import Oracle  # noqa: E402
from paper_2009_00481_amd import instances as I  # noqa: E402


def row_scale(ilp, lam):
    """S_j per canonical incidence: sum of |lambda| over the incidence's row."""
    nz = np.asarray(ilp.coef) != 0
    row_of_nnz = np.repeat(np.arange(ilp.m), np.diff(ilp.row_ptr))
    lens = np.bincount(row_of_nnz[nz], minlength=ilp.m)
    row_of = np.repeat(np.arange(ilp.m), lens)
    s = np.zeros(ilp.m)
    np.add.at(s, row_of, np.abs(lam))
    return s[row_of]


def mrf_end_state(T=500, n=100_000):
    ilp = I.config(2)
    t0 = time.perf_counter()
    o = Oracle(ilp)
    lb = [o.init()]
    for t in range(T):
        lb.append(float(o.iterate(1)[0]))
        if (t + 1) % 50 == 0:
            print(f"potts256x256_L8: {t + 1}/{T} LB {lb[-1]:.10g} ({time.perf_counter() - t0:.0f} s)", flush=True)
    lam = o.lam()
    m0, m1 = o.min_marginals()
    idx = np.sort(np.random.default_rng(0).choice(lam.shape[0], size=n, replace=False)).astype(np.int64)
    np.savez_compressed(os.path.join(HERE, "potts256x256_L8.npz"), iterations=T, idx=idx, lam=lam[idx], m0=m0[idx],
                        m1=m1[idx], scale=row_scale(ilp, lam)[idx], lb=np.asarray(lb))
    print(f"potts256x256_L8: written ({time.perf_counter() - t0:.0f} s)", flush=True)


def smooth_gradient(alpha=0.1, T=50, n=1000):
    ilp = I.config(5)
    t0 = time.perf_counter()
    g, lb = Oracle(ilp).smooth_grad(alpha, T)
    idx = np.sort(np.random.default_rng(0).choice(ilp.n, size=n, replace=False)).astype(np.int64)
    np.savez_compressed(os.path.join(HERE, "potts128x128_L4_grad.npz"), alpha=alpha, iterations=T, idx=idx, grad=g[idx],
                        lb=lb, grad_abs_max=np.abs(g).max())
    print(f"potts128x128_L4_grad: written ({time.perf_counter() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    jobs = sys.argv[1:] or ["potts256x256_L8", "potts128x128_L4_grad"]
    for j in jobs:
        {"potts256x256_L8": mrf_end_state, "potts128x128_L4_grad": smooth_gradient}[j]()
