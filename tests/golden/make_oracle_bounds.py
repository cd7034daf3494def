"""Writes oracle_bounds.json: the fp64 oracle's lower bound after every iteration of each benchmark
workload (Alg. "Min-marginal averaging", Sec. 3.2; LB_t of problem (D) after iteration t, LB_0
after the initial backward sweep), for as many iterations as the benchmark runs per step.

Only the seeded input generators and the oracle are called. Run from the repository root:

    python tests/golden/make_oracle_bounds.py [workload ...]

The 256x256x8 Potts workload takes about 12 minutes on one host core (500 iterations at ~1.4 s).
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import Oracle  # noqa: E402
from paper_2009_00481_amd import instances as I  # noqa: E402

OUT = os.path.join(HERE, "oracle_bounds.json")

# workload name: (instances.config index, iterations)
WORKLOADS = {
    "potts8x8_L3": (1, 100),
    "potts128x128_L4": (5, 50),
    "gm5000x5000": (3, 200),
    "potts256x256_L8": (2, 500),
}


def run(name):
    cfg, T = WORKLOADS[name]
    ilp = I.config(cfg)
    t0 = time.perf_counter()
    o = Oracle(ilp)
    lb = [o.init()]
    for t in range(T):
        lb.append(float(o.iterate(1)[0]))
        if (t + 1) % 25 == 0:
            print(f"{name}: {t + 1}/{T} LB {lb[-1]:.10g} ({time.perf_counter() - t0:.0f} s)", flush=True)
    return {"config": cfg, "iterations": T, "n_vars": ilp.n, "n_rows": ilp.m, "lb": lb,
            "seconds": time.perf_counter() - t0}


def main(names):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    data.setdefault("source", "fp64 oracle (oracle/bddmp_oracle.c), written by tests/golden/make_oracle_bounds.py; "
                              "inputs from paper_2009_00481_amd/instances.py config(k), the workload's own order")
    data.setdefault("workloads", {})
    for name in names:
        data["workloads"][name] = run(name)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1)
        print(f"{name}: written", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(WORKLOADS))
