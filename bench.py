"""Benchmark of the BDD min-marginal averaging hot path on one MI355X.

A step is one pass of the whole hot path over the bound instance, whose layout is already resident
in HBM: initialisation (multipliers c_i/|J_i| and the initial backward sweep), T iterations of
forward pass + backward pass + fp64 bound, then the outputs (fresh min-marginals and the rounded
primal with its objective and violated-row count). The host BDD build and the upload are timed
separately and not part of a step.

value = BDD arc-updates per second = 2 * live arcs * T per step / step time (each live arc is
relaxed and marginalised once per pass). The roofline object prices the dominant wave kernel's
algorithmic bytes (20 per node and 8 per incidence per pass) against MI355X HBM peak; cpu_baseline
is the fp64 CPU oracle on the same instance, one thread, on a bounded sample of iterations.

smoothed_vs_plain: the differentiable form (smoothed iterations with checkpoints, then the adjoint
giving d LB_alpha / d c) on Potts 128x128 with 4 labels, 50 iterations, alpha in {1, 0.1, 0.01},
against plain min-plus iterations on the same instance.

batched_vs_plain: the batched workload (256 tomography and tracking instances of uneven size) in
one schedule (every variable in its latest wave, wave-group launches of 256 consecutive waves; one
launch per wave and the dataflow launch alongside) against the same instances run one after another
through their own plans; a sample of instances is compared bitwise.

Usage: python bench.py [--gpus 1] [--steps 5] [--warmup 1] [--workload potts256x256_L8] [--no-batched]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "BDD arc-updates/sec + HBM GB/s per DBCA iter; time to bound at 1e-4; batched vs plain"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # name: (instance config, iterations per step)
    "potts256x256_L8": (2, 500),
    "potts8x8_L3": (1, 100),
    "gm5000x5000": (3, 200),
    "potts128x128_L4": (5, 50),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNEL_SOURCES = ["paper_2009_00481_amd/csrc/kernels.hip", "paper_2009_00481_amd/csrc/kernels.h",
                  "paper_2009_00481_amd/csrc/device.h",
                  "paper_2009_00481_amd/csrc/plan.cpp", "paper_2009_00481_amd/csrc/internal.h"]


def kernel_source_hash() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def committed_traffic(workload: str, kernel: str = ""):
    """HBM bytes per launch of the update kernels (kernel "": one launch per wave; "group_": the
    wave-group launch; "pair_": the wave-group launch with two tiles per workgroup) from the
    committed counter summary, or None when the summary is missing, lacks them or was taken on
    different kernel sources."""
    path = os.path.join(ROOT, "profiles", f"wave_kernels_{workload}.md")
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("traffic source_hash="):
            kv = dict(tok.split("=", 1) for tok in line.split()[1:])
            if kv.get("source_hash") != kernel_source_hash() or f"{kernel}fwd_bytes_per_launch" not in kv:
                return None
            return {"fwd": float(kv[f"{kernel}fwd_bytes_per_launch"]), "bwd": float(kv[f"{kernel}bwd_bytes_per_launch"])}
    return None


def roofline_of(kt, traffic_rec, kernel="wave_kernel"):
    """The dominant update kernel class (the pass direction with the larger summed time) priced
    against MI355X HBM peak: model bytes per launch over the average launch time (HIP events around
    whole passes on the solver's stream); traffic from the committed counter summary, or None."""
    if kt["fwd_ms"] >= kt["bwd_ms"]:
        kname, kms, kb, kl = f"{kernel}<fwd,update>", kt["fwd_ms"], kt["fwd_bytes"], kt["fwd_launches"]
    else:
        kname, kms, kb, kl = f"{kernel}<bwd,update>", kt["bwd_ms"], kt["bwd_bytes"], kt["bwd_launches"]
    achieved = (kb / kl) / ((kms / kl) * 1e-3) / 1e9
    traffic = None if traffic_rec is None else traffic_rec["fwd" if "fwd" in kname else "bwd"]
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "traffic_unit": "bytes/launch",
            "kernel": kname, "bytes_per_launch": kb / kl, "avg_launch_us": kms / kl * 1e3,
            "both_passes_gbs": round((kt["fwd_bytes"] + kt["bwd_bytes"]) / ((kt["fwd_ms"] + kt["bwd_ms"]) * 1e-3) / 1e9, 1)}


def oracle_bounds(workload: str, T: int):
    """The fp64 oracle's bounds LB_0..LB_T on the workload (written by
    tests/golden/make_oracle_bounds.py), or None when they are not stored for T iterations."""
    import numpy as np

    path = os.path.join(ROOT, "tests", "golden", "oracle_bounds.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        w = json.load(f).get("workloads", {}).get(workload)
    if w is None or len(w["lb"]) < T + 1:
        return None
    return np.asarray(w["lb"][:T + 1], dtype=np.float64)


_BATCH = {}
_BATCH_CPU = {}


def batch_instances(I, n):
    """The batched workload's instances, generated once per run (seconds of host work)."""
    if n not in _BATCH:
        t = time.perf_counter()
        _BATCH[n] = (I.batch_config(n), time.perf_counter() - t)
    return _BATCH[n]


def batched_vs_plain(args, B, I, torch):
    """The batched workload (tomography and tracking instances of uneven size) solved in one
    schedule against the same instances solved one after another through their own plans."""
    import numpy as np

    n = args.batch_instances
    insts, gen_s = batch_instances(I, n)
    probs = [B.Problem.from_ilp(q) for q in insts]
    t = time.perf_counter()
    # every variable in its latest wave (shorter instances start late; same results)
    bp = B.Plan(probs, wave_align=1)
    plan_s = time.perf_counter() - t
    st = bp.stats
    log(f"[bench] batched: {n} instances, nodes={st.n_nodes} incidences={st.n_incidences} "
        f"waves={st.waves_fwd}+{st.waves_bwd} plan {plan_s:.1f}s")
    bs = B.Solver(bp)
    T = args.batch_iters

    def timed(mode, chunk):
        bs.set_launch(mode, chunk)
        bs.iterate(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bs.iterate(T)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / T

    # one launch per wave, then wave-group launches (args.batch_group_waves consecutive waves per
    # launch; the leg's figure), each with its dominant kernel against HBM peak (events around
    # whole passes, as for the main workload), then the dataflow launch of the same passes
    G = args.batch_group_waves
    wave_ms = timed(0, 0)
    wave_roofline = roofline_of(bs.time_kernels(3), committed_traffic(f"batch{n}"))
    batched_ms = timed(3, G)
    roofline = roofline_of(bs.time_kernels(3), committed_traffic(f"batch{n}", "group_"), "group_kernel")
    dataflow_ms = timed(1, 1)
    bs.set_launch(3, G)
    # bitwise check on a sample: the same iterations from the start, batched and plain
    Tc = 5
    bs.reset()
    bs.iterate(Tc)
    lam_b = bs.get_lambda().cpu().numpy()
    _, _, inc_off = bp.instances()
    sample = sorted(set([0, 1, 2, 3, n - 2, n - 1]) & set(range(n)))
    del bs
    torch.cuda.empty_cache()
    plain_ms, plain_plan_s, equal = 0.0, 0.0, 0
    kp = args.batch_plain_iters
    for k, pr in enumerate(probs if kp > 0 else []):
        tp = time.perf_counter()
        p = B.Plan(pr)
        plain_plan_s += time.perf_counter() - tp
        s = B.Solver(p)
        s.iterate(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.iterate(kp)
        torch.cuda.synchronize()
        plain_ms += (time.perf_counter() - t0) * 1e3 / kp
        if k in sample:
            s.reset()
            s.iterate(Tc)
            lam_p = s.get_lambda().cpu().numpy()
            equal += int(np.array_equal(lam_p, lam_b[inc_off[k]:inc_off[k + 1]]))
        del s, p
    torch.cuda.empty_cache()
    arcs = 2.0 * st.n_arcs_live
    model = 40.0 * st.n_nodes + 16.0 * st.n_incidences
    cpu = _BATCH_CPU.get("result")
    return {"workload": f"batch{n}: tomography P~U{{32..128}} (even positions) + tracking D~U{{200..2000}}",
            "instances": n, "n_nodes": int(st.n_nodes), "n_incidences": int(st.n_incidences),
            "waves_per_pass": [int(st.waves_fwd), int(st.waves_bwd)],
            "launch": f"wave groups: {G} consecutive waves per launch (launch mode 3), latest waves (wave_align 1)",
            "batched_ms_per_iter": batched_ms, "plain_ms_per_iter": plain_ms,
            "wave_launch_ms_per_iter": wave_ms, "wave_launch_roofline": wave_roofline,
            "speedup": plain_ms / batched_ms if kp > 0 else None,
            "batched_arc_updates_per_s": arcs / (batched_ms * 1e-3),
            "plain_arc_updates_per_s": arcs / (plain_ms * 1e-3) if kp > 0 else None,
            "batched_model_gbps": model / (batched_ms * 1e-3) / 1e9,
            "roofline": roofline,
            "dataflow_launch_ms_per_iter": dataflow_ms,
            "timed_iters": {"batched": T, "plain_per_instance": kp},
            "bitwise_equal_instances": f"{equal}/{len(sample)} sampled after {Tc} iterations",
            "host_build_s": {"generate": gen_s, "batched_plan": plan_s, "plain_plans": plain_plan_s},
            "cpu_oracle": cpu}


def _oracle_instance(q, iters=3):
    """One instance through the fp64 oracle (a worker process): build and init untimed, then iters
    timed iterations; returns (arc-updates done, seconds)."""
    from oracle import Oracle

    o = Oracle(q)
    o.init()
    t = time.perf_counter()
    o.iterate(iters)
    return 2.0 * o.n_live_arcs * iters, time.perf_counter() - t


def host_cpu():
    """The host's processor model and logical core count, recorded beside each CPU figure."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count() or 1}


def batched_cpu_oracle(insts):
    """The oracle on a bounded sample of the batched instances, one instance per host core (at most
    16), all running at once: arc-updates of the timed iterations over the longest worker's iteration
    time."""
    import multiprocessing as mp

    cores = min(os.cpu_count() or 1, 16, len(insts))
    step = max(1, len(insts) // cores)
    sample = insts[::step][:cores]
    t = time.perf_counter()
    with mp.get_context("spawn").Pool(cores) as pool:
        res = pool.map(_oracle_instance, sample)
    wall = time.perf_counter() - t
    done = sum(r[0] for r in res)
    longest = max(r[1] for r in res)
    return {"value": done / longest, "unit": "arc-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"{len(sample)} of {len(insts)} instances (every {step}-th), 3 fp64 iterations each after "
                      f"build and init, one process per instance, rate over the longest worker's iterations; "
                      f"the batched GPU rate is over all {len(insts)} instances",
            "wall_s": wall, "host": host_cpu()}


def split_vs_plain(args, B, I, torch):
    """Sec. 6 sub-BDD split on the batched workload: each instance's variables cut into K intervals
    of about equal node count, fewer dependency waves per pass, copy-arc updates between the passes.
    Per K: waves, time per iteration, and the iterations and time until the bound reaches the one the
    unsplit schedule has after --split-iters iterations (the split converges per iteration more
    slowly, each iteration is shorter)."""
    import numpy as np

    n = args.batch_instances
    probs = [B.Problem.from_ilp(q) for q in batch_instances(I, n)[0]]
    T = args.split_iters
    ks = [int(k) for k in args.split_k.split(",") if k]

    def run(K, iters):
        t = time.perf_counter()
        plan = B.Plan(probs, hist_cap=max(4096, iters + 8), n_intervals=K)
        plan_s = time.perf_counter() - t
        st = plan.stats
        s = B.Solver(plan)
        s.iterate(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.iterate(10)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / 10
        s.reset()
        s.iterate(iters)
        hist = s.lb_history(iters + 1)
        torch.cuda.synchronize()
        del s
        torch.cuda.empty_cache()
        return st, ms, hist, plan_s

    marks = [t for t in (1, 5, 10, 20, 50, 100, 200) if t <= T]
    st0, ms0, h0, _ = run(0, T)
    # target: within 1e-4 (relative) of the unsplit schedule's bound after T iterations
    target = float(h0[-1]) - 1e-4 * max(abs(float(h0[-1])), 1.0)
    it0 = int(np.nonzero(h0 >= target)[0][0])
    out = {"workload": f"batch{n} (as batched_vs_plain)", "reference_iters": T,
           "reference_bound": float(h0[-1]), "target": target,
           "plain": {"waves_per_pass": [int(st0.waves_fwd), int(st0.waves_bwd)], "ms_per_iter": ms0,
                     "iters_to_target": it0, "ms_to_target": it0 * ms0,
                     "bound_at": {t: float(h0[t]) for t in marks}}, "split": []}
    log(f"[bench] split: plain {st0.waves_fwd} waves, {ms0:.2f} ms/iter, bound {h0[-1]:.6g} after {T}, "
        f"target at {it0} iterations")
    for K in ks:
        st, ms, h, plan_s = run(K, args.split_max_iters)
        hit = np.nonzero(h >= target)[0]
        it = int(hit[0]) if hit.size else None
        rec = {"n_intervals": K, "waves_per_pass": [int(st.waves_fwd), int(st.waves_bwd)],
               "n_cuts": int(st.n_cuts), "n_copy_pairs": int(st.n_copy_pairs), "ms_per_iter": ms,
               "bound_at": {t: float(h[t]) for t in marks}, "iters_to_target": it,
               "ms_to_target": None if it is None else it * ms, "plan_s": plan_s}
        out["split"].append(rec)
        log(f"[bench] split K={K}: {st.waves_fwd} waves, {ms:.2f} ms/iter, target at {it} iterations")
    return out


def smoothed_vs_plain(args, B, I, torch):
    """The differentiable form: smoothed DBCA forward (T iterations with per-iteration multiplier
    checkpoints) and its adjoint (d LB_alpha / d c), against plain min-plus iterations on the same
    instance (Potts 128x128, 4 labels)."""
    ilp = I.config(5)
    T = args.smooth_iters
    plan = B.Plan(B.Problem.from_ilp(ilp), hist_cap=max(4096, T + 8))
    st = plan.stats
    s = B.Solver(plan)
    nb = B.bddmp_smooth_workspace_bytes(plan.h, T)
    ws = torch.empty(max(nb, 256), dtype=torch.uint8, device="cuda")
    grad = torch.empty(max(int(st.n_vars), 1), dtype=torch.float32, device="cuda")

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / reps

    plain_ms = timed(lambda: (B.bddmp_solver_reset(s.h), B.bddmp_solver_iterate(s.h, T))) / T
    out = {"workload": "potts128x128_L4", "iterations": T, "n_nodes": int(st.n_nodes),
           "n_incidences": int(st.n_incidences), "workspace_bytes": nb, "plain_ms_per_iter": plain_ms,
           "alphas": {}}
    for alpha in (1.0, 0.1, 0.01):
        fwd = timed(lambda: B.bddmp_solver_smooth_run(s.h, alpha, T, ws, nb))
        lb = float(s.lb_history(1)[-1])
        bwd = timed(lambda: B.bddmp_solver_smooth_grad(s.h, alpha, T, ws, nb, 1.0, grad))
        out["alphas"][str(alpha)] = {"forward_ms": fwd, "adjoint_ms": bwd, "forward_ms_per_iter": fwd / T,
                                     "adjoint_over_forward": bwd / fwd, "smoothed_over_plain": fwd / T / plain_ms,
                                     "lb_alpha": lb,
                                     "grad_abs_sum": float(grad[:int(st.n_vars)].abs().sum())}
    del s, ws, grad
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="potts256x256_L8", choices=sorted(WORKLOADS))
    ap.add_argument("--iters", type=int, default=0, help="iterations per step (default: the workload's)")
    ap.add_argument("--profile-iters", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-vs-plain comparison")
    ap.add_argument("--no-smoothed", action="store_true", help="skip the smoothed-vs-plain comparison")
    ap.add_argument("--smooth-iters", type=int, default=50)
    ap.add_argument("--no-split", action="store_true", help="skip the split-vs-plain comparison")
    ap.add_argument("--split-k", default="4", help="interval counts of the split comparison")
    ap.add_argument("--split-iters", type=int, default=100)
    ap.add_argument("--split-max-iters", type=int, default=300)
    ap.add_argument("--only", choices=["batched", "smoothed", "split"], default=None,
                    help="run only this comparison and print its object (profiling)")
    ap.add_argument("--batch-instances", type=int, default=256)
    ap.add_argument("--launch-probe-iters", type=int, default=50,
                    help="iterations timed per launch form before the main workload's run")
    ap.add_argument("--batch-iters", type=int, default=20)
    ap.add_argument("--batch-group-waves", type=int, default=256,
                    help="consecutive waves per wave-group launch in the batched leg (1..256)")
    ap.add_argument("--batch-plain-iters", type=int, default=3,
                    help="timed iterations per instance of the one-by-one comparison (0: skip it)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run one plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}, WORLD_SIZE {world}); this build has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2009_00481_amd import binding as B
    from paper_2009_00481_amd import instances as I

    # the oracle baseline of the batched workload runs in worker processes: start them before this
    # process touches the GPU
    if not args.no_batched and not args.no_cpu_baseline and args.only in (None, "batched"):
        _BATCH_CPU["result"] = batched_cpu_oracle(batch_instances(I, args.batch_instances)[0])

    if args.copy_probe_mib:
        # a plain copy kernel of known size: reads and writes copy_probe_mib MiB once each
        src = torch.ones(args.copy_probe_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.only:
        torch.cuda.set_device(0)
        fn = {"batched": batched_vs_plain, "smoothed": smoothed_vs_plain, "split": split_vs_plain}[args.only]
        print(json.dumps({args.only: fn(args, B, I, torch)}), flush=True)
        return

    cfg, T = WORKLOADS[args.workload]
    if args.iters:
        T = args.iters
    torch.cuda.set_device(0)

    t = time.perf_counter()
    ilp = I.config(cfg)
    gen_s = time.perf_counter() - t
    t = time.perf_counter()
    plan = B.Plan(B.Problem.from_ilp(ilp), hist_cap=max(4096, T + 8))
    plan_s = time.perf_counter() - t
    st = plan.stats
    log(f"[bench] {args.workload}: n={st.n_vars} m={st.n_bdds} nodes={st.n_nodes} incidences={st.n_incidences} "
        f"live arcs={st.n_arcs_live} waves={st.waves_fwd}+{st.waves_bwd} plan {plan_s:.2f}s")
    t = time.perf_counter()
    s = B.Solver(plan)
    torch.cuda.synchronize()
    bind_s = time.perf_counter() - t

    # launch form: one launch per wave, or every wave of a pass in one wave-group launch with one
    # or (plans whose layers are all narrow) two tiles per workgroup (the same results bitwise); the
    # fastest on a short burst of iterations is kept
    forms = {"waves": (0, 0, "wave_kernel", ""), "wave_groups": (3, 4096, "group_kernel", "group_"),
             "wave_group_pairs": (4, 4096, "group_pair_kernel", "pair_")}
    if int(st.max_width) > 2:
        del forms["wave_group_pairs"]
    form_ms = {}
    for name, (mode, chunk, _, _) in forms.items():
        s.set_launch(mode, chunk)
        s.iterate(3)
        torch.cuda.synchronize()
        t = time.perf_counter()
        s.iterate(args.launch_probe_iters)
        torch.cuda.synchronize()
        form_ms[name] = (time.perf_counter() - t) * 1e3 / args.launch_probe_iters
    launch = min(form_ms, key=form_ms.get)
    mode, chunk, kname, tprefix = forms[launch]
    s.set_launch(mode, chunk)
    log(f"[bench] launch forms (ms per iteration): {form_ms}; using {launch}")

    I_ = int(st.n_incidences)
    m0 = torch.empty(max(I_, 1), dtype=torch.float32, device="cuda")
    m1 = torch.empty_like(m0)
    Mv = torch.empty(max(int(st.n_vars), 1), dtype=torch.float32, device="cuda")

    def step():
        B.bddmp_solver_reset(s.h)
        B.bddmp_solver_iterate(s.h, T)
        B.bddmp_solver_min_marginals(s.h, m0, m1)
        return B.bddmp_solver_round_primal(s.h, Mv, int(st.n_vars))

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # pass times (HIP events around each whole pass, on the solver's stream) for the roofline
    kt = s.time_kernels(args.profile_iters)
    log(f"[bench] kernel times over {args.profile_iters} iterations: {kt}")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = None
    for _ in range(args.steps):
        out = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    hist = s.lb_history(T + 1)
    x, obj, nviol = out

    arc_updates = 2.0 * st.n_arcs_live * T
    value = arc_updates / (ms_per_step * 1e-3)
    pass_bytes = 20.0 * st.n_nodes + 8.0 * st.n_incidences
    iter_bytes = 2 * pass_bytes
    iter_ms = kt["iter_ms"]
    gbps_iter = iter_bytes / (iter_ms * 1e-3) / 1e9 if iter_ms > 0 else None

    roofline = roofline_of(kt, committed_traffic(args.workload, tprefix), kname)

    # time to bound: first t with LB_t >= LB* - 1e-4 max(|LB*|, 1). LB* is the fp64 oracle's LB_T on
    # the same instance when it is stored for T iterations, else this run's own LB_T. Measured with
    # HIP events recorded on the solver's stream after every iteration of a separate run from the
    # reset (no host synchronisation in the loop); the reset itself is not counted.
    lb_self = float(hist[-1])
    ref = oracle_bounds(args.workload, T)
    lb_star = float(ref[-1]) if ref is not None else lb_self
    thr = lb_star - 1e-4 * max(abs(lb_star), 1.0)
    hit = hist >= thr
    t_hit = int(np.argmax(hit)) if hit.any() else None
    ttb_ms = None
    if t_hit is not None:
        stream = torch.cuda.current_stream()
        B.bddmp_solver_reset(s.h)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(t_hit + 1)]
        ev[0].record(stream)
        for t in range(1, t_hit + 1):
            B.bddmp_solver_iterate(s.h, 1)
            ev[t].record(stream)
        torch.cuda.synchronize()
        ttb_ms = ev[0].elapsed_time(ev[t_hit])
        h_ev = s.lb_history(t_hit + 1)
        assert np.array_equal(h_ev, hist[:t_hit + 1]), "per-iteration run differs from the step's trajectory"
    vs_oracle = None
    if ref is not None:
        gap = (hist - ref) / np.maximum(np.abs(ref), 1.0)
        vs_oracle = {"oracle_lb_T": lb_star, "gpu_lb_T": lb_self, "rel_gap_T": float(gap[-1]),
                     "max_abs_rel_gap": float(np.abs(gap).max()),
                     "oracle_iters_to_bound": int(np.argmax(ref >= thr)) if (ref >= thr).any() else None}

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import Oracle

        log("[bench] cpu baseline: oracle build")
        tb = time.perf_counter()
        o = Oracle(ilp)
        build_cpu_s = time.perf_counter() - tb
        ti = time.perf_counter()
        o.init()
        init_cpu_s = time.perf_counter() - ti
        done = 0
        tc = time.perf_counter()
        while done < 2 or (time.perf_counter() - tc) < args.cpu_seconds:
            o.iterate(1)
            done += 1
            if done >= T:
                break
        cpu_s = time.perf_counter() - tc
        cpu_rate = 2.0 * st.n_arcs_live * done / cpu_s
        cpu = {"value": cpu_rate, "unit": "arc-updates/s", "cores": 1, "kind": "oracle",
               "sample": f"{done} fp64 iterations of the same {args.workload} instance after its init "
                         f"(oracle BDD build {build_cpu_s:.1f}s and init {init_cpu_s:.2f}s not in the rate)",
               "s_per_iter": cpu_s / done, "host": host_cpu()}
        del o

    # primal heuristic (Sec. 4, host) from the last step's total min-marginal differences
    t = time.perf_counter()
    Mh = Mv[:int(st.n_vars)].cpu().numpy()
    # order S_i = -M_i: fixes preferred ones first (Sec. 4); on the Potts workloads the |M_i| order
    # fixes many pairwise zeros first and then dead-ends on label cycles that no single row sees
    xs, obj_s, feas_s, implied_s = plan.primal_search(Mh, 1)
    search = {"score": "-M_i", "feasible": bool(feas_s), "objective": obj_s if feas_s else None,
              "implied_by_propagation": int(implied_s), "host_s": time.perf_counter() - t,
              "sign_rounding": {"objective": obj, "violated_rows": int(nviol)}}
    log(f"[bench] primal search: {search}")

    smoothed = None
    if not args.no_smoothed:
        smoothed = smoothed_vs_plain(args, B, I, torch)
        log(f"[bench] smoothed vs plain: {json.dumps(smoothed['alphas'])}")

    batched = None
    if not args.no_batched:
        del s
        torch.cuda.empty_cache()
        batched = batched_vs_plain(args, B, I, torch)
        log(f"[bench] batched vs plain: {batched['batched_ms_per_iter']:.2f} vs {batched['plain_ms_per_iter']:.1f} ms/iter")

    split = None
    if not args.no_split:
        torch.cuda.empty_cache()
        split = split_vs_plain(args, B, I, torch)

    rec = {
        "metric": METRIC, "value": value, "unit": "arc-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "iterations_per_step": T, "n_vars": int(st.n_vars),
                   "n_bdds": int(st.n_bdds), "n_nodes": int(st.n_nodes), "n_incidences": int(st.n_incidences),
                   "n_arcs_live": int(st.n_arcs_live), "waves_per_pass": [int(st.waves_fwd), int(st.waves_bwd)],
                   "bound_dtype": "f64",
                   "launch": {"waves": "one launch per wave (launch mode 0)",
                              "wave_groups": "every wave of a pass in one wave-group launch (launch mode 3)",
                              "wave_group_pairs": "every wave of a pass in one wave-group launch, two tiles per "
                                                  "workgroup (launch mode 4)"}[launch]},
        "launch_probe_ms_per_iter": form_ms,
        "hbm_gbps_per_iter": gbps_iter, "iter_ms": iter_ms, "model_bytes_per_iter": iter_bytes,
        "time_to_bound_1e-4_ms": ttb_ms, "time_to_bound_iters": t_hit,
        "time_to_bound_from_iter_ms": None if t_hit is None else t_hit * iter_ms,
        "lb_star_source": "oracle fp64 LB_T" if ref is not None else "this run's LB_T",
        "bound_vs_oracle": vs_oracle, "lb_final": lb_self, "lb_0": float(hist[0]),
        "primal_obj": obj, "primal_violated_rows": int(nviol), "primal_search": search,
        "host_build_s": {"generate": gen_s, "plan": plan_s, "bind_upload": bind_s},
        "roofline": roofline, "cpu_baseline": cpu,
        "batched_vs_plain": batched,
        "smoothed_vs_plain": smoothed,
        "split_vs_plain": split,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
