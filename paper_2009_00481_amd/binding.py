"""Thin Python binding of the bddmp C-ABI (``include/bddmp.h``).

Functions carry the C names and only marshal arguments: every step of the
method runs inside ``libbddmp.so`` (host builder and planner, HIP kernels).
PyTorch supplies device memory (the solver arena, output tensors) and the
stream. There is no fallback: if the library is missing, loading fails loudly.

``Problem``, ``Plan`` and ``Solver`` are small owners of the handles on top of
those functions.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbddmp.so")
# BDDMP_HOST_ONLY_LIB names the host-only sanitizer test build (build.build_host_only): the host
# calls are the library's own, every device call fails with DEVICE; no HIP runtime is loaded
HOST_ONLY_LIB = os.environ.get("BDDMP_HOST_ONLY_LIB")

BDDMP_OK = 0
STATUS = {-1: "INVALID_ARG", -2: "ROW_INFEASIBLE", -3: "BDD_TOO_LARGE", -4: "NOT_INTEGER", -5: "CONFLICT",
          -6: "DEVICE", -7: "BAD_STATE", -8: "NONFINITE"}


class BddmpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"bddmp {STATUS.get(code, code)} ({code}): {msg}")
        self.code = code


class Options(C.Structure):
    _fields_ = [("order_mode", C.c_int32), ("hist_cap", C.c_int32), ("node_budget", C.c_int64),
                ("tile_work", C.c_int32), ("tiling", C.c_char_p), ("n_intervals", C.c_int32),
                ("split_gamma", C.c_float), ("wave_align", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("n_vars", C.c_int64), ("n_bdds", C.c_int64), ("n_nodes", C.c_int64), ("n_arcs_live", C.c_int64),
                ("n_arcs_bot", C.c_int64), ("n_incidences", C.c_int64), ("waves_fwd", C.c_int32),
                ("waves_bwd", C.c_int32), ("device_bytes", C.c_int64), ("max_width", C.c_int32),
                ("n_shapes", C.c_int32), ("max_rows_per_var", C.c_int32), ("bwd_contiguous", C.c_int32),
                ("fwd_tiles", C.c_int64), ("bwd_tiles", C.c_int64), ("n_instances", C.c_int32),
                ("n_intervals", C.c_int32), ("n_cuts", C.c_int64), ("n_copy_pairs", C.c_int64),
                ("fused_turn", C.c_int32), ("fused_wrap", C.c_int32), ("dataflow", C.c_int32),
                ("max_tile_deps", C.c_int32), ("n_groups", C.c_int32), ("tile_deps_fwd", C.c_int64),
                ("tile_deps_bwd", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class KernelTimes(C.Structure):
    _fields_ = [("fwd_ms", C.c_double), ("bwd_ms", C.c_double), ("lb_ms", C.c_double),
                ("fwd_launches", C.c_int64), ("bwd_launches", C.c_int64), ("lb_launches", C.c_int64),
                ("fwd_bytes", C.c_double), ("bwd_bytes", C.c_double), ("iter_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# every symbol the header declares, with (restype, argtypes)
_P, _I32, _I64, _D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
SIGNATURES = {
    "bddmp_version": (_I32, []),
    "bddmp_last_error": (C.c_char_p, []),
    "bddmp_options_default": (_I32, [C.POINTER(Options)]),
    "bddmp_problem_create": (_I32, [_I32, _P, C.POINTER(_P)]),
    "bddmp_problem_add_rows": (_I32, [_P, _I32, _P, _P, _P, _P, _P]),
    "bddmp_problem_add_rows_real": (_I32, [_P, _I32, _P, _P, _P, _P, _P]),
    "bddmp_problem_set_order": (_I32, [_P, _P]),
    "bddmp_plan_create": (_I32, [_P, C.POINTER(Options), C.POINTER(_P)]),
    "bddmp_plan_create_batch": (_I32, [_P, _I32, C.POINTER(Options), C.POINTER(_P)]),
    "bddmp_plan_instances": (_I32, [_P, _P, _P, _P]),
    "bddmp_plan_primal_search": (_I32, [_P, _P, _I32, _I64, _P, C.POINTER(_D), C.POINTER(_I32), C.POINTER(_I64)]),
    "bddmp_plan_restrict_row": (_I32, [_P, _I32, _I32, _P, _P, _P, _P, _P, C.POINTER(_I32)]),
    "bddmp_plan_stats": (_I32, [_P, C.POINTER(Stats)]),
    "bddmp_plan_export_order": (_I32, [_P, _P]),
    "bddmp_plan_export_structure": (_I32, [_P, _P, _P, _P, _P]),
    "bddmp_plan_export_waves": (_I32, [_P, _P, _P]),
    "bddmp_plan_digest": (_I32, [_P, _P]),
    "bddmp_plan_export_tile_deps": (_I32, [_P, _I32, _P, _P, _P]),
    "bddmp_plan_export_wave_split": (_I32, [_P, _I32, _P, _P, _P]),
    "bddmp_solver_bind": (_I32, [_P, _P, C.c_size_t, _P, C.POINTER(_P)]),
    "bddmp_solver_reset": (_I32, [_P]),
    "bddmp_solver_iterate": (_I32, [_P, _I32]),
    "bddmp_solver_lower_bound": (_I32, [_P, C.POINTER(_D), C.POINTER(_D), C.POINTER(_D)]),
    "bddmp_solver_instance_bounds": (_I32, [_P, _P, _I32]),
    "bddmp_solver_lb_history": (_I32, [_P, _P, _I32, C.POINTER(_I32)]),
    "bddmp_solver_min_marginals": (_I32, [_P, _P, _P]),
    "bddmp_solver_get_lambda": (_I32, [_P, _P]),
    "bddmp_solver_set_lambda": (_I32, [_P, _P]),
    "bddmp_solver_iterate_until": (_I32, [_P, _I32, _D, _I32, C.POINTER(_I32), C.POINTER(_I32), C.POINTER(_D)]),
    "bddmp_solver_get_copy_duals": (_I32, [_P, _P, _P, _P, _P]),
    "bddmp_solver_set_copy_duals": (_I32, [_P, _P, _P, _P, _P]),
    "bddmp_solver_round_primal": (_I32, [_P, _P, _P, C.POINTER(_D), C.POINTER(_I64)]),
    "bddmp_smooth_workspace_bytes": (_I32, [_P, _I32, C.POINTER(C.c_size_t)]),
    "bddmp_solver_smooth_run": (_I32, [_P, C.c_float, _I32, _P, C.c_size_t]),
    "bddmp_solver_smooth_grad": (_I32, [_P, C.c_float, _I32, _P, C.c_size_t, _D, _P]),
    "bddmp_solver_smooth_grad_noalloc": (_I32, [_P, C.c_float, _I32, _D, _P]),
    "bddmp_solver_set_costs": (_I32, [_P, _P]),
    "bddmp_solver_set_graphs": (_I32, [_P, _I32]),
    "bddmp_solver_set_launch": (_I32, [_P, _I32, _I32]),
    "bddmp_solver_get_launch": (_I32, [_P, C.POINTER(_I32), C.POINTER(_I32)]),
    "bddmp_solver_set_groups": (_I32, [_P, _P]),
    "bddmp_solver_get_groups": (_I32, [_P, _P]),
    "bddmp_solver_autotune": (_I32, [_P, _I32, _P]),
    "bddmp_solver_time_kernels": (_I32, [_P, _I32, C.POINTER(KernelTimes)]),
    "bddmp_solver_destroy": (None, [_P]),
    "bddmp_plan_destroy": (None, [_P]),
    "bddmp_problem_destroy": (None, [_P]),
}

_lib = None


def lib():
    """Load libbddmp.so (built in-tree by ``paper_2009_00481_amd/build.py``); raise if missing."""
    global _lib
    if _lib is None:
        path = HOST_ONLY_LIB or LIB_PATH
        if not HOST_ONLY_LIB:
            # torch first: its HIP runtime carries the soname the library links against, so the
            # library binds to that same runtime (one runtime, one device context, shared streams).
            # Loaded the other way round, the process would hold two HIP runtimes.
            import torch  # noqa: F401

        if not os.path.exists(path):
            raise ImportError(f"{path} is not built; run paper_2009_00481_amd/build.py "
                              "(the HIP library has no fallback)")
        L = C.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != BDDMP_OK:
        raise BddmpError(rc, lib().bddmp_last_error().decode())


def _ptr(a):
    return C.c_void_p(a.ctypes.data) if a is not None else None


def _dptr(t):
    """Device pointer of a torch tensor (or None)."""
    return C.c_void_p(t.data_ptr()) if t is not None else None


# ---------------------------------------------------------------------------
# C entry points, same names
# ---------------------------------------------------------------------------

def bddmp_version() -> int:
    return int(lib().bddmp_version())


def bddmp_options_default() -> Options:
    o = Options()
    _check(lib().bddmp_options_default(C.byref(o)))
    return o


def bddmp_problem_create(n_vars: int, cost) -> C.c_void_p:
    cost = np.ascontiguousarray(cost, np.float64)
    assert cost.shape == (n_vars,)
    h = C.c_void_p()
    _check(lib().bddmp_problem_create(int(n_vars), _ptr(cost), C.byref(h)))
    return h


def bddmp_problem_add_rows(h, row_ptr, col, coef, sense, rhs):
    row_ptr = np.ascontiguousarray(row_ptr, np.int64)
    col = np.ascontiguousarray(col, np.int32)
    coef = np.ascontiguousarray(coef, np.int64)
    sense = np.ascontiguousarray(sense, np.int8)
    rhs = np.ascontiguousarray(rhs, np.int64)
    n_rows = int(row_ptr.shape[0] - 1)
    _check(lib().bddmp_problem_add_rows(h, n_rows, _ptr(row_ptr), _ptr(col) if col.size else None,
                                        _ptr(coef) if coef.size else None, _ptr(sense), _ptr(rhs)))


def bddmp_problem_add_rows_real(h, row_ptr, col, coef, sense, rhs):
    row_ptr = np.ascontiguousarray(row_ptr, np.int64)
    col = np.ascontiguousarray(col, np.int32)
    coef = np.ascontiguousarray(coef, np.float64)
    sense = np.ascontiguousarray(sense, np.int8)
    rhs = np.ascontiguousarray(rhs, np.float64)
    n_rows = int(row_ptr.shape[0] - 1)
    _check(lib().bddmp_problem_add_rows_real(h, n_rows, _ptr(row_ptr), _ptr(col) if col.size else None,
                                             _ptr(coef) if coef.size else None, _ptr(sense), _ptr(rhs)))


def bddmp_problem_set_order(h, perm):
    if perm is None:
        _check(lib().bddmp_problem_set_order(h, None))
        return
    perm = np.ascontiguousarray(perm, np.int32)
    _check(lib().bddmp_problem_set_order(h, _ptr(perm)))


def bddmp_plan_create(problem, options: Options | None = None):
    h = C.c_void_p()
    _check(lib().bddmp_plan_create(problem, C.byref(options) if options is not None else None, C.byref(h)))
    return h


def bddmp_plan_create_batch(problems, options: Options | None = None):
    arr = (C.c_void_p * len(problems))(*[p.value if isinstance(p, C.c_void_p) else p for p in problems])
    h = C.c_void_p()
    _check(lib().bddmp_plan_create_batch(C.cast(arr, C.c_void_p), len(problems),
                                         C.byref(options) if options is not None else None, C.byref(h)))
    return h


def bddmp_plan_instances(plan, n_inst: int):
    v = np.zeros(n_inst + 1, np.int64)
    r = np.zeros(n_inst + 1, np.int64)
    c = np.zeros(n_inst + 1, np.int64)
    _check(lib().bddmp_plan_instances(plan, _ptr(v), _ptr(r), _ptr(c)))
    return v, r, c


def bddmp_plan_primal_search(plan, M, n: int, score_mode: int = 0, max_dead_ends: int = 100000):
    M = np.ascontiguousarray(M, np.float32)
    assert M.shape == (n,)
    x = np.zeros(max(n, 1), np.int8)
    obj, feas, imp = C.c_double(), C.c_int32(), C.c_int64()
    _check(lib().bddmp_plan_primal_search(plan, _ptr(M), int(score_mode), int(max_dead_ends), _ptr(x), C.byref(obj),
                                          C.byref(feas), C.byref(imp)))
    return x[:n], obj.value, bool(feas.value), imp.value


def bddmp_plan_restrict_row(plan, row: int, n_nodes: int, vars_, vals):
    vars_ = np.ascontiguousarray(vars_, np.int32)
    vals = np.ascontiguousarray(vals, np.int8)
    alive = np.zeros(max(n_nodes, 1), np.uint8)
    lo = np.zeros(max(n_nodes, 1), np.int32)
    hi = np.zeros(max(n_nodes, 1), np.int32)
    feas = C.c_int32()
    _check(lib().bddmp_plan_restrict_row(plan, int(row), int(vars_.shape[0]), _ptr(vars_) if vars_.size else None,
                                         _ptr(vals) if vals.size else None, _ptr(alive), _ptr(lo), _ptr(hi),
                                         C.byref(feas)))
    return alive[:n_nodes].astype(bool), lo[:n_nodes], hi[:n_nodes], bool(feas.value)


def bddmp_plan_stats(plan) -> Stats:
    s = Stats()
    _check(lib().bddmp_plan_stats(plan, C.byref(s)))
    return s


def bddmp_plan_export_order(plan, n: int):
    out = np.zeros(max(n, 1), np.int32)
    _check(lib().bddmp_plan_export_order(plan, _ptr(out)))
    return out[:n]


def bddmp_plan_export_structure(plan, n_incidences: int, n_nodes: int):
    w = np.zeros(max(n_incidences, 1), np.int32)
    v = np.zeros(max(n_incidences, 1), np.int32)
    lo = np.zeros(max(n_nodes, 1), np.int32)
    hi = np.zeros(max(n_nodes, 1), np.int32)
    _check(lib().bddmp_plan_export_structure(plan, _ptr(w), _ptr(v), _ptr(lo), _ptr(hi)))
    return w[:n_incidences], v[:n_incidences], lo[:n_nodes], hi[:n_nodes]


def bddmp_plan_export_waves(plan, n: int):
    f = np.zeros(max(n, 1), np.int32)
    b = np.zeros(max(n, 1), np.int32)
    _check(lib().bddmp_plan_export_waves(plan, _ptr(f), _ptr(b)))
    return f[:n], b[:n]


def bddmp_plan_digest(plan) -> int:
    d = np.zeros(1, np.uint64)
    _check(lib().bddmp_plan_digest(plan, _ptr(d)))
    return int(d[0])


def bddmp_plan_export_tile_deps(plan, pass_: int, n_tiles: int, n_deps: int):
    ptr = np.zeros(n_tiles + 1, np.int32)
    lst = np.zeros(max(n_deps, 1), np.int32)
    grp = np.zeros(max(n_tiles, 1), np.int32)
    _check(lib().bddmp_plan_export_tile_deps(plan, int(pass_), _ptr(ptr), _ptr(lst), _ptr(grp)))
    return ptr, lst[:n_deps], grp[:n_tiles]


def bddmp_plan_export_wave_split(plan, pass_: int, n_waves: int):
    begin = np.zeros(n_waves + 1, np.int32)
    mid = np.zeros(max(n_waves, 1), np.int32)
    bw = np.zeros(max(n_waves, 1), np.int32)
    _check(lib().bddmp_plan_export_wave_split(plan, int(pass_), _ptr(begin), _ptr(mid), _ptr(bw)))
    return begin, mid[:n_waves], bw[:n_waves]


def bddmp_solver_bind(plan, arena, nbytes: int, stream):
    h = C.c_void_p()
    _check(lib().bddmp_solver_bind(plan, _dptr(arena), C.c_size_t(int(nbytes)), C.c_void_p(stream), C.byref(h)))
    return h


def bddmp_solver_reset(h):
    _check(lib().bddmp_solver_reset(h))


def bddmp_solver_iterate(h, n_iters: int):
    _check(lib().bddmp_solver_iterate(h, int(n_iters)))


def bddmp_solver_lower_bound(h):
    lb, r, b = C.c_double(), C.c_double(), C.c_double()
    _check(lib().bddmp_solver_lower_bound(h, C.byref(lb), C.byref(r), C.byref(b)))
    return lb.value, r.value, b.value


def bddmp_solver_instance_bounds(h, n_inst: int):
    out = np.zeros(n_inst, np.float64)
    _check(lib().bddmp_solver_instance_bounds(h, _ptr(out), int(n_inst)))
    return out


def bddmp_solver_lb_history(h, cap: int):
    out = np.zeros(max(cap, 1), np.float64)
    n = C.c_int32()
    _check(lib().bddmp_solver_lb_history(h, _ptr(out), int(cap), C.byref(n)))
    return out[: n.value]


def bddmp_solver_min_marginals(h, m0, m1):
    _check(lib().bddmp_solver_min_marginals(h, _dptr(m0), _dptr(m1)))


def bddmp_solver_get_lambda(h, lam):
    _check(lib().bddmp_solver_get_lambda(h, _dptr(lam)))


def bddmp_solver_set_lambda(h, lam):
    _check(lib().bddmp_solver_set_lambda(h, _dptr(lam)))


def bddmp_solver_iterate_until(h, max_iters: int, min_rel_impr: float, check_every: int):
    done, at, lb = C.c_int32(), C.c_int32(), C.c_double()
    _check(lib().bddmp_solver_iterate_until(h, int(max_iters), float(min_rel_impr), int(check_every), C.byref(done),
                                            C.byref(at), C.byref(lb)))
    return done.value, at.value, lb.value


def bddmp_solver_get_copy_duals(h, mu_bar, mu, dfw, dbw):
    _check(lib().bddmp_solver_get_copy_duals(h, _dptr(mu_bar), _dptr(mu), _dptr(dfw), _dptr(dbw)))


def bddmp_solver_set_copy_duals(h, mu_bar, mu, dfw, dbw):
    _check(lib().bddmp_solver_set_copy_duals(h, _dptr(mu_bar), _dptr(mu), _dptr(dfw), _dptr(dbw)))


def bddmp_solver_round_primal(h, M, n: int):
    x = np.zeros(max(n, 1), np.int8)
    obj = C.c_double()
    nv = C.c_int64()
    _check(lib().bddmp_solver_round_primal(h, _dptr(M), _ptr(x), C.byref(obj), C.byref(nv)))
    return x[:n], obj.value, nv.value


def bddmp_smooth_workspace_bytes(plan, n_iters: int) -> int:
    b = C.c_size_t()
    _check(lib().bddmp_smooth_workspace_bytes(plan, int(n_iters), C.byref(b)))
    return int(b.value)


def bddmp_solver_smooth_run(h, alpha: float, n_iters: int, ws, ws_bytes: int):
    _check(lib().bddmp_solver_smooth_run(h, float(alpha), int(n_iters), _dptr(ws), C.c_size_t(int(ws_bytes))))


def bddmp_solver_smooth_grad(h, alpha: float, n_iters: int, ws, ws_bytes: int, dlb: float, grad):
    _check(lib().bddmp_solver_smooth_grad(h, float(alpha), int(n_iters), _dptr(ws), C.c_size_t(int(ws_bytes)),
                                          float(dlb), _dptr(grad)))


def bddmp_solver_smooth_grad_noalloc(h, alpha: float, n_iters: int, dlb: float, grad):
    _check(lib().bddmp_solver_smooth_grad_noalloc(h, float(alpha), int(n_iters), float(dlb), _dptr(grad)))


def bddmp_solver_set_costs(h, cost):
    _check(lib().bddmp_solver_set_costs(h, _dptr(cost)))


def bddmp_solver_set_graphs(h, enable: bool):
    _check(lib().bddmp_solver_set_graphs(h, int(bool(enable))))


def bddmp_solver_set_launch(h, mode: int, chunk: int = 0):
    _check(lib().bddmp_solver_set_launch(h, int(mode), int(chunk)))


def bddmp_solver_get_launch(h):
    m, c = C.c_int32(), C.c_int32()
    _check(lib().bddmp_solver_get_launch(h, C.byref(m), C.byref(c)))
    return m.value, c.value


def bddmp_solver_set_groups(h, lanes):
    arr = np.ascontiguousarray(lanes, np.int32)
    assert arr.shape == (4,)
    _check(lib().bddmp_solver_set_groups(h, _ptr(arr)))


def bddmp_solver_get_groups(h):
    arr = np.zeros(4, np.int32)
    _check(lib().bddmp_solver_get_groups(h, _ptr(arr)))
    return arr


def bddmp_solver_autotune(h, iters: int):
    arr = np.zeros(4, np.int32)
    _check(lib().bddmp_solver_autotune(h, int(iters), _ptr(arr)))
    return arr


def bddmp_solver_time_kernels(h, n_iters: int) -> KernelTimes:
    t = KernelTimes()
    _check(lib().bddmp_solver_time_kernels(h, int(n_iters), C.byref(t)))
    return t


def bddmp_solver_destroy(h):
    lib().bddmp_solver_destroy(h)


def bddmp_plan_destroy(h):
    lib().bddmp_plan_destroy(h)


def bddmp_problem_destroy(h):
    lib().bddmp_problem_destroy(h)


# ---------------------------------------------------------------------------
# owners
# ---------------------------------------------------------------------------

class Problem:
    def __init__(self, n_vars: int, cost):
        self.n = int(n_vars)
        self.h = bddmp_problem_create(self.n, cost)

    @classmethod
    def from_ilp(cls, ilp, order=True) -> "Problem":
        p = cls(ilp.n, ilp.cost)
        bddmp_problem_add_rows(p.h, ilp.row_ptr, ilp.col, ilp.coef, ilp.sense, ilp.rhs)
        if order and ilp.order is not None:
            bddmp_problem_set_order(p.h, ilp.order)
        return p

    def add_rows(self, row_ptr, col, coef, sense, rhs):
        bddmp_problem_add_rows(self.h, row_ptr, col, coef, sense, rhs)

    def set_order(self, perm):
        bddmp_problem_set_order(self.h, perm)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            bddmp_problem_destroy(self.h)
            self.h = None


class Plan:
    """A plan for one problem, or for several independent ones (``problem`` a list: batched)."""

    def __init__(self, problem, order_mode: int = 0, node_budget: int = 0, hist_cap: int = 4096,
                 tiling: str | None = None, tile_work: int = 0, n_intervals: int = 0, split_gamma: float = 0.0,
                 wave_align: int = 0):
        o = bddmp_options_default()
        o.wave_align = wave_align
        o.tile_work = tile_work
        o.n_intervals = n_intervals
        o.split_gamma = split_gamma
        o.order_mode = order_mode
        o.node_budget = node_budget
        o.hist_cap = hist_cap
        self._tiling = tiling.encode() if tiling is not None else None
        o.tiling = self._tiling
        if isinstance(problem, (list, tuple)):
            self.n = sum(p.n for p in problem)
            self.h = bddmp_plan_create_batch([p.h for p in problem], o)
        else:
            self.n = problem.n
            self.h = bddmp_plan_create(problem.h, o)
        self.stats = bddmp_plan_stats(self.h)

    def primal_search(self, M, score_mode: int = 0, max_dead_ends: int = 100000):
        """(x, objective, feasible, n_implied) of the primal heuristic from total differences M."""
        return bddmp_plan_primal_search(self.h, M, self.n, score_mode, max_dead_ends)

    def instances(self):
        """(var_off, row_off, inc_off), each [n_instances + 1]."""
        return bddmp_plan_instances(self.h, int(self.stats.n_instances))

    def order(self):
        return bddmp_plan_export_order(self.h, self.n)

    def structure(self):
        return bddmp_plan_export_structure(self.h, self.stats.n_incidences, self.stats.n_nodes)

    def waves(self):
        return bddmp_plan_export_waves(self.h, self.n)

    def digest(self) -> int:
        """64-bit digest of every array the plan uploads and of its layout sizes."""
        return bddmp_plan_digest(self.h)

    def tile_deps(self, pass_: int):
        """(dep_ptr, dep_list, tile_group) of the dataflow launch's tiles in pass 0 (forward) or 1 (backward)."""
        st = self.stats
        n = int(st.fwd_tiles if pass_ == 0 else st.bwd_tiles)
        return bddmp_plan_export_tile_deps(self.h, pass_, n, int(st.tile_deps_fwd if pass_ == 0 else st.tile_deps_bwd))

    def wave_split(self, pass_: int):
        """(tile_begin [W + 1], mid [W], b_wait [W]) of the two-branch launch of pass 0 or 1."""
        st = self.stats
        return bddmp_plan_export_wave_split(self.h, pass_, int(st.waves_fwd if pass_ == 0 else st.waves_bwd))

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            bddmp_plan_destroy(self.h)
            self.h = None


class Solver:
    """Device solver: the arena is a torch uint8 tensor on ``device``; work runs on ``stream``."""

    def __init__(self, plan: Plan, device="cuda", stream=None):
        import torch

        self.plan = plan
        self.torch = torch
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nbytes = int(plan.stats.device_bytes)
        self.arena = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        self.h = bddmp_solver_bind(plan.h, self.arena, nbytes, self.stream.cuda_stream)

    @property
    def n_incidences(self):
        return int(self.plan.stats.n_incidences)

    def reset(self):
        bddmp_solver_reset(self.h)

    def iterate(self, n_iters: int):
        bddmp_solver_iterate(self.h, n_iters)

    def iterate_until(self, max_iters: int, min_rel_impr: float = 1e-6, check_every: int = 10):
        """(iterations run, first iteration meeting the stop rule or -1, last bound)."""
        return bddmp_solver_iterate_until(self.h, max_iters, min_rel_impr, check_every)

    def lower_bound(self):
        return bddmp_solver_lower_bound(self.h)

    def lb_history(self, cap: int = 1 << 16):
        return bddmp_solver_lb_history(self.h, cap)

    def instance_bounds(self):
        return bddmp_solver_instance_bounds(self.h, int(self.plan.stats.n_instances))

    def min_marginals(self):
        I = self.n_incidences
        m0 = self.torch.empty(max(I, 1), dtype=self.torch.float32, device=self.device)
        m1 = self.torch.empty(max(I, 1), dtype=self.torch.float32, device=self.device)
        bddmp_solver_min_marginals(self.h, m0, m1)
        return m0[:I], m1[:I]

    def get_lambda(self):
        I = self.n_incidences
        lam = self.torch.empty(max(I, 1), dtype=self.torch.float32, device=self.device)
        bddmp_solver_get_lambda(self.h, lam)
        return lam[:I]

    def set_lambda(self, lam):
        assert lam.dtype == self.torch.float32 and lam.is_contiguous() and lam.numel() == self.n_incidences
        bddmp_solver_set_lambda(self.h, lam)

    def copy_duals(self):
        """Copy-arc state of a split plan per pair: (mu_bar, mu, delta_fwd, delta_bwd) device tensors."""
        n = int(self.plan.stats.n_copy_pairs)
        out = [self.torch.empty(max(n, 1), dtype=self.torch.float32, device=self.device) for _ in range(4)]
        bddmp_solver_get_copy_duals(self.h, *out)
        return tuple(t[:n] for t in out)

    def set_copy_duals(self, mu_bar, mu, dfw, dbw):
        n = int(self.plan.stats.n_copy_pairs)
        for t in (mu_bar, mu, dfw, dbw):
            assert t.dtype == self.torch.float32 and t.is_contiguous() and t.numel() >= n
        bddmp_solver_set_copy_duals(self.h, mu_bar, mu, dfw, dbw)

    def round_primal(self):
        n = self.plan.n
        M = self.torch.empty(max(n, 1), dtype=self.torch.float32, device=self.device)
        x, obj, nv = bddmp_solver_round_primal(self.h, M, n)
        return M[:n], x, obj, nv

    def set_graphs(self, enable: bool):
        bddmp_solver_set_graphs(self.h, enable)

    def set_launch(self, mode: int, chunk: int = 0):
        bddmp_solver_set_launch(self.h, mode, chunk)

    def launch(self):
        return bddmp_solver_get_launch(self.h)

    def set_groups(self, lanes):
        bddmp_solver_set_groups(self.h, lanes)

    def groups(self):
        return bddmp_solver_get_groups(self.h)

    def autotune(self, iters: int):
        return bddmp_solver_autotune(self.h, iters)

    def time_kernels(self, n_iters: int) -> dict:
        return bddmp_solver_time_kernels(self.h, n_iters).as_dict()

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            bddmp_solver_destroy(self.h)
            self.h = None
