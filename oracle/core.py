"""ctypes wrapper of the C oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

ORC_CHECK_INCREMENTAL, ORC_CHECK_PROP1, ORC_CHECK_EQUAL_D, ORC_CHECK_SUM_LAMBDA = 1, 2, 4, 8
ORC_CHECK_ALL = 15

_LIBS: dict = {}


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"oracle status {code}: {msg}")
        self.code = code


def _lib(prec: str):
    if prec in _LIBS:
        return _LIBS[prec]
    path = _build.TARGETS[prec]
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
        _build.build(force=False)
    L = C.CDLL(path)
    P, I, LL, D = C.c_void_p, C.c_int, C.c_longlong, C.c_double
    L.orc_create.argtypes = [I, P, I, P, P, P, P, P, P, LL, C.POINTER(P)]
    L.orc_create.restype = I
    L.orc_destroy.argtypes = [P]
    L.orc_stats.argtypes = [P, P]
    L.orc_structure.argtypes = [P, P, P, P, P]
    L.orc_init.argtypes = [P, I]
    L.orc_init.restype = I
    L.orc_set_lambda.argtypes = [P, P]
    L.orc_set_lambda.restype = I
    L.orc_iterate.argtypes = [P, I, P]
    L.orc_iterate.restype = I
    L.orc_lower_bound.argtypes = [P]
    L.orc_lower_bound.restype = D
    L.orc_residual.argtypes = [P, P, P]
    L.orc_lambda.argtypes = [P, P]
    L.orc_min_marginals.argtypes = [P, P, P]
    L.orc_min_marginals.restype = I
    L.orc_round.argtypes = [P, P, P, P, P]
    L.orc_round.restype = I
    L.orc_checks.argtypes = [P, P]
    L.orc_count_solutions.argtypes = [P, P]
    L.orc_error.restype = C.c_char_p
    L.orc_smooth_init.argtypes = [P, D]
    L.orc_smooth_init.restype = I
    L.orc_smooth_iterate.argtypes = [P, D, I, P]
    L.orc_smooth_iterate.restype = I
    L.orc_smooth_marginals.argtypes = [P, D, P, P]
    L.orc_smooth_marginals.restype = I
    L.orc_row_energies.argtypes = [P, D, P, P]
    L.orc_smooth_grad.argtypes = [P, D, I, P, P]
    L.orc_smooth_grad.restype = I
    L.orc_build_row.argtypes = [I, P, I, LL, LL, P, P, P, LL]
    L.orc_build_row.restype = LL
    L.orc_split.argtypes = [P, I, D]
    L.orc_split.restype = I
    L.orc_split_info.argtypes = [P, P, P]
    L.orc_copy_duals.argtypes = [P, P, P, P, P, P, P]
    _LIBS[prec] = L
    return L


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _check(L, rc):
    if rc != 0:
        raise OracleError(rc, L.orc_error().decode())


class Oracle:
    """One problem in the oracle: build, init, iterate, read results (canonical order)."""

    def __init__(self, ilp, precision: str = "f64", node_budget: int = 0, split: int = 0, gamma: float = 0.5):
        self.L = _lib(precision)
        self.precision = precision
        self._keep = [np.ascontiguousarray(ilp.cost, np.float64), np.ascontiguousarray(ilp.row_ptr, np.int64),
                      np.ascontiguousarray(ilp.col, np.int32), np.ascontiguousarray(ilp.coef, np.int64),
                      np.ascontiguousarray(ilp.sense, np.int8), np.ascontiguousarray(ilp.rhs, np.int64),
                      np.ascontiguousarray(ilp.order, np.int32)]
        cost, rp, col, coef, sense, rhs, order = self._keep
        h = C.c_void_p()
        rc = self.L.orc_create(int(ilp.n), _p(cost), int(rp.shape[0] - 1), _p(rp), _p(col), _p(coef), _p(sense),
                               _p(rhs), _p(order), int(node_budget), C.byref(h))
        _check(self.L, rc)
        self.h = h
        st = np.zeros(6, np.int64)
        self.L.orc_stats(self.h, _p(st))
        self.n, self.m, self.n_nodes, self.n_live_arcs, self.n_incidences, self.max_J = (int(v) for v in st)
        if split > 1:
            _check(self.L, self.L.orc_split(self.h, int(split), float(gamma)))

    def split_info(self):
        """(K, cut levels, copy-arc pairs, interval of each variable) of Sec. 6's split."""
        out = np.zeros(3, np.int64)
        intv = np.zeros(max(self.n, 1), np.int32)
        self.L.orc_split_info(self.h, _p(out), _p(intv))
        return int(out[0]), int(out[1]), int(out[2]), intv[:self.n]

    def copy_duals(self):
        """Per copy-arc pair in canonical order: dict of mu_bar, mu, row, level, node, label."""
        n = self.split_info()[2]
        mb, mu = np.zeros(max(n, 1)), np.zeros(max(n, 1))
        r, l, u, b = (np.zeros(max(n, 1), np.int32) for _ in range(4))
        self.L.orc_copy_duals(self.h, _p(mb), _p(mu), _p(r), _p(l), _p(u), _p(b))
        return dict(mu_bar=mb[:n], mu=mu[:n], row=r[:n], level=l[:n], node=u[:n], label=b[:n])

    def __del__(self):
        if getattr(self, "h", None):
            self.L.orc_destroy(self.h)
            self.h = None

    def structure(self):
        """(level_width[I], level_var[I], lo[N], hi[N]) in canonical order; BOT = -1, TOP = -2."""
        w = np.zeros(self.n_incidences, np.int32)
        v = np.zeros(self.n_incidences, np.int32)
        lo = np.zeros(self.n_nodes, np.int32)
        hi = np.zeros(self.n_nodes, np.int32)
        self.L.orc_structure(self.h, _p(w), _p(v), _p(lo), _p(hi))
        return w, v, lo, hi

    def init(self, checks: int = 0) -> float:
        _check(self.L, self.L.orc_init(self.h, int(checks)))
        return self.lower_bound()

    def set_lambda(self, lam):
        lam = np.ascontiguousarray(lam, np.float64)
        assert lam.shape == (self.n_incidences,)
        _check(self.L, self.L.orc_set_lambda(self.h, _p(lam)))

    def iterate(self, iters: int) -> np.ndarray:
        tr = np.zeros(max(iters, 1), np.float64)
        _check(self.L, self.L.orc_iterate(self.h, int(iters), _p(tr)))
        return tr[:iters]

    def lower_bound(self) -> float:
        return float(self.L.orc_lower_bound(self.h))

    def residual(self):
        r = C.c_double()
        b = C.c_double()
        self.L.orc_residual(self.h, C.byref(r), C.byref(b))
        return r.value, b.value

    def lam(self) -> np.ndarray:
        out = np.zeros(self.n_incidences, np.float64)
        self.L.orc_lambda(self.h, _p(out))
        return out

    def min_marginals(self):
        m0 = np.zeros(self.n_incidences, np.float64)
        m1 = np.zeros(self.n_incidences, np.float64)
        _check(self.L, self.L.orc_min_marginals(self.h, _p(m0), _p(m1)))
        return m0, m1

    def round(self):
        M = np.zeros(self.n, np.float64)
        x = np.zeros(self.n, np.int8)
        obj = C.c_double()
        nv = C.c_longlong()
        _check(self.L, self.L.orc_round(self.h, _p(M), _p(x), C.byref(obj), C.byref(nv)))
        return M, x, obj.value, nv.value

    # smoothed variant (App. "Smoothing")
    def smooth_init(self, alpha: float) -> float:
        _check(self.L, self.L.orc_smooth_init(self.h, float(alpha)))
        return self.lower_bound()

    def smooth_iterate(self, alpha: float, iters: int) -> np.ndarray:
        tr = np.zeros(max(iters, 1), np.float64)
        _check(self.L, self.L.orc_smooth_iterate(self.h, float(alpha), int(iters), _p(tr)))
        return tr[:iters]

    def smooth_marginals(self, alpha: float):
        m0 = np.zeros(self.n_incidences, np.float64)
        m1 = np.zeros(self.n_incidences, np.float64)
        _check(self.L, self.L.orc_smooth_marginals(self.h, float(alpha), _p(m0), _p(m1)))
        return m0, m1

    def row_energies(self, alpha: float):
        """(E^j, E^j_alpha) per row at the current multipliers, from scratch."""
        e = np.zeros(max(self.m, 1), np.float64)
        ea = np.zeros(max(self.m, 1), np.float64)
        self.L.orc_row_energies(self.h, float(alpha), _p(e), _p(ea))
        return e[:self.m], ea[:self.m]

    def smooth_grad(self, alpha: float, iters: int):
        """(d LB_alpha(T) / d c, LB_alpha(T)) after T smoothed iterations from the initialisation."""
        g = np.zeros(max(self.n, 1), np.float64)
        lb = C.c_double()
        _check(self.L, self.L.orc_smooth_grad(self.h, float(alpha), int(iters), _p(g), C.byref(lb)))
        return g[:self.n], lb.value

    def count_solutions(self) -> np.ndarray:
        out = np.zeros(self.m, np.float64)
        self.L.orc_count_solutions(self.h, _p(out))
        return out

    def checks(self) -> np.ndarray:
        out = np.zeros(4, np.float64)
        self.L.orc_checks(self.h, _p(out))
        return out


def build_row(coefs, sense: int, rhs: int, precision: str = "f64", budget: int = 0):
    """One row's diagram with levels in the given coefficient order: (widths, lo, hi)."""
    L = _lib(precision)
    a = np.ascontiguousarray(coefs, np.int64)
    k = int(a.shape[0])
    cap = 1 << 16
    w = np.zeros(max(k, 1), np.int32)
    lo = np.zeros(cap, np.int32)
    hi = np.zeros(cap, np.int32)
    nn = int(L.orc_build_row(k, _p(a), int(sense), int(rhs), int(budget), _p(w), _p(lo), _p(hi), cap))
    if nn < 0:
        raise OracleError(nn, L.orc_error().decode())
    assert nn <= cap
    return w[:k].copy(), lo[:nn].copy(), hi[:nn].copy()
