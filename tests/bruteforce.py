"""Brute-force references used to pin the oracle (tests only).

Everything here works from definitions by enumeration, independent of any
decision-diagram code:
- ``truth_table_bdd``: the canonical quasi-reduced BDD of a row read off its
  truth table (Prop. "Canonicity": one diagram per Boolean function; a level's
  nodes are the distinct nonzero residual functions of the reachable prefixes,
  numbered in breadth-first discovery order, 0-arc child first);
- ``BruteDBCA``: Alg. "Min-marginal averaging" with min-marginals taken by
  enumerating each row's feasible set (eq. "min-marginals") in exact rational
  arithmetic;
- ``ilp_optimum``: the ILP optimum by enumerating {0,1}^n.
"""
from __future__ import annotations

import itertools
import math
from fractions import Fraction

import numpy as np

BOT, TOP = -1, -2
INF = float("inf")


def row_ok(sense, lhs, rhs):
    return lhs == rhs if sense == 0 else (lhs <= rhs if sense == 1 else lhs >= rhs)


def truth_table_bdd(coefs, sense, rhs):
    """Canonical BDD of one row by enumeration. Returns (widths, lo, hi) or None if the row is infeasible."""
    a = list(coefs)
    k = len(a)
    # f over all assignments; bit index = integer with x_0 as the most significant bit
    f = 0
    for idx in range(1 << k):
        bits = [(idx >> (k - 1 - t)) & 1 for t in range(k)]
        if row_ok(sense, sum(c * x for c, x in zip(a, bits)), rhs):
            f |= 1 << idx
    if f == 0:
        return None

    def split(g, rest):
        # g is a residual over `rest` variables; return (g | x=0, g | x=1) over rest-1 variables
        half = 1 << (rest - 1)
        mask = (1 << half) - 1
        return g & mask, (g >> half) & mask

    levels = [[f]]
    lo, hi = [], []
    for t in range(k):
        rest = k - t
        nxt = []
        for g in levels[t]:
            g0, g1 = split(g, rest)
            ch = []
            for h in (g0, g1):
                if t == k - 1:
                    ch.append(TOP if h else BOT)
                elif h == 0:
                    ch.append(BOT)
                else:
                    if h not in nxt:
                        nxt.append(h)
                    ch.append(nxt.index(h))
            lo.append(ch[0])
            hi.append(ch[1])
        if t < k - 1:
            levels.append(nxt)
    return [len(L) for L in levels], lo, hi


def feasible_set(coefs, sense, rhs):
    k = len(coefs)
    return [x for x in itertools.product((0, 1), repeat=k)
            if row_ok(sense, sum(c * v for c, v in zip(coefs, x)), rhs)]


class BruteDBCA:
    """Alg. "Min-marginal averaging" with enumerated min-marginals, exact rationals.

    Reading for rows that force a variable (infinite difference): the rows in F
    absorb the finite differences of the others (as in the oracle); the paper is
    silent there.
    """

    def __init__(self, ilp):
        self.n = ilp.n
        self.cost = [Fraction(float(c)) for c in ilp.cost]
        rank = np.empty(ilp.n, np.int64)
        rank[np.asarray(ilp.order)] = np.arange(ilp.n)
        self.order = [int(v) for v in ilp.order]
        self.rows = []  # (vars in processing order, feasible assignments)
        for j in range(ilp.m):
            cols, coefs, s, b = ilp.row(j)
            pairs = sorted([(int(rank[v]), int(v), int(c)) for v, c in zip(cols, coefs) if c != 0])
            vs = [p[1] for p in pairs]
            cs = [p[2] for p in pairs]
            X = feasible_set(cs, s, b)
            assert X, f"row {j} infeasible"
            self.rows.append((vs, X))
        self.J = [[] for _ in range(self.n)]
        for j, (vs, _) in enumerate(self.rows):
            for v in vs:
                self.J[v].append(j)
        self.lam = [dict() for _ in self.rows]
        for i in range(self.n):
            for j in self.J[i]:
                self.lam[j][i] = self.cost[i] / len(self.J[i])
        self.const = sum((c for i, c in enumerate(self.cost) if not self.J[i] and c < 0), Fraction(0))

    def energy(self, j):
        vs, X = self.rows[j]
        if not vs:
            return Fraction(0)
        return min(sum((self.lam[j][v] for v, xv in zip(vs, x) if xv), Fraction(0)) for x in X)

    def mm(self, j, i, beta):
        vs, X = self.rows[j]
        t = vs.index(i)
        vals = [sum((self.lam[j][v] for v, xv in zip(vs, x) if xv), Fraction(0)) for x in X if x[t] == beta]
        return min(vals) if vals else INF

    def lb(self):
        return sum((self.energy(j) for j in range(len(self.rows))), Fraction(0)) + self.const

    def update(self, i):
        Ji = self.J[i]
        if not Ji:
            return
        d = []
        for j in Ji:
            m1, m0 = self.mm(j, i, 1), self.mm(j, i, 0)
            d.append(INF if m1 == INF else (-INF if m0 == INF else m1 - m0))
        F = [q for q, v in enumerate(d) if v in (INF, -INF)]
        if not F:
            avg = sum(d, Fraction(0)) / len(Ji)
            for q, j in enumerate(Ji):
                self.lam[j][i] = self.lam[j][i] - d[q] + avg
        else:
            signs = {d[q] > 0 for q in F}
            assert len(signs) == 1, "conflict"
            fin = sum((d[q] for q in range(len(Ji)) if q not in F), Fraction(0))
            for q, j in enumerate(Ji):
                if q in F:
                    self.lam[j][i] = self.lam[j][i] + fin / len(F)
                else:
                    self.lam[j][i] = self.lam[j][i] - d[q]

    def iterate(self, iters):
        trace = []
        for _ in range(iters):
            for i in self.order:
                self.update(i)
            for i in reversed(self.order):
                self.update(i)
            trace.append(self.lb())
        return trace

    def lam_canonical(self):
        out = []
        for j, (vs, _) in enumerate(self.rows):
            out.extend(self.lam[j][v] for v in vs)
        return out


def ilp_optimum(ilp):
    """min c^T x over {0,1}^n satisfying all rows (None if infeasible), by enumeration (n <= 20)."""
    n = ilp.n
    assert n <= 20
    X = ((np.arange(1 << n)[:, None] >> np.arange(n)[None, :]) & 1).astype(np.int64)
    ok = np.ones(X.shape[0], bool)
    for j in range(ilp.m):
        cols, coefs, s, b = ilp.row(j)
        lhs = X[:, cols] @ coefs
        ok &= (lhs == b) if s == 0 else ((lhs <= b) if s == 1 else (lhs >= b))
    if not ok.any():
        return None
    return float((X[ok] @ ilp.cost).min())


def as_float(v):
    return float(v) if not (isinstance(v, float) and math.isinf(v)) else v


class BruteSplitDBCA:
    """Sec. 6, Alg. "Parallel min-marginal averaging", by enumeration in exact rationals.

    Each row's diagram comes from ``truth_table_bdd``; it is cut between levels whose variables lie
    in different intervals (``intervals``), and every sub-BDD is kept as the list of its paths:
    (entering arc or None, bits of its levels, closing copy-arc or None), where an entering arc
    (u, beta) leaves node u of the level before the cut and a closing copy-arc (u, beta) leaves
    node u of its last level. A path costs mu of its entering arc, lambda on its 1-bits and mu_bar
    of its copy-arc. Min-marginals, arc-marginals and energies are minima over these lists; the
    updates follow the algorithm (forward pass, forward copy-arc update, backward pass, backward
    copy-arc update), with the readings the oracle states (the entering arc costs mu alone, the
    minimum of an update runs over one cut's pairs, forced rows absorb finite differences).
    """

    def __init__(self, ilp, K, gamma=Fraction(1, 2)):
        self.base = BruteDBCA(ilp)
        self.gamma = Fraction(gamma)
        b = self.base
        shapes = []
        for j, (vs, _) in enumerate(b.rows):
            cols, coefs, s, rhs = ilp.row(j)
            cmap = {int(v): int(c) for v, c in zip(cols, coefs)}
            shapes.append(truth_table_bdd([cmap[v] for v in vs], s, rhs) if vs else None)
        self.shapes = shapes
        self.intv = intervals(ilp, K, [sh[0] if sh else [] for sh in shapes], [vs for vs, _ in b.rows])
        self.segs = []   # per row: list of (s0, s1, paths)
        self.mux, self.mue, self.dfw, self.dbw = {}, {}, {}, {}
        for j, (vs, _) in enumerate(b.rows):
            if not vs:
                self.segs.append([])
                continue
            widths, lo, hi = shapes[j]
            first = [0]
            for w in widths:
                first.append(first[-1] + w)
            k = len(vs)
            cuts = [l for l in range(k - 1) if self.intv[vs[l]] != self.intv[vs[l + 1]]]
            bounds = [0] + [l + 1 for l in cuts] + [k]
            segs = []
            for s0, s1 in zip(bounds[:-1], bounds[1:]):
                paths = []
                if s0 == 0:
                    starts = [(None, 0)]
                else:
                    starts = []
                    for u in range(widths[s0 - 1]):
                        for beta, ch in ((0, lo[first[s0 - 1] + u]), (1, hi[first[s0 - 1] + u])):
                            if ch >= 0:
                                starts.append(((s0 - 1, u, beta), ch))

                def walk(l, u, bits, entry):
                    for beta, ch in ((0, lo[first[l] + u]), (1, hi[first[l] + u])):
                        if ch == BOT:
                            continue
                        if l == s1 - 1:
                            if s1 == k:
                                assert ch == TOP
                                paths.append((entry, bits + [beta], None))
                            else:
                                paths.append((entry, bits + [beta], (l, u, beta)))
                        else:
                            walk(l + 1, ch, bits + [beta], entry)

                for entry, v in starts:
                    walk(s0, v, [], entry)
                segs.append((s0, s1, paths))
            for l in cuts:
                for u in range(widths[l]):
                    for beta, ch in ((0, lo[first[l] + u]), (1, hi[first[l] + u])):
                        if ch >= 0:
                            for d in (self.mux, self.mue, self.dfw, self.dbw):
                                d[(j, l, u, beta)] = Fraction(0)
            self.segs.append(segs)

    def _cost(self, j, s0, path):
        entry, bits, exit_ = path
        vs = self.base.rows[j][0]
        c = self.mue[(j,) + entry] if entry else Fraction(0)
        c += sum((self.base.lam[j][vs[s0 + t]] for t, x in enumerate(bits) if x), Fraction(0))
        if exit_:
            c += self.mux[(j,) + exit_]
        return c

    def _seg_of(self, j, l):
        for s0, s1, paths in self.segs[j]:
            if s0 <= l < s1:
                return s0, paths
        raise AssertionError

    def mm(self, j, i, beta):
        vs = self.base.rows[j][0]
        l = vs.index(i)
        s0, paths = self._seg_of(j, l)
        vals = [self._cost(j, s0, p) for p in paths if p[1][l - s0] == beta]
        return min(vals) if vals else INF

    def lb(self):
        e = Fraction(0)
        for j, segs in enumerate(self.segs):
            for s0, _, paths in segs:
                e += min(self._cost(j, s0, p) for p in paths)
        return e + self.base.const

    def _update(self, i):
        b = self.base
        Ji = b.J[i]
        if not Ji:
            return
        d = []
        for j in Ji:
            m1, m0 = self.mm(j, i, 1), self.mm(j, i, 0)
            d.append(INF if m1 == INF else (-INF if m0 == INF else m1 - m0))
        F = [q for q, v in enumerate(d) if v in (INF, -INF)]
        if not F:
            avg = sum(d, Fraction(0)) / len(Ji)
            for q, j in enumerate(Ji):
                b.lam[j][i] = b.lam[j][i] - d[q] + avg
        else:
            fin = sum((d[q] for q in range(len(Ji)) if q not in F), Fraction(0))
            for q, j in enumerate(Ji):
                b.lam[j][i] = b.lam[j][i] + fin / len(F) if q in F else b.lam[j][i] - d[q]

    def _copy_update(self, forward):
        g = self.gamma
        for j, segs in enumerate(self.segs):
            for si in range(len(segs) - 1):
                s0, s1, paths = segs[si] if forward else segs[si + 1]
                key = 2 if forward else 0
                m = {}
                for p in paths:
                    a = p[key]
                    c = self._cost(j, s0, p)
                    m[a] = min(m.get(a, INF), c)
                mn = min(m.values())
                for a, v in m.items():
                    kk = (j,) + a
                    if forward:
                        self.dfw[kk] = v - mn
                        self.mux[kk] = self.mux[kk] - g * self.dfw[kk] + g * self.dbw[kk]
                    else:
                        self.dbw[kk] = v - mn
                        self.mue[kk] = self.mue[kk] - g * self.dbw[kk] + g * self.dfw[kk]

    def iterate(self, iters):
        trace = []
        for _ in range(iters):
            for i in self.base.order:
                self._update(i)
            self._copy_update(True)
            for i in reversed(self.base.order):
                self._update(i)
            self._copy_update(False)
            trace.append(self.lb())
        return trace


def intervals(ilp, K, widths_of_row, vars_of_row):
    """Interval of each variable (Sec. 6): the processing order cut into K runs of about equal node
    count, a variable counting its levels' nodes over all rows; floor(K * before / total)."""
    cnt = [0] * ilp.n
    for ws, vs in zip(widths_of_row, vars_of_row):
        for w, v in zip(ws, vs):
            cnt[v] += w
    total = sum(cnt)
    out = [0] * ilp.n
    before = 0
    for v in ilp.order:
        v = int(v)
        out[v] = (K * before) // total if total else 0
        before += cnt[v]
    return out
