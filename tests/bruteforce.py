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
