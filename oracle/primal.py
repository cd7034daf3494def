"""Oracle of the primal heuristic (Sec. 4; App. "Primal heuristic"), for small instances.

TEST INFRASTRUCTURE: only the test suite uses it; it shares no code with the product library.

Each row's feasible set X_j is enumerated; fixing x_i = beta keeps the solutions of every row of
J_i with x_i = beta (Alg. "Restriction-Propagation"), and a variable whose value is the same in every
remaining solution of one of its rows is fixed in turn, until nothing changes or a set is empty.
Alg. "Primal-Heuristic" as a depth-first search: the open variable of largest score is fixed to
beta_i = [M_i <= 0]; when that empties a set the other value is tried from the same state; when
both fail the search returns to the latest fixation whose other value is untried, until a complete
assignment or max_dead_ends dead ends.
Scores: |M_i| (mode 0), -M_i (mode 1), sign(R_i) M_i (mode 2) with R_i = sum over J_i of
|{x in X_j : x_i = 1}| - |{x in X_j : x_i = 0}| (eq. "search-space-reduction-coeff"). Ties: index.
"""
import itertools

import numpy as np


def _row_solutions(ilp, j):
    cols, coefs, sense, rhs = ilp.row(j)
    keep = [t for t in range(len(cols)) if coefs[t] != 0]
    vars_ = [int(cols[t]) for t in keep]
    a = [int(coefs[t]) for t in keep]
    sols = []
    for x in itertools.product((0, 1), repeat=len(vars_)):
        s = sum(ai * xi for ai, xi in zip(a, x))
        if (sense == 0 and s == rhs) or (sense == 1 and s <= rhs) or (sense == 2 and s >= rhs):
            sols.append(x)
    return vars_, sols


def _propagate(rows, rows_of, X, value, i, b):
    X = list(X)
    value = dict(value)
    queue = [(i, b)]
    while queue:
        i, b = queue.pop(0)
        if i in value:
            if value[i] != b:
                return None
            continue
        value[i] = b
        for j in rows_of[i]:
            vars_ = rows[j]
            p = vars_.index(i)
            X[j] = [x for x in X[j] if x[p] == b]
            if not X[j]:
                return None
            for q, v in enumerate(vars_):
                vals = {x[q] for x in X[j]}
                if len(vals) == 1:
                    (w,) = vals
                    if v in value and value[v] != w:
                        return None
                    if v not in value:
                        queue.append((v, w))
    return X, value


def primal_heuristic(ilp, M, mode=0, max_dead_ends=100000):
    """(x with -1 for undecided, objective over x = 1, feasible)."""
    M = np.asarray(M, np.float32).astype(np.float64)
    rows, X = [], []
    rows_of = [[] for _ in range(ilp.n)]
    for j in range(ilp.m):
        vars_, sols = _row_solutions(ilp, j)
        rows.append(vars_)
        X.append(sols)
        for v in vars_:
            rows_of[v].append(j)
    R = np.zeros(ilp.n)
    for j, vars_ in enumerate(rows):
        for q, v in enumerate(vars_):
            R[v] += sum(1 for x in X[j] if x[q] == 1) - sum(1 for x in X[j] if x[q] == 0)
    if mode == 0:
        score = np.abs(M)
    elif mode == 1:
        score = -M
    else:
        score = np.where(R > 0, M, np.where(R < 0, -M, 0.0))
    order = sorted(range(ilp.n), key=lambda i: (-score[i], i))
    value = {i: int(ilp.cost[i] < 0) for i in range(ilp.n) if not rows_of[i]}
    ok = True
    stack = []  # (position, value in force, no other value left, state before)
    state = (X, value)
    pos, dead = 0, 0
    while True:
        while pos < ilp.n and order[pos] in state[1]:
            pos += 1
        if pos == ilp.n:
            break
        i = order[pos]
        beta = 1 if M[i] <= 0 else 0
        r = _propagate(rows, rows_of, state[0], state[1], i, beta)
        if r is not None:
            stack.append((pos, beta, False, state))
            state = r
            continue
        r = _propagate(rows, rows_of, state[0], state[1], i, 1 - beta)
        if r is not None:
            stack.append((pos, 1 - beta, True, state))
            state = r
            continue
        dead += 1
        resumed = False
        while stack and dead <= max_dead_ends:
            p, v, last, prev = stack.pop()
            state = prev
            if last:
                continue
            r = _propagate(rows, rows_of, prev[0], prev[1], order[p], 1 - v)
            if r is not None:
                stack.append((p, 1 - v, True, prev))
                state = r
                pos = p
                resumed = True
                break
            dead += 1
        if not resumed:
            ok = False
            break
    X, value = state
    x = np.array([value.get(i, -1) for i in range(ilp.n)], np.int8)
    obj = float(sum(ilp.cost[i] for i in range(ilp.n) if x[i] == 1))
    return x, obj, ok
