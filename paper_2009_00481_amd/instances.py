"""Seeded synthetic 0-1 ILP instances shaped like the paper's workloads.

This module produces inputs only: costs, integer constraint rows and a
variable processing order. It holds none of the method's arithmetic, so both
the GPU path and the CPU oracle may consume what it produces.

Problem format (the paper's binary program over linear rows, Sec. 3, Example
"ILP"): ``min c^T x`` subject to ``sum_i a_ji x_i (sense_j) b_j`` for every
row ``j``, ``x`` in {0,1}^n. Rows are CSR (``row_ptr``, ``col``, ``coef``);
``sense`` is 0 for '=', 1 for '<=' and 2 for '>='. ``order[r]`` is the variable
processed r-th by the forward pass (Alg. "Min-marginal averaging" takes the
order as an input; the paper suggests bandwidth minimisation, App. A.3).

Workload recipes (ILP formulations of App. E):
- ``potts_grid``: MRF local polytope on a 4-neighbour grid (App. E.1) with
  unary simplex rows and both-side marginalisation rows (the redundant
  pairwise simplex row is implied and omitted).
- ``graph_matching``: assignment variables with <=1 rows on both sides and
  linearised pair products (App. E.2 with a sparse, linearised pair term).
- ``tomography``: discrete tomography (App. E.3): a 3-label Potts grid with
  zero unary costs plus one projection row per image row, column and diagonal
  (both directions) whose right-hand side comes from a random ground truth.
- ``tracking``: flow-conservation rows over detections in consecutive frames
  (the structure of the cell-tracking instances, App. E.4, without the
  division and exclusion rows).
- ``batch_config``: the uneven mix of tomography and tracking instances that
  the batched solver takes in one schedule.
- ``random_ilp``: small mixed-sense rows with coefficients in [-3, 3].
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SENSE_EQ, SENSE_LE, SENSE_GE = 0, 1, 2


@dataclass
class ILP:
    n: int
    cost: np.ndarray      # float64 [n]
    row_ptr: np.ndarray   # int64 [m+1]
    col: np.ndarray       # int32 [nnz]
    coef: np.ndarray      # int64 [nnz]
    sense: np.ndarray     # int8 [m]
    rhs: np.ndarray       # int64 [m]
    order: np.ndarray     # int32 [n], order[r] = variable processed r-th
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def row(self, j):
        a, b = int(self.row_ptr[j]), int(self.row_ptr[j + 1])
        return self.col[a:b], self.coef[a:b], int(self.sense[j]), int(self.rhs[j])

    def check(self) -> "ILP":
        assert self.cost.dtype == np.float64 and self.cost.shape == (self.n,)
        assert self.row_ptr.dtype == np.int64 and self.row_ptr[0] == 0
        assert self.col.dtype == np.int32 and self.coef.dtype == np.int64
        assert self.sense.dtype == np.int8 and self.rhs.dtype == np.int64
        assert self.order.dtype == np.int32 and self.order.shape == (self.n,)
        assert self.row_ptr[-1] == self.col.shape[0] == self.coef.shape[0]
        assert self.sense.shape == self.rhs.shape == (self.m,)
        return self


def _csr(rows_vars, rows_coef):
    lens = np.fromiter((len(v) for v in rows_vars), dtype=np.int64, count=len(rows_vars))
    row_ptr = np.zeros(len(rows_vars) + 1, dtype=np.int64)
    np.cumsum(lens, out=row_ptr[1:])
    col = np.concatenate(rows_vars).astype(np.int32) if rows_vars else np.zeros(0, np.int32)
    coef = np.concatenate(rows_coef).astype(np.int64) if rows_coef else np.zeros(0, np.int64)
    return row_ptr, col, coef


# ---------------------------------------------------------------------------
# Potts MRF on a grid (local polytope, App. E.1)
# ---------------------------------------------------------------------------

def grid_edges(H: int, W: int) -> np.ndarray:
    """4-neighbour edges, node-major: for each node (row-major) its right edge, then its down edge."""
    u = np.arange(H * W, dtype=np.int64).reshape(H, W)
    right = np.full((H, W), -1, np.int64)
    down = np.full((H, W), -1, np.int64)
    right[:, :-1] = u[:, 1:]
    down[:-1, :] = u[1:, :]
    src = np.stack([u, u], axis=-1).reshape(-1)
    dst = np.stack([right, down], axis=-1).reshape(-1)
    keep = dst >= 0
    return np.stack([src[keep], dst[keep]], axis=1)


def potts_grid(H: int, W: int, L: int, *, unary: str = "normal", weight=(0.2, 1.0),
               seed: int = 0, name: str = "") -> ILP:
    """Potts MRF on an H x W grid with L labels as a 0-1 ILP.

    Variables: unary x[u,l] = u*L + l (node-major, label-minor), then pairwise
    y[e,l,k] = nU + e*L*L + l*L + k (edge-major, (l,k) lexicographic). The
    processing order is the index order.

    Rows: for each node, sum_l x[u,l] = 1; for each edge e=(u,v) and label l,
    x[u,l] - sum_k y[e,l,k] = 0; for each label k, x[v,k] - sum_l y[e,l,k] = 0.
    Rows are listed as all node rows, then per edge its L u-side rows followed by
    its L v-side rows.

    Costs (fp32 values stored in float64): unary U[0,1) ("uniform") or N(0,1)
    ("normal"); pairwise w_e * [l != k] with w_e a constant or U[lo, hi) per edge.
    Draw order from one generator: unary table (nodes x labels), then weights.
    """
    rng = np.random.default_rng(seed)
    nV = H * W
    E = grid_edges(H, W)
    nE = E.shape[0]
    if unary == "uniform":
        un = rng.random((nV, L), dtype=np.float32)
    elif unary == "normal":
        un = rng.standard_normal((nV, L), dtype=np.float32)
    elif unary == "zero":
        un = np.zeros((nV, L), dtype=np.float32)
    else:
        raise ValueError(unary)
    if isinstance(weight, (tuple, list)):
        lo, hi = weight
        w = rng.uniform(lo, hi, size=nE).astype(np.float32)
    else:
        w = np.full(nE, weight, dtype=np.float32)
    nU = nV * L
    n = nU + nE * L * L
    cost = np.empty(n, np.float64)
    cost[:nU] = un.reshape(-1).astype(np.float64)
    neq = (np.arange(L)[:, None] != np.arange(L)[None, :]).astype(np.float32)
    pair = (w[:, None, None] * neq[None, :, :]).astype(np.float32)
    cost[nU:] = pair.reshape(-1).astype(np.float64)

    # node rows
    node_rows = np.arange(nU, dtype=np.int64).reshape(nV, L)
    # edge rows: [nE, 2, L, 1+L]
    ybase = nU + np.arange(nE, dtype=np.int64)[:, None, None] * L * L
    lab = np.arange(L, dtype=np.int64)
    y_u = ybase + lab[None, :, None] * L + lab[None, None, :]          # [nE, L(l), L(k)]
    y_v = ybase + lab[None, None, :] * L + lab[None, :, None]          # [nE, L(k), L(l)]
    xu = E[:, 0:1] * L + lab[None, :]                                  # [nE, L]
    xv = E[:, 1:2] * L + lab[None, :]
    rows_u = np.concatenate([xu[:, :, None], y_u], axis=2)             # [nE, L, 1+L]
    rows_v = np.concatenate([xv[:, :, None], y_v], axis=2)
    edge_rows = np.stack([rows_u, rows_v], axis=1).reshape(-1, 1 + L)  # [nE*2L, 1+L]

    m_node, m_edge = nV, nE * 2 * L
    row_ptr = np.empty(m_node + m_edge + 1, np.int64)
    row_ptr[: m_node + 1] = np.arange(m_node + 1, dtype=np.int64) * L
    row_ptr[m_node + 1:] = m_node * L + np.arange(1, m_edge + 1, dtype=np.int64) * (1 + L)
    col = np.concatenate([node_rows.reshape(-1), edge_rows.reshape(-1)]).astype(np.int32)
    ecoef = np.full((m_edge, 1 + L), -1, np.int64)
    ecoef[:, 0] = 1
    coef = np.concatenate([np.ones(m_node * L, np.int64), ecoef.reshape(-1)])
    sense = np.zeros(m_node + m_edge, np.int8)
    rhs = np.concatenate([np.ones(m_node, np.int64), np.zeros(m_edge, np.int64)])
    order = np.arange(n, dtype=np.int32)
    return ILP(n, cost, row_ptr, col, coef, sense, rhs, order,
               name=name or f"potts{H}x{W}_L{L}",
               meta=dict(kind="potts", H=H, W=W, L=L, n_edges=nE, seed=seed)).check()


def potts_counts(H: int, W: int, L: int) -> dict:
    """Closed-form sizes of ``potts_grid`` (rows, incidences and nodes of its BDDs).

    A simplex row over k variables has a 2k-1 node diagram; a marginalisation
    row (its unary first, then L pairwise) has 2L+1 nodes.
    """
    nV = H * W
    nE = H * (W - 1) + (H - 1) * W
    m_edge = nE * 2 * L
    return dict(n=nV * L + nE * L * L, m=nV + m_edge, n_edges=nE,
                incidences=nV * L + m_edge * (L + 1),
                nodes=nV * (2 * L - 1) + m_edge * (2 * L + 1))


# ---------------------------------------------------------------------------
# Graph matching (App. E.2, sparse candidates, linearised pair products)
# ---------------------------------------------------------------------------

def graph_matching(nL: int, nR: int, cand: int, n_pairs: int, *, seed: int = 0,
                   name: str = "") -> ILP:
    """Graph matching with sparse candidates and linearised pairwise terms.

    Assignment variables x[a], a = l*cand + q, link left node l to its q-th of
    ``cand`` distinct uniformly drawn right nodes (so right degrees are uneven,
    about Poisson). Pair variables y[p] = nA + p for ``n_pairs`` distinct
    unordered pairs {a, b} with different left and different right endpoints.
    Costs: x ~ N(0,1), y ~ U[-1, 0) (fp32 values).
    Rows: sum over a left node <= 1; sum over a right node <= 1 (right nodes
    with at least one candidate); per pair y - x_a <= 0, y - x_b <= 0 and
    x_a + x_b - y <= 1.
    Order: greedy colouring of the shares-a-row graph (``greedy_colour_order``).
    """
    rng = np.random.default_rng(seed)
    right = np.stack([rng.choice(nR, size=cand, replace=False) for _ in range(nL)]).astype(np.int64)
    nA = nL * cand
    a_left = np.repeat(np.arange(nL, dtype=np.int64), cand)
    a_right = right.reshape(-1)
    cx = rng.standard_normal(nA, dtype=np.float32)
    # pairs by rejection, keeping draw order
    pa = np.zeros(0, np.int64)
    pb = np.zeros(0, np.int64)
    seen = set()
    while pa.shape[0] < n_pairs:
        need = n_pairs - pa.shape[0]
        a = rng.integers(0, nA, size=2 * need + 16)
        b = rng.integers(0, nA, size=2 * need + 16)
        ok = (a_left[a] != a_left[b]) & (a_right[a] != a_right[b])
        a, b = a[ok], b[ok]
        lo_, hi_ = np.minimum(a, b), np.maximum(a, b)
        keep_a, keep_b = [], []
        for x, y in zip(lo_.tolist(), hi_.tolist()):
            if (x, y) in seen:
                continue
            seen.add((x, y))
            keep_a.append(x)
            keep_b.append(y)
            if pa.shape[0] + len(keep_a) >= n_pairs:
                break
        pa = np.concatenate([pa, np.array(keep_a, np.int64)])
        pb = np.concatenate([pb, np.array(keep_b, np.int64)])
    pa, pb = pa[:n_pairs], pb[:n_pairs]
    cy = rng.uniform(-1.0, 0.0, size=n_pairs).astype(np.float32)
    n = nA + n_pairs
    cost = np.concatenate([cx, cy]).astype(np.float64)

    rows_v, rows_c, sense, rhs = [], [], [], []
    for l in range(nL):
        rows_v.append(np.arange(l * cand, (l + 1) * cand, dtype=np.int64))
        rows_c.append(np.ones(cand, np.int64))
        sense.append(SENSE_LE)
        rhs.append(1)
    by_right = np.argsort(a_right, kind="stable")
    rcount = np.bincount(a_right, minlength=nR)
    start = 0
    for r in range(nR):
        c = int(rcount[r])
        if c:
            rows_v.append(by_right[start:start + c].astype(np.int64))
            rows_c.append(np.ones(c, np.int64))
            sense.append(SENSE_LE)
            rhs.append(1)
        start += c
    y = nA + np.arange(n_pairs, dtype=np.int64)
    for p in range(n_pairs):
        a, b, yy = int(pa[p]), int(pb[p]), int(y[p])
        rows_v += [np.array([yy, a]), np.array([yy, b]), np.array([a, b, yy])]
        rows_c += [np.array([1, -1]), np.array([1, -1]), np.array([1, 1, -1])]
        sense += [SENSE_LE] * 3
        rhs += [0, 0, 1]
    row_ptr, col, coef = _csr(rows_v, rows_c)
    ilp = ILP(n, cost, row_ptr, col, coef, np.array(sense, np.int8), np.array(rhs, np.int64),
              np.arange(n, dtype=np.int32), name=name or f"gm{nL}x{nR}_c{cand}_p{n_pairs}",
              meta=dict(kind="graph_matching", nL=nL, nR=nR, cand=cand, n_pairs=n_pairs, seed=seed))
    ilp.order = greedy_colour_order(ilp)
    return ilp.check()


def greedy_colour_order(ilp: ILP) -> np.ndarray:
    """Greedy colouring of the graph whose edges join variables sharing a row.

    Variables are coloured in index order with the smallest colour unused by
    already coloured neighbours; the order lists colour 0 first, then colour 1,
    and so on, index order within a colour.

    The colours of a variable's coloured neighbours are the union, over its
    rows, of the colours already taken in that row, so each row keeps the set
    of its members' colours as a bit set.
    """
    n, m = ilp.n, ilp.m
    rp, col = ilp.row_ptr, ilp.col
    # variable -> rows
    rows_of = np.repeat(np.arange(m, dtype=np.int64), np.diff(rp))
    perm = np.argsort(col, kind="stable")
    vrows = rows_of[perm]
    vptr = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(col, minlength=n), out=vptr[1:])
    colour = np.full(n, -1, np.int64)
    vptr_l, vrows_l = vptr.tolist(), vrows.tolist()
    taken = [0] * m
    for v in range(n):
        rows = vrows_l[vptr_l[v]:vptr_l[v + 1]]
        used = 0
        for j in rows:
            used |= taken[j]
        c = (~used & (used + 1)).bit_length() - 1
        colour[v] = c
        bit = 1 << c
        for j in rows:
            taken[j] |= bit
    return np.argsort(colour, kind="stable").astype(np.int32)


# ---------------------------------------------------------------------------
# Discrete tomography (App. E.3) and tracking-style flow instances (App. E.4)
# ---------------------------------------------------------------------------

def tomography_truth(P: int, seed: int) -> np.ndarray:
    """Ground-truth image: label 0 background and ceil(P/8) discs painted in turn, each with a
    uniform centre in [0, P)^2, radius U[P/16, P/4] and label 1 or 2 (later discs on top)."""
    rng = np.random.default_rng(seed)
    img = np.zeros((P, P), np.int64)
    ii, jj = np.meshgrid(np.arange(P), np.arange(P), indexing="ij")
    for _ in range((P + 7) // 8):
        ci, cj = rng.uniform(0, P, size=2)
        r = rng.uniform(P / 16, P / 4)
        lab = int(rng.integers(1, 3))
        img[(ii - ci) ** 2 + (jj - cj) ** 2 <= r * r] = lab
    return img


def tomography_lines(P: int) -> list:
    """Projection lines as pixel index arrays: rows, columns, diagonals (i - j constant, from
    -(P-1)), anti-diagonals (i + j constant, from 0)."""
    idx = np.arange(P * P, dtype=np.int64).reshape(P, P)
    lines = [idx[i, :] for i in range(P)] + [idx[:, j] for j in range(P)]
    lines += [np.diagonal(idx, offset=o).copy() for o in range(-(P - 1), P)]
    flip = idx[:, ::-1]
    lines += [np.diagonal(flip, offset=o).copy() for o in range(P - 1, -P, -1)]
    return lines


def tomography(P: int, *, seed: int = 0, potts: float = 0.1, unary: str = "zero", name: str = "") -> ILP:
    """Discrete tomography on a P x P image with labels {0, 1, 2} (label value = intensity).

    The Potts part is ``potts_grid(P, P, 3)`` with weight ``potts`` on every edge (same variables
    and rows) and unary costs ``unary``: "zero" (the workload) or "normal" (N(0,1), for tests that
    need every multiplier to move: with zero unary costs the multipliers of the unary variables in
    projection rows never leave 0). Then one equality row per projection line (rows, columns, both
    diagonal directions): sum over its pixels p of 1 x[p,1] + 2 x[p,2] = b, with b the line's sum of
    ``tomography_truth(P, seed)``; label 0 has coefficient 0 and is left out of the row. The
    ground truth with consistent pairwise variables is feasible. Order: greedy colouring.
    """
    base = potts_grid(P, P, 3, unary=unary, weight=potts, seed=seed)
    img = tomography_truth(P, seed)
    flat = img.reshape(-1)
    rows_v, rows_c, rhs = [], [], []
    for ln in tomography_lines(P):
        v = np.stack([ln * 3 + 1, ln * 3 + 2], axis=1).reshape(-1)
        c = np.tile(np.array([1, 2], np.int64), ln.shape[0])
        rows_v.append(v)
        rows_c.append(c)
        rhs.append(int(flat[ln].sum()))
    rp2, col2, coef2 = _csr(rows_v, rows_c)
    nnz0 = base.col.shape[0]
    row_ptr = np.concatenate([base.row_ptr, nnz0 + rp2[1:]])
    col = np.concatenate([base.col, col2])
    coef = np.concatenate([base.coef, coef2])
    sense = np.concatenate([base.sense, np.zeros(len(rows_v), np.int8)])
    rhs_all = np.concatenate([base.rhs, np.array(rhs, np.int64)])
    ilp = ILP(base.n, base.cost, row_ptr, col, coef, sense, rhs_all, base.order,
              name=name or f"tomo{P}_s{seed}",
              meta=dict(kind="tomography", P=P, seed=seed, n_lines=len(rows_v), truth=img))
    ilp.order = greedy_colour_order(ilp)
    return ilp.check()


def tomography_truth_point(ilp: ILP) -> np.ndarray:
    """The 0/1 point of a tomography instance's ground truth (one-hot pixels, consistent pairs)."""
    P = ilp.meta["P"]
    img = ilp.meta["truth"].reshape(-1)
    x = np.zeros(ilp.n, np.int8)
    x[np.arange(P * P) * 3 + img] = 1
    E = grid_edges(P, P)
    nU = P * P * 3
    x[nU + np.arange(E.shape[0]) * 9 + img[E[:, 0]] * 3 + img[E[:, 1]]] = 1
    return x


def tracking(D: int, *, seed: int = 0, name: str = "") -> ILP:
    """Flow conservation over D detections split evenly into F = ceil(D/100) frames.

    Each detection of a frame other than the last links to 1 or 2 distinct random detections of the
    next frame. Variables: appear a_d = 2d and disappear z_d = 2d + 1 for each detection d, then the
    links in creation order (frame by frame, source by source). One row per detection:
    a_d + sum(links into d) - z_d - sum(links out of d) = 0. Costs N(0,1) fp32 (drawn after the
    structure). Order: index order.
    """
    rng = np.random.default_rng(seed)
    F = (D + 99) // 100
    bounds = [(f * D) // F for f in range(F + 1)]
    src, dst = [], []
    for f in range(F - 1):
        a0, a1, b0, b1 = bounds[f], bounds[f + 1], bounds[f + 1], bounds[f + 2]
        for d in range(a0, a1):
            k = min(int(rng.integers(1, 3)), b1 - b0)
            for t in rng.choice(b1 - b0, size=k, replace=False):
                src.append(d)
                dst.append(b0 + int(t))
    nlink = len(src)
    n = 2 * D + nlink
    cost = rng.standard_normal(n, dtype=np.float32).astype(np.float64)
    ins = [[] for _ in range(D)]
    outs = [[] for _ in range(D)]
    for e, (s_, t_) in enumerate(zip(src, dst)):
        outs[s_].append(2 * D + e)
        ins[t_].append(2 * D + e)
    rows_v, rows_c = [], []
    for d in range(D):
        v = [2 * d] + ins[d] + [2 * d + 1] + outs[d]
        c = [1] * (1 + len(ins[d])) + [-1] * (1 + len(outs[d]))
        rows_v.append(np.array(v, np.int64))
        rows_c.append(np.array(c, np.int64))
    row_ptr, col, coef = _csr(rows_v, rows_c)
    return ILP(n, cost, row_ptr, col, coef, np.zeros(D, np.int8), np.zeros(D, np.int64),
               np.arange(n, dtype=np.int32), name=name or f"track{D}_s{seed}",
               meta=dict(kind="tracking", D=D, frames=F, links=nlink, seed=seed)).check()


def batch_config(n_inst: int = 256, *, p_range=(32, 128), d_range=(200, 2000)) -> list:
    """The batched workload: tomography and tracking instances interleaved (even positions
    tomography, odd ones tracking), instance seed = position. Sizes from the instance's own seed:
    P ~ U{p_range}, D ~ U{d_range} (inclusive)."""
    out = []
    for k in range(n_inst):
        r = np.random.default_rng([k, 7])
        if k % 2 == 0:
            out.append(tomography(int(r.integers(p_range[0], p_range[1] + 1)), seed=k))
        else:
            out.append(tracking(int(r.integers(d_range[0], d_range[1] + 1)), seed=k))
    return out


def concat(ilps: list, name: str = "") -> ILP:
    """Block-diagonal union of instances: variables, rows and orders concatenated in instance
    order (instance k's variables shifted by the sizes before it)."""
    voff = np.cumsum([0] + [q.n for q in ilps])
    noff = np.cumsum([0] + [q.nnz for q in ilps])
    row_ptr = np.concatenate([np.zeros(1, np.int64)] + [q.row_ptr[1:] + noff[k] for k, q in enumerate(ilps)])
    col = np.concatenate([q.col.astype(np.int64) + voff[k] for k, q in enumerate(ilps)]).astype(np.int32)
    order = np.concatenate([q.order.astype(np.int64) + voff[k] for k, q in enumerate(ilps)]).astype(np.int32)
    return ILP(int(voff[-1]), np.concatenate([q.cost for q in ilps]), row_ptr, col,
               np.concatenate([q.coef for q in ilps]), np.concatenate([q.sense for q in ilps]),
               np.concatenate([q.rhs for q in ilps]), order, name=name or f"concat{len(ilps)}",
               meta=dict(kind="concat", var_off=voff, row_off=np.cumsum([0] + [q.m for q in ilps]))).check()


# ---------------------------------------------------------------------------
# Small random mixed-sense ILPs (tests)
# ---------------------------------------------------------------------------

def random_ilp(n: int, m: int, *, kmin: int = 1, kmax: int = 5, cmax: int = 3,
               senses=(SENSE_EQ, SENSE_LE, SENSE_GE), seed: int = 0, shuffle_order: bool = True,
               cover_all: bool = True, name: str = "") -> ILP:
    """Random rows over distinct variables with nonzero coefficients in [-cmax, cmax].

    The right-hand sides are set from a hidden random 0/1 point x0 (equal for
    '=', slack U{0..2} otherwise), so the whole ILP is feasible. With
    ``cover_all`` every variable appears in at least one row.
    Costs are N(0,1) fp32 values; the order is a random permutation.
    """
    rng = np.random.default_rng(seed)
    x0 = rng.integers(0, 2, size=n)
    rows_v, rows_c, sense, rhs = [], [], [], []
    uncovered = list(rng.permutation(n)) if cover_all else []
    for j in range(m):
        k = int(rng.integers(kmin, min(kmax, n) + 1))
        vs = list(rng.choice(n, size=k, replace=False))
        if uncovered:
            # put some uncovered variables in so that every variable gets a row
            take = [v for v in uncovered[:k] if v not in vs]
            for t, v in enumerate(take):
                vs[t] = v
            vs = list(dict.fromkeys(vs))
            uncovered = [v for v in uncovered if v not in vs]
        vs = np.array(vs, np.int64)
        cs = rng.integers(1, cmax + 1, size=vs.shape[0]) * rng.choice([-1, 1], size=vs.shape[0])
        s = int(rng.choice(np.array(senses)))
        act = int(cs @ x0[vs])
        slack = int(rng.integers(0, 3))
        r = act if s == SENSE_EQ else (act + slack if s == SENSE_LE else act - slack)
        rows_v.append(vs)
        rows_c.append(cs.astype(np.int64))
        sense.append(s)
        rhs.append(r)
    row_ptr, col, coef = _csr(rows_v, rows_c)
    cost = rng.standard_normal(n, dtype=np.float32).astype(np.float64)
    order = rng.permutation(n).astype(np.int32) if shuffle_order else np.arange(n, dtype=np.int32)
    return ILP(n, cost, row_ptr, col, coef, np.array(sense, np.int8), np.array(rhs, np.int64),
               order, name=name or f"rand_n{n}_m{m}_s{seed}",
               meta=dict(kind="random", seed=seed)).check()


def from_rows(n, cost, rows, order=None, name="") -> ILP:
    """Build an ILP from a list of (vars, coefs, sense, rhs) tuples."""
    rows_v = [np.asarray(r[0], np.int64) for r in rows]
    rows_c = [np.asarray(r[1], np.int64) for r in rows]
    row_ptr, col, coef = _csr(rows_v, rows_c) if rows else (np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int64))
    sense = np.array([r[2] for r in rows], np.int8)
    rhs = np.array([r[3] for r in rows], np.int64)
    order = np.arange(n, dtype=np.int32) if order is None else np.asarray(order, np.int32)
    return ILP(n, np.asarray(cost, np.float64), row_ptr, col, coef, sense, rhs, order, name=name).check()


def config(idx: int, **kw) -> ILP:
    """The benchmark workloads by number.

    1: Potts 8x8, 3 labels, unary U[0,1), Potts weight 0.5, seed 0.
    2: Potts 256x256, 8 labels, unary N(0,1), weight U[0.2,1.0] per edge, seed 0.
    3: graph matching 5000x5000, 10 candidates per left node, 200k pairs, seed 0.
    5: Potts 128x128, 4 labels, the distributions of 2.
    "5sub": the 16x16 top-left stand-in of 5 used for finite differences.
    """
    if idx == 1:
        return potts_grid(8, 8, 3, unary="uniform", weight=0.5, seed=kw.get("seed", 0), name="potts8x8_L3")
    if idx == 2:
        return potts_grid(256, 256, 8, unary="normal", weight=(0.2, 1.0), seed=kw.get("seed", 0),
                          name="potts256x256_L8")
    if idx == 3:
        return graph_matching(5000, 5000, 10, 200_000, seed=kw.get("seed", 0), name="gm5000x5000")
    if idx == 5:
        return potts_grid(128, 128, 4, unary="normal", weight=(0.2, 1.0), seed=kw.get("seed", 0),
                          name="potts128x128_L4")
    if idx == "5sub":
        return potts_grid(16, 16, 4, unary="normal", weight=(0.2, 1.0), seed=kw.get("seed", 0),
                          name="potts16x16_L4")
    raise ValueError(idx)
