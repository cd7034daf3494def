/*
 * CPU oracle for BDD-based min-marginal averaging on 0-1 ILPs
 * (J.-H. Lange and P. Swoboda, "Efficient Message Passing for 0-1 ILPs with
 * Binary Decision Diagrams", ICML 2021).
 *
 * TEST INFRASTRUCTURE. This is the plain, slow, single-threaded reference the
 * GPU path is checked against. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load it. It shares no code, header or table
 * with the product library, and the product never loads it.
 *
 * Every step follows the paper in its own order:
 *   - one decision diagram per linear row (Sec. 3, Example "ILP": I_j holds the
 *     variables with a nonzero coefficient), built straight from the definition
 *     of a quasi-reduced ordered BDD (Sec. 5.1, Def. "Binary decision diagram",
 *     Prop. "Canonicity"): two partial assignments share a node exactly when
 *     they admit the same set of completions;
 *   - arc costs (Sec. 5.3, Def. "BDD arc costs"), forward and backward steps
 *     (Alg. "Forward BDD update step", Alg. "Backward BDD update step"),
 *     terminal values and min-marginals via arc-marginals (Sec. 5.3, eqs.
 *     "arc-marginal" and "marginal-aggregation");
 *   - the incremental schedule of Sec. 5.4 inside Alg. "Min-marginal
 *     averaging" (Sec. 3.2) with the update of eq. "mma-update";
 *   - the dual bound sum_j E^j of problem (D) (Sec. 3.1);
 *   - total min-marginal differences and preferred values (Sec. 4, Def. "Total
 *     min-marginal difference", eq. "preferred-variable-value").
 *
 * Readings where the paper is silent or garbled (each listed in the design notes):
 *   - Within a level, nodes are numbered in breadth-first discovery order from
 *     the root, 0-arc child before 1-arc child.
 *   - In the backward pass the backward step of a level runs after the update
 *     of that level's multiplier (Sec. 5.4 box; Prop. "correctness" needs it).
 *   - When a row forces a variable, its min-marginal difference is infinite
 *     and eq. "mma-update" is undefined. Rows with an infinite difference
 *     (set F) absorb the finite differences of the others: lambda^k -= d_k for
 *     k not in F, lambda^j += (sum_{k not in F} d_k)/|F| for j in F. Both signs
 *     of infinity in F mean an infeasible problem (ORC_CONFLICT).
 *   - Variables in no row add min(0, c_i) to the bound (App. A.1: the y-term of
 *     the dual with no multipliers) and round to [c_i < 0].
 *   - The J_i sum runs in ascending row order; the update is evaluated as
 *     (lambda - d) + (S / |J_i|); arc-marginals as (m_fwd + theta) + m_bwd.
 *
 * REAL is double unless the build defines ORC_REAL_FLOAT, which gives a float
 * mirror of the same steps (initial multipliers rounded from double, bound
 * accumulated in double) for bit-level comparisons at single precision.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#ifdef ORC_REAL_FLOAT
typedef float REAL;
#define REAL_INF ((float)INFINITY)
#else
typedef double REAL;
#define REAL_INF ((double)INFINITY)
#endif

#define ORC_OK 0
#define ORC_INVALID_ARG (-1)
#define ORC_ROW_INFEASIBLE (-2)
#define ORC_BDD_TOO_LARGE (-3)
#define ORC_CONFLICT (-5)
#define ORC_BAD_STATE (-7)
#define ORC_NOMEM (-9)

#define BOT (-1)
#define TOP (-2)

/* debug checks, see orc_init */
#define CHK_INCREMENTAL 1 /* incremental min-marginals equal from-scratch ones */
#define CHK_PROP1 2       /* bound gain of each update equals Prop. 1          */
#define CHK_EQUAL_D 4     /* after an update all differences equal the mean    */
#define CHK_SUM_LAMBDA 8  /* sum_j lambda^j_i stays c_i                        */

static char g_err[512];

static int fail(int code, const char *msg, long long a) {
  snprintf(g_err, sizeof g_err, "%s (%lld)", msg, a);
  return code;
}

const char *orc_error(void) { return g_err; }

static REAL rmin(REAL a, REAL b) { return b < a ? b : a; }

/* ---------------------------------------------------------------------------
 * One decision diagram
 * ------------------------------------------------------------------------- */
typedef struct {
  int k;        /* levels = variables of the row */
  int *var;     /* [k] variable of level l (processing order) */
  int *first;   /* [k+1] first node of level l; level l has first[l+1]-first[l] nodes */
  int *lo, *hi; /* [nodes] child index inside level l+1, or BOT / TOP */
  REAL *mf;     /* forward messages (cost of the best root-to-node path) */
  REAL *mb;     /* backward messages (cost of the best node-to-TOP path) */
  REAL *lam;    /* [k] lambda^j of each level's variable */
  /* Sec. 6 split (NULL without one): cut[l] = 1 when levels l and l+1 lie in different variable
   * intervals. For an arc (u, beta) leaving a cut level, index 2u+beta: mux = mu of its copy-arc
   * (the arc to TOP ending the sub-BDD before the cut), mue = mu of the arc itself (entering the
   * sub-BDD after the cut), dfw / dbw = the last forward / backward copy-arc updates. */
  unsigned char *cut;
  REAL *mux, *mue, *dfw, *dbw;
} bdd_t;

static int cmp_ll(const void *a, const void *b) {
  long long x = *(const long long *)a, y = *(const long long *)b;
  return (x > y) - (x < y);
}

static int row_holds(int sense, long long lhs, long long rhs) {
  if (sense == 0) return lhs == rhs;
  if (sense == 1) return lhs <= rhs;
  return lhs >= rhs;
}

/* Growable node list of one level: a representative partial sum and the set
 * of feasible completion sums (as flags over the sorted suffix-sum set). */
typedef struct {
  int cnt, cap, setlen;
  long long *rep;
  unsigned char *sets; /* cnt * setlen */
} level_t;

static int level_push(level_t *L, long long rep, const unsigned char *set) {
  if (L->cnt == L->cap) {
    int nc = L->cap ? 2 * L->cap : 4;
    long long *r = (long long *)realloc(L->rep, (size_t)nc * sizeof(long long));
    if (!r) return -1;
    L->rep = r;
    unsigned char *s = (unsigned char *)realloc(L->sets, (size_t)nc * (size_t)(L->setlen ? L->setlen : 1));
    if (!s) return -1;
    L->sets = s;
    L->cap = nc;
  }
  L->rep[L->cnt] = rep;
  if (L->setlen) memcpy(L->sets + (size_t)L->cnt * L->setlen, set, (size_t)L->setlen);
  return L->cnt++;
}

/*
 * Build the BDD of  sum_t a[t] x_{vars[t]}  (sense)  b,  t = 0..k-1 in
 * processing order, straight from the definition (Sec. 5.1):
 *   R_k = {0},  R_t = R_{t+1} U (a_t + R_{t+1})   (all sums the suffix can reach);
 *   a prefix with partial sum s at level t has completion set
 *   F_t(s) = { r in R_t : s + r satisfies the row };
 *   it is a node iff F_t(s) is nonempty (else the arc goes to BOT), and two
 *   prefixes share a node iff their completion sets are equal (every r in R_t
 *   is reached by some completion, so equal sets mean equal residual
 *   functions, which is the reduction of condition (vi)).
 * Nodes whose two arcs meet the same child are kept (consecutive indices on
 * every path, condition (iv)).
 */
static int build_bdd(int k, const int *vars, const long long *a, int sense, long long b,
                     long long budget, bdd_t *out) {
  memset(out, 0, sizeof *out);
  out->k = k;
  if (k == 0) {
    if (!row_holds(sense, 0, b)) return fail(ORC_ROW_INFEASIBLE, "row without variables fails", b);
    out->first = (int *)calloc(1, sizeof(int));
    return out->first ? ORC_OK : ORC_NOMEM;
  }
  long long **R = (long long **)calloc((size_t)k + 1, sizeof(long long *));
  int *Rn = (int *)calloc((size_t)k + 1, sizeof(int));
  level_t *lv = (level_t *)calloc((size_t)k, sizeof(level_t));
  unsigned char *tmp = NULL;
  int rc = ORC_OK;
  if (!R || !Rn || !lv) { rc = ORC_NOMEM; goto done; }
  R[k] = (long long *)malloc(sizeof(long long));
  R[k][0] = 0;
  Rn[k] = 1;
  int maxR = 1;
  for (int t = k - 1; t >= 0; --t) {
    int n1 = Rn[t + 1];
    long long *buf = (long long *)malloc((size_t)2 * n1 * sizeof(long long));
    if (!buf) { rc = ORC_NOMEM; goto done; }
    for (int q = 0; q < n1; ++q) { buf[q] = R[t + 1][q]; buf[n1 + q] = a[t] + R[t + 1][q]; }
    qsort(buf, (size_t)2 * n1, sizeof(long long), cmp_ll);
    int u = 0;
    for (int q = 0; q < 2 * n1; ++q)
      if (u == 0 || buf[q] != buf[u - 1]) buf[u++] = buf[q];
    R[t] = buf;
    Rn[t] = u;
    if (u > maxR) maxR = u;
    if (budget > 0 && u > budget) { rc = fail(ORC_BDD_TOO_LARGE, "suffix sum set exceeds the budget", u); goto done; }
  }
  for (int t = 0; t < k; ++t) lv[t].setlen = Rn[t];
  tmp = (unsigned char *)malloc((size_t)maxR);
  if (!tmp) { rc = ORC_NOMEM; goto done; }

  /* root: s = 0 */
  int any = 0;
  for (int q = 0; q < Rn[0]; ++q) { tmp[q] = (unsigned char)row_holds(sense, R[0][q], b); any |= tmp[q]; }
  if (!any) { rc = fail(ORC_ROW_INFEASIBLE, "row has no 0/1 solution", b); goto done; }
  if (level_push(&lv[0], 0, tmp) < 0) { rc = ORC_NOMEM; goto done; }

  /* children of every node, level by level; lo/hi kept in growable arrays */
  int cap = 16, nn = 0;
  int *lo = (int *)malloc((size_t)cap * sizeof(int)), *hi = (int *)malloc((size_t)cap * sizeof(int));
  if (!lo || !hi) { free(lo); free(hi); rc = ORC_NOMEM; goto done; }
  long long total = 0;
  for (int t = 0; t < k; ++t) {
    total += lv[t].cnt;
    if (budget > 0 && total > budget) { free(lo); free(hi); rc = fail(ORC_BDD_TOO_LARGE, "node budget exceeded", total); goto done; }
    for (int u = 0; u < lv[t].cnt; ++u) {
      int child[2];
      for (int beta = 0; beta < 2; ++beta) {
        long long s = lv[t].rep[u] + (beta ? a[t] : 0);
        if (t == k - 1) {
          child[beta] = row_holds(sense, s, b) ? TOP : BOT;
          continue;
        }
        int nz = 0;
        for (int q = 0; q < Rn[t + 1]; ++q) { tmp[q] = (unsigned char)row_holds(sense, s + R[t + 1][q], b); nz |= tmp[q]; }
        if (!nz) { child[beta] = BOT; continue; }
        int found = -1;
        for (int w = 0; w < lv[t + 1].cnt && found < 0; ++w)
          if (memcmp(lv[t + 1].sets + (size_t)w * Rn[t + 1], tmp, (size_t)Rn[t + 1]) == 0) found = w;
        if (found < 0) {
          found = level_push(&lv[t + 1], s, tmp);
          if (found < 0) { free(lo); free(hi); rc = ORC_NOMEM; goto done; }
        }
        child[beta] = found;
      }
      if (nn == cap) {
        cap *= 2;
        int *l2 = (int *)realloc(lo, (size_t)cap * sizeof(int)), *h2;
        if (!l2) { free(lo); free(hi); rc = ORC_NOMEM; goto done; }
        lo = l2;
        h2 = (int *)realloc(hi, (size_t)cap * sizeof(int));
        if (!h2) { free(lo); free(hi); rc = ORC_NOMEM; goto done; }
        hi = h2;
      }
      lo[nn] = child[0];
      hi[nn] = child[1];
      ++nn;
    }
  }
  out->var = (int *)malloc((size_t)k * sizeof(int));
  out->first = (int *)malloc((size_t)(k + 1) * sizeof(int));
  out->mf = (REAL *)malloc((size_t)nn * sizeof(REAL));
  out->mb = (REAL *)malloc((size_t)nn * sizeof(REAL));
  out->lam = (REAL *)calloc((size_t)k, sizeof(REAL));
  out->lo = lo;
  out->hi = hi;
  if (!out->var || !out->first || !out->mf || !out->mb || !out->lam) { rc = ORC_NOMEM; goto done; }
  out->first[0] = 0;
  for (int t = 0; t < k; ++t) {
    out->var[t] = vars[t];
    out->first[t + 1] = out->first[t] + lv[t].cnt;
  }
done:
  if (R)
    for (int t = 0; t <= k; ++t) free(R[t]);
  free(R);
  free(Rn);
  if (lv)
    for (int t = 0; t < k; ++t) { free(lv[t].rep); free(lv[t].sets); }
  free(lv);
  free(tmp);
  return rc;
}

static void free_bdd(bdd_t *B) {
  free(B->var); free(B->first); free(B->lo); free(B->hi);
  free(B->mf); free(B->mb); free(B->lam);
  free(B->cut); free(B->mux); free(B->mue); free(B->dfw); free(B->dbw);
}

/* ---------------------------------------------------------------------------
 * Dynamic-programming steps on one diagram (Sec. 5.3)
 * ------------------------------------------------------------------------- */

/* arc cost (Def. "BDD arc costs"): lambda of the tail's variable on 1-arcs, 0 on 0-arcs */
static REAL theta(const bdd_t *B, int l, int beta) { return beta ? B->lam[l] : (REAL)0; }

/* backward message of a child of level l (terminal values: BOT = inf, TOP = 0) */
static REAL child_mb(const REAL *mb, const bdd_t *B, int l, int c) {
  if (c == TOP) return (REAL)0;
  if (c == BOT) return REAL_INF;
  return mb[B->first[l + 1] + c];
}

/* backward value behind arc (u, beta) of level l (u a node index of the diagram): the child's
 * backward message, or, where the diagram is cut after level l (Sec. 6, Def. "Sub-BDD"), the
 * cost mu of the arc's copy-arc into TOP, which ends the sub-BDD before the cut. */
static REAL behind(const bdd_t *B, const REAL *mb, int l, int u, int beta) {
  int c = beta ? B->hi[u] : B->lo[u];
  if (B->cut && B->cut[l] && c != BOT) return B->mux[2 * u + beta];
  return child_mb(mb, B, l, c);
}

/* Alg. "Forward BDD update step" at level l: m_fwd(v) = min over in-arcs uv of m_fwd(u) + theta_uv;
 * the root has m_fwd = 0. After a cut the tails of the in-arcs are roots of the sub-BDD (m_fwd
 * 0) and each in-arc costs its copy dual mu alone (its lambda belongs to the sub-BDD before). */
static void forward_step(const bdd_t *B, REAL *mf, int l) {
  if (l == 0) { mf[B->first[0]] = 0; return; }
  for (int v = B->first[l]; v < B->first[l + 1]; ++v) mf[v] = REAL_INF;
  if (B->cut && B->cut[l - 1]) {
    for (int u = B->first[l - 1]; u < B->first[l]; ++u) {
      int c[2] = {B->lo[u], B->hi[u]};
      for (int beta = 0; beta < 2; ++beta) {
        if (c[beta] < 0) continue;
        int v = B->first[l] + c[beta];
        mf[v] = rmin(mf[v], B->mue[2 * u + beta]);
      }
    }
    return;
  }
  for (int u = B->first[l - 1]; u < B->first[l]; ++u) {
    int c[2] = {B->lo[u], B->hi[u]};
    for (int beta = 0; beta < 2; ++beta) {
      if (c[beta] < 0) continue; /* arcs into terminals do not reach level l */
      int v = B->first[l] + c[beta];
      mf[v] = rmin(mf[v], mf[u] + theta(B, l - 1, beta));
    }
  }
}

/* Alg. "Backward BDD update step" at level l: m_bwd(v) = min over the two out-arcs of m_bwd(child) + theta. */
static void backward_step(const bdd_t *B, REAL *mb, int l) {
  for (int u = B->first[l]; u < B->first[l + 1]; ++u)
    mb[u] = rmin(behind(B, mb, l, u, 0) + theta(B, l, 0), behind(B, mb, l, u, 1) + theta(B, l, 1));
}

/* eqs. "arc-marginal" and "marginal-aggregation": m^beta = min over beta-arcs uv leaving level l of
 * (m_fwd(u) + theta_uv) + m_bwd(v). */
static void level_min_marginals(const bdd_t *B, const REAL *mf, const REAL *mb, int l, REAL *m0, REAL *m1) {
  REAL best[2] = {REAL_INF, REAL_INF};
  for (int u = B->first[l]; u < B->first[l + 1]; ++u) {
    for (int beta = 0; beta < 2; ++beta) {
      REAL arc = (mf[u] + theta(B, l, beta)) + behind(B, mb, l, u, beta);
      best[beta] = rmin(best[beta], arc);
    }
  }
  *m0 = best[0];
  *m1 = best[1];
}

/* From scratch, on private message arrays: all forward steps, all backward steps. */
static void full_dp(const bdd_t *B, REAL *mf, REAL *mb) {
  for (int l = 0; l < B->k; ++l) forward_step(B, mf, l);
  for (int l = B->k - 1; l >= 0; --l) backward_step(B, mb, l);
}

/* E^j(lambda^j) = min over X_j of x^T lambda^j: the backward message of the root (0 without levels). */
static double energy_scratch(const bdd_t *B) {
  if (B->k == 0) return 0.0;
  int nn = B->first[B->k];
  REAL *mf = (REAL *)malloc((size_t)nn * sizeof(REAL)), *mb = (REAL *)malloc((size_t)nn * sizeof(REAL));
  full_dp(B, mf, mb);
  double e = (double)mb[B->first[0]];
  free(mf); free(mb);
  return e;
}

static void mm_scratch(const bdd_t *B, int l, REAL *m0, REAL *m1) {
  int nn = B->first[B->k];
  REAL *mf = (REAL *)malloc((size_t)nn * sizeof(REAL)), *mb = (REAL *)malloc((size_t)nn * sizeof(REAL));
  full_dp(B, mf, mb);
  level_min_marginals(B, mf, mb, l, m0, m1);
  free(mf); free(mb);
}

/* ---------------------------------------------------------------------------
 * Solver state
 * ------------------------------------------------------------------------- */
typedef struct orc_state {
  int n, m;
  double *cost;
  long long *row_ptr, *coef, *rhs;
  int *col;
  signed char *sense;
  int *order;
  bdd_t *bdd;                /* [m], one per row in row order */
  long long *canon;          /* [m+1] first canonical incidence of each diagram */
  long long *ncanon;         /* [m+1] first canonical node of each diagram */
  int *inc_ptr;              /* [n+1] incidences of each variable ... */
  int *inc_bdd, *inc_lvl;    /* ... as (row, level), ascending row */
  long long n_inc, n_nodes, n_live;
  double lb_const;           /* sum of min(0, c_i) over variables in no row */
  double lb;
  int inited, flags;
  double chk[4];
  REAL *dbuf;                /* scratch of max |J_i| differences */
  int maxJ;
  int split_k;               /* Sec. 6 variable intervals (0: no split) */
  REAL gamma;                /* copy-arc step size */
  int *intv;                 /* [n] interval of each variable */
  long long n_cuts, n_copy;  /* cut levels and copy-arc pairs */
} orc_state;

void orc_destroy(orc_state *S) {
  if (!S) return;
  if (S->bdd)
    for (int j = 0; j < S->m; ++j) free_bdd(&S->bdd[j]);
  free(S->bdd); free(S->cost); free(S->row_ptr); free(S->coef); free(S->rhs); free(S->col);
  free(S->sense); free(S->order); free(S->canon); free(S->ncanon); free(S->inc_ptr);
  free(S->inc_bdd); free(S->inc_lvl); free(S->dbuf); free(S->intv);
  free(S);
}

/*
 * Build every row's diagram. order[r] is the variable processed r-th; each row's
 * variables are taken in that order (the levels of its diagram).
 */
int orc_create(int n, const double *cost, int m, const long long *row_ptr, const int *col,
               const long long *coef, const signed char *sense, const long long *rhs,
               const int *order, long long node_budget, orc_state **out) {
  *out = NULL;
  if (n < 0 || m < 0 || (n > 0 && (!cost || !order)) || !row_ptr) return fail(ORC_INVALID_ARG, "null or negative argument", 0);
  orc_state *S = (orc_state *)calloc(1, sizeof(orc_state));
  if (!S) return ORC_NOMEM;
  S->n = n; S->m = m;
  long long nnz = row_ptr[m];
  S->cost = (double *)malloc((size_t)(n ? n : 1) * sizeof(double));
  S->row_ptr = (long long *)malloc((size_t)(m + 1) * sizeof(long long));
  S->col = (int *)malloc((size_t)(nnz ? nnz : 1) * sizeof(int));
  S->coef = (long long *)malloc((size_t)(nnz ? nnz : 1) * sizeof(long long));
  S->sense = (signed char *)malloc((size_t)(m ? m : 1));
  S->rhs = (long long *)malloc((size_t)(m ? m : 1) * sizeof(long long));
  S->order = (int *)malloc((size_t)(n ? n : 1) * sizeof(int));
  S->bdd = (bdd_t *)calloc((size_t)(m ? m : 1), sizeof(bdd_t));
  S->canon = (long long *)calloc((size_t)m + 1, sizeof(long long));
  S->ncanon = (long long *)calloc((size_t)m + 1, sizeof(long long));
  int *rank = (int *)malloc((size_t)(n ? n : 1) * sizeof(int));
  int *seen = (int *)malloc((size_t)(n ? n : 1) * sizeof(int));
  if (!S->cost || !S->row_ptr || !S->col || !S->coef || !S->sense || !S->rhs || !S->order || !S->bdd ||
      !S->canon || !S->ncanon || !rank || !seen) {
    free(rank); free(seen); orc_destroy(S); return ORC_NOMEM;
  }
  memcpy(S->cost, cost, (size_t)n * sizeof(double));
  memcpy(S->row_ptr, row_ptr, (size_t)(m + 1) * sizeof(long long));
  memcpy(S->col, col, (size_t)nnz * sizeof(int));
  memcpy(S->coef, coef, (size_t)nnz * sizeof(long long));
  memcpy(S->sense, sense, (size_t)m);
  memcpy(S->rhs, rhs, (size_t)m * sizeof(long long));
  memcpy(S->order, order, (size_t)n * sizeof(int));
  for (int i = 0; i < n; ++i) { rank[i] = -1; seen[i] = -1; }
  for (int r = 0; r < n; ++r) {
    if (order[r] < 0 || order[r] >= n || rank[order[r]] >= 0) { free(rank); free(seen); orc_destroy(S); return fail(ORC_INVALID_ARG, "order is not a permutation", r); }
    rank[order[r]] = r;
  }
  int rc = ORC_OK;
  int *vbuf = NULL; long long *abuf = NULL; long long vcap = 0;
  for (int j = 0; j < m && rc == ORC_OK; ++j) {
    long long a0 = row_ptr[j], a1 = row_ptr[j + 1];
    if (a1 < a0 || (sense[j] < 0 || sense[j] > 2)) { rc = fail(ORC_INVALID_ARG, "bad row", j); break; }
    if (a1 - a0 > vcap) {
      vcap = a1 - a0;
      free(vbuf); free(abuf);
      vbuf = (int *)malloc((size_t)vcap * sizeof(int));
      abuf = (long long *)malloc((size_t)vcap * sizeof(long long));
      if (!vbuf || !abuf) { rc = ORC_NOMEM; break; }
    }
    /* I_j: variables with a nonzero coefficient (Example "ILP"), sorted by processing rank */
    int k = 0;
    for (long long q = a0; q < a1; ++q) {
      int v = col[q];
      if (v < 0 || v >= n) { rc = fail(ORC_INVALID_ARG, "column out of range", q); break; }
      if (seen[v] == j) { rc = fail(ORC_INVALID_ARG, "duplicate column in a row", q); break; }
      seen[v] = j;
      if (coef[q] == 0) continue;
      /* insertion by rank keeps it simple */
      int p = k++;
      while (p > 0 && rank[vbuf[p - 1]] > rank[v]) { vbuf[p] = vbuf[p - 1]; abuf[p] = abuf[p - 1]; --p; }
      vbuf[p] = v; abuf[p] = coef[q];
    }
    if (rc != ORC_OK) break;
    rc = build_bdd(k, vbuf, abuf, sense[j], rhs[j], node_budget, &S->bdd[j]);
    if (rc == ORC_ROW_INFEASIBLE || rc == ORC_BDD_TOO_LARGE) {
      char m2[sizeof g_err];
      memcpy(m2, g_err, sizeof m2);
      snprintf(g_err, sizeof g_err, "row %d: %.400s", j, m2);
    }
  }
  free(vbuf); free(abuf); free(rank); free(seen);
  if (rc != ORC_OK) { orc_destroy(S); return rc; }

  /* canonical offsets and J_i in ascending row order */
  S->inc_ptr = (int *)calloc((size_t)n + 1, sizeof(int));
  if (!S->inc_ptr) { orc_destroy(S); return ORC_NOMEM; }
  for (int j = 0; j < m; ++j) {
    bdd_t *B = &S->bdd[j];
    S->canon[j + 1] = S->canon[j] + B->k;
    S->ncanon[j + 1] = S->ncanon[j] + B->first[B->k];
    for (int l = 0; l < B->k; ++l) S->inc_ptr[B->var[l] + 1]++;
    for (int u = 0; u < B->first[B->k]; ++u) S->n_live += (B->lo[u] != BOT) + (B->hi[u] != BOT);
  }
  S->n_inc = S->canon[m];
  S->n_nodes = S->ncanon[m];
  for (int i = 0; i < n; ++i) {
    if (S->inc_ptr[i + 1] > S->maxJ) S->maxJ = S->inc_ptr[i + 1];
    S->inc_ptr[i + 1] += S->inc_ptr[i];
  }
  S->inc_bdd = (int *)malloc((size_t)(S->n_inc ? S->n_inc : 1) * sizeof(int));
  S->inc_lvl = (int *)malloc((size_t)(S->n_inc ? S->n_inc : 1) * sizeof(int));
  S->dbuf = (REAL *)malloc((size_t)(S->maxJ ? S->maxJ : 1) * sizeof(REAL));
  int *fill = (int *)malloc((size_t)(n ? n : 1) * sizeof(int));
  if (!S->inc_bdd || !S->inc_lvl || !S->dbuf || !fill) { free(fill); orc_destroy(S); return ORC_NOMEM; }
  for (int i = 0; i < n; ++i) fill[i] = S->inc_ptr[i];
  for (int j = 0; j < m; ++j)
    for (int l = 0; l < S->bdd[j].k; ++l) {
      int v = S->bdd[j].var[l];
      S->inc_bdd[fill[v]] = j;
      S->inc_lvl[fill[v]] = l;
      fill[v]++;
    }
  free(fill);
  S->lb_const = 0.0;
  for (int i = 0; i < n; ++i)
    if (S->inc_ptr[i] == S->inc_ptr[i + 1] && cost[i] < 0) S->lb_const += cost[i];
  *out = S;
  return ORC_OK;
}

void orc_stats(const orc_state *S, long long *st) {
  st[0] = S->n; st[1] = S->m; st[2] = S->n_nodes; st[3] = S->n_live; st[4] = S->n_inc;
  st[5] = S->maxJ;
}

/* Canonical structure: per incidence (row, then level) the level's width and variable; per node
 * (row, level, in-level index) its children. */
void orc_structure(const orc_state *S, int *level_width, int *level_var, int *lo, int *hi) {
  long long qi = 0, qn = 0;
  for (int j = 0; j < S->m; ++j) {
    const bdd_t *B = &S->bdd[j];
    for (int l = 0; l < B->k; ++l) {
      level_width[qi] = B->first[l + 1] - B->first[l];
      level_var[qi] = B->var[l];
      ++qi;
    }
    for (int u = 0; u < B->first[B->k]; ++u) { lo[qn] = B->lo[u]; hi[qn] = B->hi[u]; ++qn; }
  }
}

/* E of the sub-BDD that starts after the cut at level l (Sec. 6): the best path enters through
 * one arc uv, costing its copy dual mu plus the backward message of v. */
static REAL cut_energy(const bdd_t *B, int l) {
  REAL e = REAL_INF;
  for (int u = B->first[l]; u < B->first[l + 1]; ++u) {
    int c[2] = {B->lo[u], B->hi[u]};
    for (int beta = 0; beta < 2; ++beta)
      if (c[beta] >= 0) e = rmin(e, B->mue[2 * u + beta] + B->mb[B->first[l + 1] + c[beta]]);
  }
  return e;
}

/* The dual bound: sum of E over all (sub-)BDDs, plus the variables in no row. */
static double lower_bound(const orc_state *S) {
  double lb = 0.0;
  for (int j = 0; j < S->m; ++j) {
    const bdd_t *B = &S->bdd[j];
    if (!B->k) continue;
    lb += (double)B->mb[B->first[0]];
    if (B->cut)
      for (int l = 0; l + 1 < B->k; ++l)
        if (B->cut[l]) lb += (double)cut_energy(B, l);
  }
  return lb + S->lb_const;
}

/*
 * The update of eq. "mma-update" for variable i given its differences d (one per row of J_i in
 * ascending row order). Forced rows (infinite d) follow the reading in the file header.
 */
static int apply_update(orc_state *S, int i, const REAL *d) {
  int a0 = S->inc_ptr[i], cnt = S->inc_ptr[i + 1] - a0;
  int nF = 0, pos = 0, neg = 0;
  REAL sum_fin = 0;
  for (int q = 0; q < cnt; ++q) {
    if (isinf(d[q])) { ++nF; if (d[q] > 0) pos = 1; else neg = 1; }
    else sum_fin += d[q];
  }
  if (pos && neg) return fail(ORC_CONFLICT, "rows force variable to both values", i);
  if (nF == 0) {
    REAL s = 0;
    for (int q = 0; q < cnt; ++q) s += d[q];
    REAL avg = s / (REAL)cnt;
    for (int q = 0; q < cnt; ++q) {
      bdd_t *B = &S->bdd[S->inc_bdd[a0 + q]];
      int l = S->inc_lvl[a0 + q];
      B->lam[l] = (B->lam[l] - d[q]) + avg;
    }
  } else {
    REAL share = sum_fin / (REAL)nF;
    for (int q = 0; q < cnt; ++q) {
      bdd_t *B = &S->bdd[S->inc_bdd[a0 + q]];
      int l = S->inc_lvl[a0 + q];
      if (isinf(d[q])) B->lam[l] = B->lam[l] + share;
      else B->lam[l] = B->lam[l] - d[q];
    }
  }
  return ORC_OK;
}

static double energy_of_var_rows(const orc_state *S, int i) {
  double e = 0.0;
  for (int q = S->inc_ptr[i]; q < S->inc_ptr[i + 1]; ++q) e += energy_scratch(&S->bdd[S->inc_bdd[q]]);
  return e;
}

static void note(double *slot, double v) { if (v > *slot || isnan(v)) *slot = v; }

/* process one variable inside a pass; fwd selects the forward box of Sec. 5.4 */
static int process_variable(orc_state *S, int i, int fwd) {
  int a0 = S->inc_ptr[i], cnt = S->inc_ptr[i + 1] - a0;
  if (cnt == 0) return ORC_OK;
  REAL *d = S->dbuf;
  for (int q = 0; q < cnt; ++q) {
    bdd_t *B = &S->bdd[S->inc_bdd[a0 + q]];
    int l = S->inc_lvl[a0 + q];
    REAL m0, m1;
    if (fwd) forward_step(B, B->mf, l); /* forward box: step, then min-marginals */
    level_min_marginals(B, B->mf, B->mb, l, &m0, &m1);
    d[q] = m1 - m0;
    if (S->flags & CHK_INCREMENTAL) {
      REAL f0, f1;
      mm_scratch(B, l, &f0, &f1);
      double e0 = (isinf(f0) && isinf(m0)) ? 0.0 : fabs((double)f0 - (double)m0);
      double e1 = (isinf(f1) && isinf(m1)) ? 0.0 : fabs((double)f1 - (double)m1);
      note(&S->chk[0], e0 > e1 ? e0 : e1);
    }
  }
  double before = 0.0, gain = 0.0;
  if (S->flags & CHK_PROP1) {
    before = energy_of_var_rows(S, i);
    /* Prop. 1: gain = min{0, sum_j d_j} - sum_j min{0, d_j}. With forced rows F the finite rows
     * gain -min{0, d_k} each; rows forcing x_i = 1 have E^j moving one-for-one with lambda^j_i and
     * so also gain the sum of the finite differences they absorb, rows forcing x_i = 0 gain nothing. */
    int nF = 0, to_one = 0; double sfin = 0.0, negpart = 0.0;
    for (int q = 0; q < cnt; ++q) {
      if (isinf(d[q])) { ++nF; to_one = d[q] < 0; continue; }
      sfin += (double)d[q];
      if (d[q] < 0) negpart += (double)d[q];
    }
    gain = nF ? (-negpart + (to_one ? sfin : 0.0)) : ((sfin < 0 ? sfin : 0.0) - negpart);
  }
  int rc = apply_update(S, i, d);
  if (rc != ORC_OK) return rc;
  if (S->flags & CHK_PROP1) {
    double after = energy_of_var_rows(S, i);
    double scale = fabs(before) + fabs(after) + 1.0;
    note(&S->chk[1], fabs((after - before) - gain) / scale);
  }
  if (S->flags & CHK_EQUAL_D) {
    /* after the update every row's difference is the mean (proof of Prop. 1); forced rows keep
     * their infinite difference and the others drop to zero */
    int nF = 0; double s = 0.0;
    for (int q = 0; q < cnt; ++q) { if (isinf(d[q])) ++nF; else s += (double)d[q]; }
    for (int q = 0; q < cnt; ++q) {
      bdd_t *B = &S->bdd[S->inc_bdd[a0 + q]];
      REAL f0, f1;
      mm_scratch(B, S->inc_lvl[a0 + q], &f0, &f1);
      double dn = (double)f1 - (double)f0;
      double want = nF ? 0.0 : s / cnt;
      if (nF && isinf(d[q])) continue;
      note(&S->chk[2], fabs(dn - want) / (1.0 + fabs(want)));
    }
  }
  if (S->flags & CHK_SUM_LAMBDA) {
    double s = 0.0;
    for (int q = 0; q < cnt; ++q) s += (double)S->bdd[S->inc_bdd[a0 + q]].lam[S->inc_lvl[a0 + q]];
    note(&S->chk[3], fabs(s - S->cost[i]) / (1.0 + fabs(S->cost[i])));
  }
  if (!fwd) /* backward box (read with the step after the update): min-marginals, update, step */
    for (int q = 0; q < cnt; ++q) {
      bdd_t *B = &S->bdd[S->inc_bdd[a0 + q]];
      backward_step(B, B->mb, S->inc_lvl[a0 + q]);
    }
  return ORC_OK;
}

/*
 * Initialisation of Alg. "Min-marginal averaging": lambda^j_i = c_i / |J_i|, then all backward
 * messages by backward steps from the last level up ("after initialization of all messages",
 * Prop. "correctness"). check_flags selects the per-update self checks (tiny inputs only).
 */
static void reset_copy_duals(orc_state *S);

int orc_init(orc_state *S, int check_flags) {
  if (S->split_k && check_flags) return fail(ORC_INVALID_ARG, "self checks apply to the unsplit decomposition", check_flags);
  reset_copy_duals(S);
  S->flags = check_flags;
  for (int k = 0; k < 4; ++k) S->chk[k] = 0.0;
  for (int i = 0; i < S->n; ++i) {
    int cnt = S->inc_ptr[i + 1] - S->inc_ptr[i];
    for (int q = S->inc_ptr[i]; q < S->inc_ptr[i + 1]; ++q)
      S->bdd[S->inc_bdd[q]].lam[S->inc_lvl[q]] = (REAL)(S->cost[i] / (double)cnt);
  }
  for (int j = 0; j < S->m; ++j) {
    bdd_t *B = &S->bdd[j];
    for (int l = B->k - 1; l >= 0; --l) backward_step(B, B->mb, l);
  }
  S->lb = lower_bound(S);
  S->inited = 1;
  return ORC_OK;
}

/* Replace every multiplier (canonical order) and re-initialise the backward messages. */
int orc_set_lambda(orc_state *S, const double *lam) {
  for (int j = 0; j < S->m; ++j)
    for (int l = 0; l < S->bdd[j].k; ++l) S->bdd[j].lam[l] = (REAL)lam[S->canon[j] + l];
  for (int j = 0; j < S->m; ++j)
    for (int l = S->bdd[j].k - 1; l >= 0; --l) backward_step(&S->bdd[j], S->bdd[j].mb, l);
  S->lb = lower_bound(S);
  S->inited = 1;
  return ORC_OK;
}

static void copy_update_forward(orc_state *S);
static void copy_update_backward(orc_state *S);

/* iters rounds of a forward pass over order[0..n-1] then a backward pass over order[n-1..0];
 * lb_trace[t] receives the bound after round t. With a split (Sec. 6, Alg. "Parallel min-marginal
 * averaging") each pass is followed by the copy-arc updates; the intervals are independent
 * within a pass, so visiting all variables in processing order is the parallel pass. */
int orc_iterate(orc_state *S, int iters, double *lb_trace) {
  if (!S->inited) return fail(ORC_BAD_STATE, "orc_init first", 0);
  for (int t = 0; t < iters; ++t) {
    for (int r = 0; r < S->n; ++r) {
      int rc = process_variable(S, S->order[r], 1);
      if (rc) return rc;
    }
    if (S->split_k) copy_update_forward(S);
    for (int r = S->n - 1; r >= 0; --r) {
      int rc = process_variable(S, S->order[r], 0);
      if (rc) return rc;
    }
    if (S->split_k) copy_update_backward(S);
    S->lb = lower_bound(S);
    if (lb_trace) lb_trace[t] = S->lb;
  }
  return ORC_OK;
}

double orc_lower_bound(const orc_state *S) { return S->lb; }

/* residual max_i |c_i - sum_j lambda^j_i| over variables with rows, and the bound that holds for any
 * lambda: sum_j E^j + sum_i min(0, c_i - sum_j lambda^j_i) (App. A.1). */
void orc_residual(const orc_state *S, double *resid, double *any_lambda_bound) {
  double r = 0.0, corr = 0.0;
  for (int i = 0; i < S->n; ++i) {
    if (S->inc_ptr[i] == S->inc_ptr[i + 1]) continue;
    double s = 0.0;
    for (int q = S->inc_ptr[i]; q < S->inc_ptr[i + 1]; ++q) s += (double)S->bdd[S->inc_bdd[q]].lam[S->inc_lvl[q]];
    double g = S->cost[i] - s;
    if (fabs(g) > r) r = fabs(g);
    if (g < 0) corr += g;
  }
  *resid = r;
  *any_lambda_bound = S->lb + corr;
}

void orc_lambda(const orc_state *S, double *lam) {
  for (int j = 0; j < S->m; ++j)
    for (int l = 0; l < S->bdd[j].k; ++l) lam[S->canon[j] + l] = (double)S->bdd[j].lam[l];
}

/* Fresh min-marginals at the current multipliers: a forward sweep without updates over every
 * diagram, then eq. "marginal-aggregation" per level (backward messages are current after a
 * backward pass or the initialisation). Canonical order. */
int orc_min_marginals(orc_state *S, double *m0, double *m1) {
  if (!S->inited) return fail(ORC_BAD_STATE, "orc_init first", 0);
  for (int j = 0; j < S->m; ++j) {
    bdd_t *B = &S->bdd[j];
    for (int l = 0; l < B->k; ++l) {
      REAL a, b;
      forward_step(B, B->mf, l);
      level_min_marginals(B, B->mf, B->mb, l, &a, &b);
      m0[S->canon[j] + l] = (double)a;
      m1[S->canon[j] + l] = (double)b;
    }
  }
  return ORC_OK;
}

/* Total min-marginal differences M_i = sum_j (m1 - m0) in ascending row order (Sec. 4), preferred
 * values x_i = [M_i <= 0], x_i = [c_i < 0] for variables in no row, the objective c^T x and the
 * number of rows x violates (integer arithmetic on the rows). Uses fresh min-marginals. */
int orc_round(orc_state *S, double *M, signed char *x, double *obj, long long *nviol) {
  if (!S->inited) return fail(ORC_BAD_STATE, "orc_init first", 0);
  long long I = S->n_inc;
  double *m0 = (double *)malloc((size_t)(I ? I : 1) * sizeof(double));
  double *m1 = (double *)malloc((size_t)(I ? I : 1) * sizeof(double));
  if (!m0 || !m1) { free(m0); free(m1); return ORC_NOMEM; }
  orc_min_marginals(S, m0, m1);
  for (int i = 0; i < S->n; ++i) {
    if (S->inc_ptr[i] == S->inc_ptr[i + 1]) { M[i] = 0.0; x[i] = S->cost[i] < 0; continue; }
    REAL s = 0;
    for (int q = S->inc_ptr[i]; q < S->inc_ptr[i + 1]; ++q) {
      long long c = S->canon[S->inc_bdd[q]] + S->inc_lvl[q];
      s += (REAL)m1[c] - (REAL)m0[c];
    }
    M[i] = (double)s;
    x[i] = s <= 0;
  }
  double o = 0.0;
  for (int i = 0; i < S->n; ++i)
    if (x[i]) o += S->cost[i];
  *obj = o;
  long long bad = 0;
  for (int j = 0; j < S->m; ++j) {
    long long lhs = 0;
    for (long long q = S->row_ptr[j]; q < S->row_ptr[j + 1]; ++q) lhs += S->coef[q] * (long long)x[S->col[q]];
    bad += !row_holds(S->sense[j], lhs, S->rhs[j]);
  }
  *nviol = bad;
  free(m0); free(m1);
  return ORC_OK;
}

/* |X_j| per row by the counting algebra of Table "algebras" ((*, +, 1, 0, [1, 1]) in the abstract
 * backward step), accumulated in double. */
void orc_count_solutions(const orc_state *S, double *count) {
  for (int j = 0; j < S->m; ++j) {
    const bdd_t *B = &S->bdd[j];
    if (B->k == 0) { count[j] = 1.0; continue; }
    int nn = B->first[B->k];
    double *c = (double *)malloc((size_t)nn * sizeof(double));
    for (int l = B->k - 1; l >= 0; --l)
      for (int u = B->first[l]; u < B->first[l + 1]; ++u) {
        double s = 0.0;
        int ch[2] = {B->lo[u], B->hi[u]};
        for (int beta = 0; beta < 2; ++beta)
          s += ch[beta] == TOP ? 1.0 : ch[beta] == BOT ? 0.0 : c[B->first[l + 1] + ch[beta]];
        c[u] = s;
      }
    count[j] = c[B->first[0]];
    free(c);
  }
}

/* ---------------------------------------------------------------------------
 * Sec. 6: variable intervals, sub-BDDs and copy-arc duals
 *
 * The processing order is cut into K intervals of about equal node count: a variable counts the
 * nodes of its levels over all its rows, and the variable at order position r (c_r nodes before
 * it, N in total) lies in interval floor(K c_r / N). A row's diagram is cut between consecutive
 * levels in different intervals (Def. "Sub-BDD"): the sub-BDD before the cut ends with arcs into
 * TOP (the copy-arcs), the sub-BDD after it starts at the same arcs, whose tails act as its
 * roots. Each pair carries a dual: mu_bar on the copy-arc, mu on the arc; their sum stays <= 0.
 * Readings: the arc's lambda is counted in the sub-BDD before the cut (the tail's variable lies
 * in that interval), so the entering arc costs mu alone; the minimum in the copy-arc updates
 * runs over the pairs of one cut (the arcs a sub-BDD ends or starts with), which keeps every
 * difference non-negative as Prop. "correctness-parallel" uses; the forward update takes the
 * arc-marginals after the pass (with the last level's updated lambda), the backward one the
 * backward messages after the pass; the bound is taken after the backward copy update.
 * ------------------------------------------------------------------------- */

static void reset_copy_duals(orc_state *S) {
  if (!S->split_k) return;
  for (int j = 0; j < S->m; ++j) {
    bdd_t *B = &S->bdd[j];
    if (!B->mux) continue;
    size_t na = (size_t)2 * (size_t)B->first[B->k];
    for (size_t q = 0; q < na; ++q) B->mux[q] = B->mue[q] = B->dfw[q] = B->dbw[q] = 0;
  }
}

/* after the forward pass: for the copy-arcs closing each cut's earlier sub-BDD,
 * delta_fwd = m(copy-arc) - min over the cut's copy-arcs, mu_bar <- mu_bar - g delta_fwd + g delta_bwd */
static void copy_update_forward(orc_state *S) {
  REAL g = S->gamma;
  for (int j = 0; j < S->m; ++j) {
    bdd_t *B = &S->bdd[j];
    if (!B->cut) continue;
    for (int l = 0; l + 1 < B->k; ++l) {
      if (!B->cut[l]) continue;
      REAL mn = REAL_INF;
      for (int u = B->first[l]; u < B->first[l + 1]; ++u)
        for (int beta = 0; beta < 2; ++beta) {
          if ((beta ? B->hi[u] : B->lo[u]) < 0) continue;
          int q = 2 * u + beta;
          mn = rmin(mn, (B->mf[u] + theta(B, l, beta)) + B->mux[q]);
        }
      for (int u = B->first[l]; u < B->first[l + 1]; ++u)
        for (int beta = 0; beta < 2; ++beta) {
          if ((beta ? B->hi[u] : B->lo[u]) < 0) continue;
          int q = 2 * u + beta;
          REAL m = (B->mf[u] + theta(B, l, beta)) + B->mux[q];
          B->dfw[q] = m - mn;
          B->mux[q] = (B->mux[q] - g * B->dfw[q]) + g * B->dbw[q];
        }
    }
  }
}

/* after the backward pass: for the arcs opening each cut's later sub-BDD,
 * delta_bwd = m(arc) - min over the cut's arcs, mu <- mu - g delta_bwd + g delta_fwd */
static void copy_update_backward(orc_state *S) {
  REAL g = S->gamma;
  for (int j = 0; j < S->m; ++j) {
    bdd_t *B = &S->bdd[j];
    if (!B->cut) continue;
    for (int l = 0; l + 1 < B->k; ++l) {
      if (!B->cut[l]) continue;
      REAL mn = REAL_INF;
      for (int u = B->first[l]; u < B->first[l + 1]; ++u)
        for (int beta = 0; beta < 2; ++beta) {
          int c = beta ? B->hi[u] : B->lo[u];
          if (c < 0) continue;
          mn = rmin(mn, B->mue[2 * u + beta] + B->mb[B->first[l + 1] + c]);
        }
      for (int u = B->first[l]; u < B->first[l + 1]; ++u)
        for (int beta = 0; beta < 2; ++beta) {
          int c = beta ? B->hi[u] : B->lo[u];
          if (c < 0) continue;
          int q = 2 * u + beta;
          REAL m = B->mue[q] + B->mb[B->first[l + 1] + c];
          B->dbw[q] = m - mn;
          B->mue[q] = (B->mue[q] - g * B->dbw[q]) + g * B->dfw[q];
        }
    }
  }
}

/* Split every row at the boundaries of K variable intervals (K <= 1: no split) with copy-arc step
 * size gamma in (0, 1]. Call before orc_init; the duals start at 0. */
int orc_split(orc_state *S, int K, double gamma) {
  if (K < 0 || !(gamma > 0.0 && gamma <= 1.0)) return fail(ORC_INVALID_ARG, "K >= 0 and 0 < gamma <= 1", K);
  for (int j = 0; j < S->m; ++j) {
    bdd_t *B = &S->bdd[j];
    free(B->cut); free(B->mux); free(B->mue); free(B->dfw); free(B->dbw);
    B->cut = NULL; B->mux = B->mue = B->dfw = B->dbw = NULL;
  }
  free(S->intv);
  S->intv = NULL;
  S->split_k = 0;
  S->n_cuts = S->n_copy = 0;
  S->inited = 0;
  if (K <= 1) return ORC_OK;
  S->split_k = K;
  S->gamma = (REAL)gamma;
  S->intv = (int *)calloc((size_t)(S->n ? S->n : 1), sizeof(int));
  long long *cnt = (long long *)calloc((size_t)(S->n ? S->n : 1), sizeof(long long));
  if (!S->intv || !cnt) { free(cnt); return ORC_NOMEM; }
  long long total = 0;
  for (int j = 0; j < S->m; ++j) {
    bdd_t *B = &S->bdd[j];
    for (int l = 0; l < B->k; ++l) cnt[B->var[l]] += B->first[l + 1] - B->first[l];
  }
  for (int i = 0; i < S->n; ++i) total += cnt[i];
  long long before = 0;
  for (int r = 0; r < S->n; ++r) {
    int i = S->order[r];
    S->intv[i] = total ? (int)((long long)K * before / total) : 0;
    before += cnt[i];
  }
  free(cnt);
  for (int j = 0; j < S->m; ++j) {
    bdd_t *B = &S->bdd[j];
    int any = 0;
    for (int l = 0; l + 1 < B->k; ++l) any |= S->intv[B->var[l]] != S->intv[B->var[l + 1]];
    if (!any) continue;
    size_t na = (size_t)2 * (size_t)B->first[B->k];
    B->cut = (unsigned char *)calloc((size_t)B->k, 1);
    B->mux = (REAL *)calloc(na, sizeof(REAL));
    B->mue = (REAL *)calloc(na, sizeof(REAL));
    B->dfw = (REAL *)calloc(na, sizeof(REAL));
    B->dbw = (REAL *)calloc(na, sizeof(REAL));
    if (!B->cut || !B->mux || !B->mue || !B->dfw || !B->dbw) return ORC_NOMEM;
    for (int l = 0; l + 1 < B->k; ++l)
      if (S->intv[B->var[l]] != S->intv[B->var[l + 1]]) {
        B->cut[l] = 1;
        S->n_cuts++;
        for (int u = B->first[l]; u < B->first[l + 1]; ++u) S->n_copy += (B->lo[u] >= 0) + (B->hi[u] >= 0);
      }
  }
  return ORC_OK;
}

/* split summary: K, cut levels, copy-arc pairs; intv[n] (may be NULL) receives each variable's interval */
void orc_split_info(const orc_state *S, long long *out3, int *intv) {
  out3[0] = S->split_k;
  out3[1] = S->n_cuts;
  out3[2] = S->n_copy;
  if (intv)
    for (int i = 0; i < S->n; ++i) intv[i] = S->intv ? S->intv[i] : 0;
}

/* Copy duals per pair in canonical order (rows, cut levels ascending, tail node, arc label):
 * mu_bar[n_copy], mu[n_copy]; row_of, level_of, node_of (in-level index), label_of may be NULL. */
void orc_copy_duals(const orc_state *S, double *mu_bar, double *mu, int *row_of, int *level_of, int *node_of,
                    int *label_of) {
  long long q = 0;
  for (int j = 0; j < S->m; ++j) {
    const bdd_t *B = &S->bdd[j];
    if (!B->cut) continue;
    for (int l = 0; l + 1 < B->k; ++l) {
      if (!B->cut[l]) continue;
      for (int u = B->first[l]; u < B->first[l + 1]; ++u)
        for (int beta = 0; beta < 2; ++beta) {
          if ((beta ? B->hi[u] : B->lo[u]) < 0) continue;
          int a = 2 * u + beta;
          if (mu_bar) mu_bar[q] = (double)B->mux[a];
          if (mu) mu[q] = (double)B->mue[a];
          if (row_of) row_of[q] = j;
          if (level_of) level_of[q] = l;
          if (node_of) node_of[q] = u - B->first[l];
          if (label_of) label_of[q] = beta;
          ++q;
        }
    }
  }
}

void orc_checks(const orc_state *S, double *out4) {
  for (int k = 0; k < 4; ++k) out4[k] = S->chk[k];
}

/* One row's diagram on its own (tests): levels in the given order. Returns the node count,
 * or a negative status; writes widths[k], lo/hi[nodes] when the buffers are large enough. */
long long orc_build_row(int k, const long long *a, int sense, long long b, long long budget,
                        int *widths, int *lo, int *hi, long long cap) {
  bdd_t B;
  int *vars = (int *)malloc((size_t)(k ? k : 1) * sizeof(int));
  for (int t = 0; t < k; ++t) vars[t] = t;
  int rc = build_bdd(k, vars, a, sense, b, budget, &B);
  free(vars);
  if (rc != ORC_OK) { free_bdd(&B); return rc; }
  long long nn = B.first[k];
  if (nn <= cap) {
    for (int t = 0; t < k; ++t) widths[t] = B.first[t + 1] - B.first[t];
    for (long long u = 0; u < nn; ++u) { lo[u] = B.lo[u]; hi[u] = B.hi[u]; }
  }
  free_bdd(&B);
  return nn;
}

/* ---------------------------------------------------------------------------
 * Smoothed variant (App. "Smoothing"). The (+, min) algebra of the steps becomes the marginal
 * log-sum-exp algebra of Table "algebras", kept in the log domain: min(a, b) is replaced by the
 * soft minimum smin(a, b) = -alpha log(exp(-a/alpha) + exp(-b/alpha)), so the forward, backward
 * and marginal values are -alpha log of the path sums of exp(-cost/alpha). The update is eq.
 * "mma-update" on these marginal values. Readings (design notes): the bound adds
 * smin(0, c_i) for each variable in no row (its two assignments); several arguments fold left in
 * the order of the min-plus code. When rows force the variable (an infinite difference), the
 * smoothed block maximum is not attained, and the min-plus forced-row rule can lower the smoothed
 * bound (by up to alpha log 2 per row it moves); instead only the rows whose move raises the bound
 * hand their difference to the forced rows: with rows forcing x_i = 1 those with d_k > 0, with
 * rows forcing x_i = 0 those with d_k < 0 (each then has d_k = 0; the forced rows share the sum).
 *
 * The derivative of the smoothed bound after T iterations with respect to the costs is computed
 * by reverse accumulation: lambda after each iteration is kept (an iteration is a function of
 * lambda alone, because the backward messages it starts from are the backward sweep of lambda),
 * each iteration is recomputed from its checkpoint, then its backward pass and its forward pass
 * are undone in reverse order, every step passing adjoints back through the soft-minimum weights
 * exp(-(argument - result)/alpha), which are the derivatives of smin.
 * ------------------------------------------------------------------------- */

static REAL smin(REAL a, REAL b, double alpha) {
  REAL lo = a < b ? a : b, hi = a < b ? b : a;
  if (isinf(hi)) return lo;
  return (REAL)((double)lo - alpha * log1p(exp(-((double)hi - (double)lo) / alpha)));
}

/* derivative of s = smin(..., a, ...) with respect to argument a */
static double sweight(REAL a, REAL s, double alpha) {
  if (isinf(a) || isinf(s)) return 0.0;
  return exp(-((double)a - (double)s) / alpha);
}

static REAL child_val(const REAL *mb, const bdd_t *B, int l, int c) {
  if (c == TOP) return (REAL)0;
  if (c == BOT) return REAL_INF;
  return mb[B->first[l + 1] + c];
}

/* smoothed Alg. "Forward BDD update step" at level l (lam: the diagram's multipliers) */
static void forward_step_s(const bdd_t *B, const REAL *lam, REAL *mf, int l, double alpha) {
  if (l == 0) { mf[B->first[0]] = 0; return; }
  for (int v = B->first[l]; v < B->first[l + 1]; ++v) mf[v] = REAL_INF;
  for (int u = B->first[l - 1]; u < B->first[l]; ++u) {
    int c[2] = {B->lo[u], B->hi[u]};
    for (int beta = 0; beta < 2; ++beta) {
      if (c[beta] < 0) continue;
      int v = B->first[l] + c[beta];
      mf[v] = smin(mf[v], mf[u] + (beta ? lam[l - 1] : (REAL)0), alpha);
    }
  }
}

/* smoothed Alg. "Backward BDD update step" at level l */
static void backward_step_s(const bdd_t *B, const REAL *lam, REAL *mb, int l, double alpha) {
  for (int u = B->first[l]; u < B->first[l + 1]; ++u)
    mb[u] = smin(child_val(mb, B, l, B->lo[u]), child_val(mb, B, l, B->hi[u]) + lam[l], alpha);
}

/* eq. "marginal-log-sum-exp" at level l through arc values (m_fwd + theta) + m_bwd */
static void level_marginals_s(const bdd_t *B, const REAL *lam, const REAL *mf, const REAL *mb, int l,
                              REAL *m0, REAL *m1, double alpha) {
  REAL best[2] = {REAL_INF, REAL_INF};
  for (int u = B->first[l]; u < B->first[l + 1]; ++u) {
    int c[2] = {B->lo[u], B->hi[u]};
    for (int beta = 0; beta < 2; ++beta) {
      REAL arc = (mf[u] + (beta ? lam[l] : (REAL)0)) + child_val(mb, B, l, c[beta]);
      best[beta] = smin(best[beta], arc, alpha);
    }
  }
  *m0 = best[0];
  *m1 = best[1];
}

static double lower_bound_s(const orc_state *S, double alpha) {
  double lb = 0.0;
  for (int j = 0; j < S->m; ++j)
    if (S->bdd[j].k) lb += (double)S->bdd[j].mb[S->bdd[j].first[0]];
  for (int i = 0; i < S->n; ++i)
    if (S->inc_ptr[i] == S->inc_ptr[i + 1]) lb += (double)smin((REAL)0, (REAL)S->cost[i], alpha);
  return lb;
}

/* the smoothed update (forced rows as in the header of this section) */
static int apply_update_s(orc_state *S, int i, const REAL *d) {
  int a0 = S->inc_ptr[i], cnt = S->inc_ptr[i + 1] - a0;
  int nF = 0, pos = 0, neg = 0;
  for (int q = 0; q < cnt; ++q)
    if (isinf(d[q])) { ++nF; if (d[q] > 0) pos = 1; else neg = 1; }
  if (pos && neg) return fail(ORC_CONFLICT, "rows force variable to both values", i);
  if (nF == 0) return apply_update(S, i, d);
  REAL moved = 0;
  for (int q = 0; q < cnt; ++q)
    if (!isinf(d[q]) && (neg ? d[q] > 0 : d[q] < 0)) moved += d[q];
  REAL share = moved / (REAL)nF;
  for (int q = 0; q < cnt; ++q) {
    bdd_t *B = &S->bdd[S->inc_bdd[a0 + q]];
    int l = S->inc_lvl[a0 + q];
    if (isinf(d[q])) B->lam[l] = B->lam[l] + share;
    else if (neg ? d[q] > 0 : d[q] < 0) B->lam[l] = B->lam[l] - d[q];
  }
  return ORC_OK;
}

static int process_variable_s(orc_state *S, int i, int fwd, double alpha) {
  int a0 = S->inc_ptr[i], cnt = S->inc_ptr[i + 1] - a0;
  if (cnt == 0) return ORC_OK;
  REAL *d = S->dbuf;
  for (int q = 0; q < cnt; ++q) {
    bdd_t *B = &S->bdd[S->inc_bdd[a0 + q]];
    int l = S->inc_lvl[a0 + q];
    REAL m0, m1;
    if (fwd) forward_step_s(B, B->lam, B->mf, l, alpha);
    level_marginals_s(B, B->lam, B->mf, B->mb, l, &m0, &m1, alpha);
    d[q] = m1 - m0;
  }
  int rc = apply_update_s(S, i, d);
  if (rc != ORC_OK) return rc;
  if (!fwd)
    for (int q = 0; q < cnt; ++q) {
      bdd_t *B = &S->bdd[S->inc_bdd[a0 + q]];
      backward_step_s(B, B->lam, B->mb, S->inc_lvl[a0 + q], alpha);
    }
  return ORC_OK;
}

static void sweep_s(orc_state *S, double alpha) {
  for (int j = 0; j < S->m; ++j) {
    bdd_t *B = &S->bdd[j];
    for (int l = B->k - 1; l >= 0; --l) backward_step_s(B, B->lam, B->mb, l, alpha);
  }
}

static void init_lambda(orc_state *S) {
  for (int i = 0; i < S->n; ++i) {
    int cnt = S->inc_ptr[i + 1] - S->inc_ptr[i];
    for (int q = S->inc_ptr[i]; q < S->inc_ptr[i + 1]; ++q)
      S->bdd[S->inc_bdd[q]].lam[S->inc_lvl[q]] = (REAL)(S->cost[i] / (double)cnt);
  }
}

/* Smoothed initialisation: lambda = c / |J_i|, smoothed backward messages, LB_alpha. */
int orc_smooth_init(orc_state *S, double alpha) {
  if (S->split_k) return fail(ORC_INVALID_ARG, "the smoothed variant runs on the unsplit decomposition", S->split_k);
  if (!(alpha > 0)) return fail(ORC_INVALID_ARG, "alpha must be positive", 0);
  S->flags = 0;
  init_lambda(S);
  sweep_s(S, alpha);
  S->lb = lower_bound_s(S, alpha);
  S->inited = 2;
  return ORC_OK;
}

static int smooth_round(orc_state *S, double alpha) {
  for (int r = 0; r < S->n; ++r) {
    int rc = process_variable_s(S, S->order[r], 1, alpha);
    if (rc) return rc;
  }
  for (int r = S->n - 1; r >= 0; --r) {
    int rc = process_variable_s(S, S->order[r], 0, alpha);
    if (rc) return rc;
  }
  return ORC_OK;
}

int orc_smooth_iterate(orc_state *S, double alpha, int iters, double *lb_trace) {
  if (S->inited != 2) return fail(ORC_BAD_STATE, "orc_smooth_init first", 0);
  for (int t = 0; t < iters; ++t) {
    int rc = smooth_round(S, alpha);
    if (rc) return rc;
    S->lb = lower_bound_s(S, alpha);
    if (lb_trace) lb_trace[t] = S->lb;
  }
  return ORC_OK;
}

/* Fresh marginal log-sum-exp values at the current multipliers (canonical order). */
int orc_smooth_marginals(orc_state *S, double alpha, double *m0, double *m1) {
  if (S->inited != 2) return fail(ORC_BAD_STATE, "orc_smooth_init first", 0);
  for (int j = 0; j < S->m; ++j) {
    bdd_t *B = &S->bdd[j];
    for (int l = 0; l < B->k; ++l) {
      REAL a, b;
      forward_step_s(B, B->lam, B->mf, l, alpha);
      level_marginals_s(B, B->lam, B->mf, B->mb, l, &a, &b, alpha);
      m0[S->canon[j] + l] = (double)a;
      m1[S->canon[j] + l] = (double)b;
    }
  }
  return ORC_OK;
}

/* Per row at the current multipliers, from scratch: E^j (min-plus) and E^j_alpha (smoothed). */
void orc_row_energies(const orc_state *S, double alpha, double *e, double *e_alpha) {
  for (int j = 0; j < S->m; ++j) {
    const bdd_t *B = &S->bdd[j];
    if (B->k == 0) { e[j] = e_alpha[j] = 0.0; continue; }
    e[j] = energy_scratch(B);
    int nn = B->first[B->k];
    REAL *mb = (REAL *)malloc((size_t)nn * sizeof(REAL));
    for (int l = B->k - 1; l >= 0; --l) backward_step_s(B, B->lam, mb, l, alpha);
    e_alpha[j] = (double)mb[B->first[0]];
    free(mb);
  }
}

/* ---- reverse accumulation ---- */

typedef struct {
  double alpha;
  const REAL *mf;    /* forward messages the pass used (flat, canonical node order) */
  const REAL *mb;    /* backward messages the step read (flat) */
  const REAL *lam0;  /* multipliers before the update (flat, canonical incidence order) */
  const REAL *lam1;  /* multipliers after the update */
  double *gmf, *gmb, *glam;
} rev_t;

static void set_lam(orc_state *S, const double *lam) {
  for (int j = 0; j < S->m; ++j)
    for (int l = 0; l < S->bdd[j].k; ++l) S->bdd[j].lam[l] = (REAL)lam[S->canon[j] + l];
}
static void get_lam(const orc_state *S, REAL *lam) {
  for (int j = 0; j < S->m; ++j)
    for (int l = 0; l < S->bdd[j].k; ++l) lam[S->canon[j] + l] = S->bdd[j].lam[l];
}
static void get_msgs(const orc_state *S, REAL *flat, int which) {
  for (int j = 0; j < S->m; ++j) {
    const bdd_t *B = &S->bdd[j];
    if (!B->k) continue;
    memcpy(flat + S->ncanon[j], which ? B->mb : B->mf, (size_t)B->first[B->k] * sizeof(REAL));
  }
}

/* undo the backward step of level l of diagram j (its values: mb, multiplier lam[l]) */
static void rev_bstep(const orc_state *S, int j, int l, const REAL *mb, const REAL *lam, double *gmb,
                      double *glam, double alpha) {
  const bdd_t *B = &S->bdd[j];
  long long nb = S->ncanon[j], c = S->canon[j];
  for (int u = B->first[l]; u < B->first[l + 1]; ++u) {
    double g = gmb[nb + u];
    gmb[nb + u] = 0.0;
    if (g == 0.0) continue;
    REAL x0 = child_val(mb + nb, B, l, B->lo[u]), x1 = child_val(mb + nb, B, l, B->hi[u]) + lam[c + l];
    REAL s = mb[nb + u];
    double w0 = sweight(x0, s, alpha), w1 = sweight(x1, s, alpha);
    if (B->lo[u] >= 0) gmb[nb + B->first[l + 1] + B->lo[u]] += g * w0;
    if (B->hi[u] >= 0) gmb[nb + B->first[l + 1] + B->hi[u]] += g * w1;
    glam[c + l] += g * w1;
  }
}

/* undo the marginals of level l: adjoints gm0, gm1 of m0, m1 go to mf (level l), mb (level l+1)
 * and the multiplier lam[l] */
static void rev_marginals(const orc_state *S, int j, int l, const rev_t *R, double gm0, double gm1) {
  const bdd_t *B = &S->bdd[j];
  long long nb = S->ncanon[j], c = S->canon[j];
  REAL m0, m1;
  level_marginals_s(B, R->lam0 + c, R->mf + nb, R->mb + nb, l, &m0, &m1, R->alpha);
  for (int u = B->first[l]; u < B->first[l + 1]; ++u) {
    int ch[2] = {B->lo[u], B->hi[u]};
    for (int beta = 0; beta < 2; ++beta) {
      double g = beta ? gm1 : gm0;
      if (g == 0.0) continue;
      REAL arc = (R->mf[nb + u] + (beta ? R->lam0[c + l] : (REAL)0)) + child_val(R->mb + nb, B, l, ch[beta]);
      double w = sweight(arc, beta ? m1 : m0, R->alpha);
      R->gmf[nb + u] += g * w;
      if (ch[beta] >= 0) R->gmb[nb + B->first[l + 1] + ch[beta]] += g * w;
      if (beta) R->glam[c + l] += g * w;
    }
  }
}

/* undo the forward step that produced level l (l >= 1) from level l-1 with multiplier lam[l-1] */
static void rev_fstep(const orc_state *S, int j, int l, const REAL *mf, const REAL *lam, double *gmf,
                      double *glam, double alpha) {
  const bdd_t *B = &S->bdd[j];
  long long nb = S->ncanon[j], c = S->canon[j];
  for (int u = B->first[l - 1]; u < B->first[l]; ++u) {
    int ch[2] = {B->lo[u], B->hi[u]};
    for (int beta = 0; beta < 2; ++beta) {
      if (ch[beta] < 0) continue;
      int v = B->first[l] + ch[beta];
      double g = gmf[nb + v];
      if (g == 0.0) continue;
      REAL arg = mf[nb + u] + (beta ? lam[c + l - 1] : (REAL)0);
      double w = sweight(arg, mf[nb + v], alpha);
      gmf[nb + u] += g * w;
      if (beta) glam[c + l - 1] += g * w;
    }
  }
  for (int v = B->first[l]; v < B->first[l + 1]; ++v) gmf[nb + v] = 0.0;
}

/* undo the update of variable i: glam holds the adjoints of the updated multipliers; on return
 * it holds those of the multipliers before the update, and gd the adjoints of the differences */
static void rev_update(const orc_state *S, int i, const REAL *d, const double *glam1, double *gd) {
  int a0 = S->inc_ptr[i], cnt = S->inc_ptr[i + 1] - a0;
  int nF = 0, neg = 0;
  double gsum = 0.0, gforced = 0.0;
  for (int q = 0; q < cnt; ++q) {
    if (isinf(d[q])) { ++nF; gforced += glam1[q]; if (d[q] < 0) neg = 1; }
    gsum += glam1[q];
  }
  for (int q = 0; q < cnt; ++q) {
    if (nF == 0) gd[q] = -glam1[q] + gsum / cnt;
    else if (!isinf(d[q]) && (neg ? d[q] > 0 : d[q] < 0)) gd[q] = -glam1[q] + gforced / nF;
    else gd[q] = 0.0;
  }
}

/*
 * Gradient of LB_alpha after T smoothed iterations (started by orc_smooth_init) with respect to
 * the costs: grad[n]; *lb_out = LB_alpha(T). Leaves the state after the T iterations.
 */
int orc_smooth_grad(orc_state *S, double alpha, int T, double *grad, double *lb_out) {
  if (S->split_k) return fail(ORC_INVALID_ARG, "the smoothed variant runs on the unsplit decomposition", S->split_k);
  int rc = orc_smooth_init(S, alpha);
  if (rc) return rc;
  long long I = S->n_inc, N = S->n_nodes;
  size_t nI = (size_t)(I ? I : 1), nN = (size_t)(N ? N : 1);
  REAL *ck = (REAL *)malloc(nI * (size_t)(T + 1) * sizeof(REAL));
  REAL *lam_mid = (REAL *)malloc(nI * sizeof(REAL)), *lam_end = (REAL *)malloc(nI * sizeof(REAL));
  REAL *mf = (REAL *)malloc(nN * sizeof(REAL)), *mbT = (REAL *)malloc(nN * sizeof(REAL));
  REAL *mbE = (REAL *)malloc(nN * sizeof(REAL));
  double *gmf = (double *)calloc(nN, sizeof(double)), *gmb = (double *)calloc(nN, sizeof(double));
  double *glam = (double *)calloc(nI, sizeof(double));
  double *gl1 = (double *)malloc((size_t)(S->maxJ ? S->maxJ : 1) * sizeof(double));
  double *gd = (double *)malloc((size_t)(S->maxJ ? S->maxJ : 1) * sizeof(double));
  REAL *dv = (REAL *)malloc((size_t)(S->maxJ ? S->maxJ : 1) * sizeof(REAL));
  if (!ck || !lam_mid || !lam_end || !mf || !mbT || !mbE || !gmf || !gmb || !glam || !gl1 || !gd || !dv) {
    rc = ORC_NOMEM;
    goto out;
  }
  get_lam(S, ck);
  for (int t = 0; t < T; ++t) {
    if ((rc = smooth_round(S, alpha))) goto out;
    get_lam(S, ck + nI * (size_t)(t + 1));
  }
  S->lb = lower_bound_s(S, alpha);
  if (lb_out) *lb_out = S->lb;
  /* seed: d LB / d (root backward message) = 1 for every diagram */
  for (int j = 0; j < S->m; ++j)
    if (S->bdd[j].k) gmb[S->ncanon[j] + S->bdd[j].first[0]] = 1.0;
  for (int t = T - 1; t >= 0; --t) {
    /* recompute iteration t from its checkpoint */
    double *lt = (double *)malloc(nI * sizeof(double));
    for (size_t q = 0; q < (size_t)I; ++q) lt[q] = (double)ck[nI * (size_t)t + q];
    set_lam(S, lt);
    free(lt);
    sweep_s(S, alpha);
    get_msgs(S, mbT, 1);
    for (int r = 0; r < S->n; ++r)
      if ((rc = process_variable_s(S, S->order[r], 1, alpha))) goto out;
    get_lam(S, lam_mid);
    get_msgs(S, mf, 0);
    for (int r = S->n - 1; r >= 0; --r)
      if ((rc = process_variable_s(S, S->order[r], 0, alpha))) goto out;
    get_lam(S, lam_end);
    get_msgs(S, mbE, 1);
    /* undo the backward pass: variables in forward order */
    rev_t RB = {alpha, mf, mbE, lam_mid, lam_end, gmf, gmb, glam};
    for (int r = 0; r < S->n; ++r) {
      int i = S->order[r], a0 = S->inc_ptr[i], cnt = S->inc_ptr[i + 1] - a0;
      if (!cnt) continue;
      for (int q = 0; q < cnt; ++q)
        rev_bstep(S, S->inc_bdd[a0 + q], S->inc_lvl[a0 + q], mbE, lam_end, gmb, glam, alpha);
      for (int q = 0; q < cnt; ++q) {
        int j = S->inc_bdd[a0 + q], l = S->inc_lvl[a0 + q];
        long long nb = S->ncanon[j], c = S->canon[j];
        REAL m0, m1;
        level_marginals_s(&S->bdd[j], lam_mid + c, mf + nb, mbE + nb, l, &m0, &m1, alpha);
        dv[q] = m1 - m0;
        gl1[q] = glam[c + l];
      }
      rev_update(S, i, dv, gl1, gd);
      for (int q = 0; q < cnt; ++q)
        if (!isinf(dv[q])) rev_marginals(S, S->inc_bdd[a0 + q], S->inc_lvl[a0 + q], &RB, -gd[q], gd[q]);
    }
    /* undo the forward pass: variables in backward order */
    rev_t RF = {alpha, mf, mbT, ck + nI * (size_t)t, lam_mid, gmf, gmb, glam};
    for (int r = S->n - 1; r >= 0; --r) {
      int i = S->order[r], a0 = S->inc_ptr[i], cnt = S->inc_ptr[i + 1] - a0;
      if (!cnt) continue;
      for (int q = 0; q < cnt; ++q) {
        int j = S->inc_bdd[a0 + q], l = S->inc_lvl[a0 + q];
        long long nb = S->ncanon[j], c = S->canon[j];
        REAL m0, m1;
        level_marginals_s(&S->bdd[j], RF.lam0 + c, mf + nb, mbT + nb, l, &m0, &m1, alpha);
        dv[q] = m1 - m0;
        gl1[q] = glam[c + l];
      }
      rev_update(S, i, dv, gl1, gd);
      for (int q = 0; q < cnt; ++q) {
        int j = S->inc_bdd[a0 + q], l = S->inc_lvl[a0 + q];
        if (!isinf(dv[q])) rev_marginals(S, j, l, &RF, -gd[q], gd[q]);
        if (l > 0) rev_fstep(S, j, l, mf, lam_mid, gmf, glam, alpha);
        else gmf[S->ncanon[j] + S->bdd[j].first[0]] = 0.0;
      }
    }
  }
  /* undo the initial backward sweep (multipliers c / |J_i|), root level first */
  {
    double *l0 = (double *)malloc(nI * sizeof(double));
    for (size_t q = 0; q < (size_t)I; ++q) l0[q] = (double)ck[q];
    set_lam(S, l0);
    free(l0);
    sweep_s(S, alpha);
    get_msgs(S, mbT, 1);
    for (int j = 0; j < S->m; ++j)
      for (int l = 0; l < S->bdd[j].k; ++l) rev_bstep(S, j, l, mbT, ck, gmb, glam, alpha);
  }
  for (int i = 0; i < S->n; ++i) {
    int a0 = S->inc_ptr[i], cnt = S->inc_ptr[i + 1] - a0;
    if (!cnt) {
      REAL s = smin((REAL)0, (REAL)S->cost[i], alpha);
      grad[i] = sweight((REAL)S->cost[i], s, alpha);
      continue;
    }
    double g = 0.0;
    for (int q = 0; q < cnt; ++q) g += glam[S->canon[S->inc_bdd[a0 + q]] + S->inc_lvl[a0 + q]];
    grad[i] = g / cnt;
  }
  /* leave the state after the T iterations */
  {
    double *le = (double *)malloc(nI * sizeof(double));
    for (size_t q = 0; q < (size_t)I; ++q) le[q] = (double)ck[nI * (size_t)T + q];
    set_lam(S, le);
    free(le);
    sweep_s(S, alpha);
  }
out:
  free(ck); free(lam_mid); free(lam_end); free(mf); free(mbT); free(mbE);
  free(gmf); free(gmb); free(glam); free(gl1); free(gd); free(dv);
  return rc;
}
