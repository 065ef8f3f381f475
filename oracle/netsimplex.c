/*
 * netsimplex.c -- exact optimum of the transportation problem by the primal
 * network simplex method.  TEST INFRASTRUCTURE ONLY: it gives the oracle an
 * exact optimal value for instances too large for a generic LP solver; the
 * GPU library never links or calls it.
 *
 * The problem is eq. (1) of the paper,
 *     min <C, X>  s.t.  X e = p,  X^T f = q,  X >= 0,
 * a minimum-cost flow on the bipartite network with a source node i of supply
 * p_i per row, a sink node j of demand q_j per column, and an uncapacitated
 * arc i -> j of cost C_ij for every pair.  Its dual is eq. (3):
 *     max p^T u + q^T v  s.t.  u_i + v_j <= C_ij.
 *
 * Method (the textbook primal network simplex with a big-M start):
 *  - an extra root node and one artificial arc per node (source i -> root
 *    with flow p_i, or root -> i when p_i = 0; root -> sink j with flow q_j),
 *    each of cost M larger than the cost of any path of real arcs, form the
 *    first spanning-tree basis (every zero-flow tree arc points away from the
 *    root, so the tree is strongly feasible);
 *  - node potentials pi make every tree arc's reduced cost
 *    c + pi(tail) - pi(head) zero; a real arc with a negative reduced cost
 *    enters (the most negative of a block of arcs, blocks taken in turn);
 *  - the entering arc closes a cycle with the tree path between its ends;
 *    the flow around the cycle grows until a tree arc traversed against its
 *    direction reaches zero, and that arc leaves -- with ties broken by the
 *    last such arc met when walking the cycle from its apex in the direction
 *    of the entering arc, which keeps the tree strongly feasible and rules
 *    out cycling;
 *  - the subtree cut off by the leaving arc is re-hung from the entering arc
 *    and its potentials shift by one constant;
 *  - optimal when no real arc has a reduced cost below -eps.
 * With the marginals on a dyadic grid (as every generator in this project
 * makes them) all flows are exact binary fractions, so the plan meets its
 * marginals exactly.  u_i = -pi_i, v_j = pi_j are the dual variables.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int64_t m, n, N; /* sources 0..m-1, sinks m..m+n-1, root N-1 */
  const double* C;
  double M;        /* cost of the artificial arcs */
  double* pi;      /* node potentials */
  int64_t* parent;
  int64_t* arc;    /* tree arc to the parent: i * n + j for a real arc, -1 artificial */
  unsigned char* up; /* the tree arc points from the node to its parent */
  double* flow;    /* flow on the tree arc to the parent */
  int64_t* depth;
  int64_t *child, *next, *prev; /* first child; doubly linked siblings */
  int64_t* stack;
} Tree;

static void unlink_child(Tree* t, int64_t w) {
  const int64_t par = t->parent[w];
  if (t->prev[w] >= 0) t->next[t->prev[w]] = t->next[w];
  else t->child[par] = t->next[w];
  if (t->next[w] >= 0) t->prev[t->next[w]] = t->prev[w];
  t->prev[w] = t->next[w] = -1;
}

static void link_child(Tree* t, int64_t par, int64_t w) {
  t->parent[w] = par;
  t->prev[w] = -1;
  t->next[w] = t->child[par];
  if (t->child[par] >= 0) t->prev[t->child[par]] = w;
  t->child[par] = w;
}

/* Reduced cost of the real arc i -> sink j. */
static inline double rcost(const Tree* t, int64_t i, int64_t j) {
  return t->C[i * t->n + j] + t->pi[i] - t->pi[t->m + j];
}

/* Returns 0 on success, -1 on allocation failure, -2 if the problem is
 * infeasible (unequal masses), -3 if the pivot limit is reached.
 * Outputs (each may be NULL): X (m x n, dense, row-major), u (m), v (n),
 * *obj (sum C_ij X_ij), *pivots. */
int drot_ref_netsimplex(int64_t m, int64_t n, const double* C, const double* p, const double* q,
                        double eps, int64_t max_pivots, double* X, double* u, double* v,
                        double* obj, int64_t* pivots) {
  Tree t;
  memset(&t, 0, sizeof t);
  t.m = m;
  t.n = n;
  t.N = m + n + 1;
  t.C = C;
  const int64_t N = t.N, root = N - 1;
  double cmax = 0.0;
  for (int64_t k = 0; k < m * n; ++k) cmax = fmax(cmax, fabs(C[k]));
  t.M = (cmax + 1.0) * (double)N;
  t.pi = malloc(sizeof(double) * N);
  t.parent = malloc(sizeof(int64_t) * N);
  t.arc = malloc(sizeof(int64_t) * N);
  t.up = malloc(N);
  t.flow = malloc(sizeof(double) * N);
  t.depth = malloc(sizeof(int64_t) * N);
  t.child = malloc(sizeof(int64_t) * N);
  t.next = malloc(sizeof(int64_t) * N);
  t.prev = malloc(sizeof(int64_t) * N);
  t.stack = malloc(sizeof(int64_t) * N);
  int rc = 0;
  if (!t.pi || !t.parent || !t.arc || !t.up || !t.flow || !t.depth || !t.child || !t.next ||
      !t.prev || !t.stack) {
    rc = -1;
    goto out;
  }
  /* Star basis of artificial arcs. */
  for (int64_t w = 0; w < N; ++w) {
    t.child[w] = t.next[w] = t.prev[w] = -1;
    t.arc[w] = -1;
  }
  t.parent[root] = -1;
  t.depth[root] = 0;
  t.pi[root] = 0.0;
  t.flow[root] = 0.0;
  t.up[root] = 0;
  for (int64_t w = 0; w < m + n; ++w) {
    link_child(&t, root, w);
    t.depth[w] = 1;
    if (w < m && p[w] > 0.0) {  /* source -> root, cost M: pi_w = -M */
      t.up[w] = 1;
      t.flow[w] = p[w];
      t.pi[w] = -t.M;
    } else {                   /* root -> node, cost M: pi_w = +M */
      t.up[w] = 0;
      t.flow[w] = w < m ? 0.0 : q[w - m];
      t.pi[w] = t.M;
    }
  }

  const int64_t arcs = m * n;
  int64_t block = (int64_t)sqrt((double)arcs);
  if (block < 64) block = 64;
  if (block > arcs) block = arcs;
  int64_t pos = 0, npiv = 0;
  for (;;) {
    /* Pricing: the most negative reduced cost of the next block that has one. */
    int64_t best = -1;
    double best_rc = -eps;
    int64_t scanned = 0;
    while (scanned < arcs) {
      const int64_t end = pos + block < arcs ? pos + block : arcs;
      for (int64_t a = pos; a < end; ++a) {
        const double r = rcost(&t, a / n, a % n);
        if (r < best_rc) {
          best_rc = r;
          best = a;
        }
      }
      scanned += end - pos;
      pos = end == arcs ? 0 : end;
      if (best >= 0) break;
    }
    if (best < 0) break; /* optimal */
    if (npiv >= max_pivots) {
      rc = -3;
      goto out;
    }
    ++npiv;
    const int64_t s = best / n, tt = m + best % n; /* entering arc s -> tt */

    /* Apex of the cycle. */
    int64_t a = s, b = tt;
    while (a != b) {
      if (t.depth[a] >= t.depth[b]) a = t.parent[a];
      else b = t.parent[b];
    }
    const int64_t join = a;

    /* Leaving arc: the s side is walked against the cycle's direction
     * (first minimum wins), the tt side along it (last minimum wins). */
    double delta = INFINITY;
    int64_t out_node = -1;
    int side = 0;
    for (int64_t w = s; w != join; w = t.parent[w])
      if (t.up[w] && t.flow[w] < delta) {
        delta = t.flow[w];
        out_node = w;
        side = 1;
      }
    for (int64_t w = tt; w != join; w = t.parent[w])
      if (!t.up[w] && t.flow[w] <= delta) {
        delta = t.flow[w];
        out_node = w;
        side = 2;
      }
    if (out_node < 0) { /* cannot happen: the artificial arcs bound every cycle */
      rc = -2;
      goto out;
    }
    for (int64_t w = s; w != join; w = t.parent[w]) t.flow[w] += t.up[w] ? -delta : delta;
    for (int64_t w = tt; w != join; w = t.parent[w]) t.flow[w] += t.up[w] ? delta : -delta;

    /* Re-hang the cut subtree: its new root `r0` is the entering arc's end
     * inside it, its new parent the other end. */
    const int64_t r0 = side == 1 ? s : tt, newpar = side == 1 ? tt : s;
    const double shift = side == 1 ? -best_rc : best_rc;
    int64_t prev_node = newpar, carry_arc = best;
    unsigned char carry_up = side == 1 ? 1 : 0;
    double carry_flow = delta;
    for (int64_t w = r0;;) {
      const int64_t old_par = t.parent[w];
      const int64_t oa = t.arc[w];
      const unsigned char ou = t.up[w];
      const double of = t.flow[w];
      unlink_child(&t, w);
      link_child(&t, prev_node, w);
      t.arc[w] = carry_arc;
      t.up[w] = carry_up;
      t.flow[w] = carry_flow;
      if (w == out_node) break;
      prev_node = w;
      carry_arc = oa;
      carry_up = (unsigned char)!ou;
      carry_flow = of;
      w = old_par;
    }
    /* Depths and potentials of the re-hung subtree. */
    int64_t sp = 0;
    t.stack[sp++] = r0;
    while (sp > 0) {
      const int64_t w = t.stack[--sp];
      t.depth[w] = t.depth[t.parent[w]] + 1;
      t.pi[w] += shift;
      for (int64_t c = t.child[w]; c >= 0; c = t.next[c]) t.stack[sp++] = c;
    }
  }

  /* Every artificial arc must carry zero flow at the optimum. */
  for (int64_t w = 0; w < m + n; ++w)
    if (t.arc[w] < 0 && t.flow[w] != 0.0) {
      rc = -2;
      goto out;
    }
  {
    long double total = 0.0L;
    if (X) memset(X, 0, sizeof(double) * (size_t)(m * n));
    for (int64_t w = 0; w < m + n; ++w) {
      if (t.arc[w] < 0) continue;
      if (X) X[t.arc[w]] = t.flow[w];
      total += (long double)C[t.arc[w]] * (long double)t.flow[w];
    }
    if (obj) *obj = (double)total;
    if (u)
      for (int64_t i = 0; i < m; ++i) u[i] = -t.pi[i];
    if (v)
      for (int64_t j = 0; j < n; ++j) v[j] = t.pi[m + j];
    if (pivots) *pivots = npiv;
  }
out:
  free(t.pi);
  free(t.parent);
  free(t.arc);
  free(t.up);
  free(t.flow);
  free(t.depth);
  free(t.child);
  free(t.next);
  free(t.prev);
  free(t.stack);
  return rc;
}
