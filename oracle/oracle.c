/*
 * ORACLE -- test infrastructure, not part of the product.
 *
 * A plain, slow, sequential CPU implementation of max-flow min-cut pair
 * refinement as described in Section 4.1 of Sanders & Schulz, "Engineering
 * Multilevel Graph Partitioning Algorithms" ("Using Max-Flow Min-Cut
 * Computations for Local Improvement").  Only the test suite, the smoke check
 * and the CPU-baseline leg of the benchmark may load it.  It shares no code,
 * header or table with the GPU library.
 *
 * Everything is integer; flows, cuts and weights are int64.
 *
 * Steps, in the paper's order:
 *   - boundary nodes delta_l / delta_r            (Sec. 4.1, notation)
 *   - two bounded BFS growing the corridor B      (Sec. 4.1, construction)
 *   - corridor border and the s-t network G'      (Sec. 4.1, construction)
 *   - max flow (Dinic's blocking-flow algorithm, Dinic 1970: any exact
 *     max-flow algorithm gives the same value and residual closure)
 *   - smallest source set = vertices reachable from s in the residual graph
 *     (Sec. 4.1.1, Ford-Fulkerson labelling)
 *   - optionally, the most balanced minimum cut instead (Sec. 4.1.1): strongly
 *     connected components of the residual graph, removal of the sink's
 *     component with its predecessors and of the source's with its
 *     successors, then sweeps along random topological orders of what is left
 *   - balance check and adaptive flow iterations  (Sec. 4.1, improvements)
 *   - balance constraint L_max and cut objective  (Sec. 2.1)
 *
 * Readings where the paper is silent (all listed in the design notes):
 *   R2  only blocks a and b matter: border and BFS work in G[A u B]
 *   R3  BFS levels in ascending vertex id; a level is walked in that order
 *       and the walk stops at the first vertex that would exceed the bound
 *   R4  area bound U_x(alpha) = floor((1+alpha*eps) c(V)/k) - c(other block),
 *       eps in parts per million, clamped at 0
 *   R5  acceptance uses L_max with the original eps (plus max_v c(v))
 *   R6  adaptive loop: start at the given alpha; apply => alpha=min(2a,amax);
 *       reject => alpha=max(a/2,1) (stop if it was 1); feasible and not
 *       improving => stop; at most max_iters solves
 *   R6b restart_alpha > 0 (set with a learned start, which the paper does
 *       not have): a search that started below min(restart_alpha, amax),
 *       has applied nothing and meets a feasible, non-improving solve
 *       continues once from that factor instead of stopping, within the
 *       same max_iters, so the plain search decides before the pair gives up
 *   R8  the first block of the pair is the source side
 *   R9  DEPTH mode includes BFS distance <= depth from the boundary
 *   R12 2-way FM before the flow (Sec. 2.2, KaPPa's local search with TopGain):
 *       one queue per block of the pair, ordered by gain, equal gains by a
 *       per-vertex SplitMix64 key (larger first); boundary vertices start in
 *       the queues, a vertex joins its queue when a neighbour moves, and moves
 *       at most once; TopGain picks the block with the larger top gain (a
 *       random bit on ties), the heavier block while one is overloaded;
 *       stop after fm_limit moves without a better state or when both queues
 *       are empty; roll back to the best state: feasible before infeasible,
 *       then the smaller cut (feasible) or the lighter heavier block
 *       (infeasible), the earliest on ties
 *   R30 terminals 1: instead of pinning the corridor border to s and t with
 *       infinite arcs, the parts of blocks a and b outside the corridor are
 *       contracted into s and t; a corridor vertex gets an arc s -> u with the
 *       weight of its edges into a outside the corridor and an arc u -> t with
 *       the weight of its edges into b outside; edges between the two
 *       outside parts are cut whatever happens (constant); so every corridor
 *       vertex may change sides and the min cut is the best reassignment of
 *       the corridor
 *   R11 most balanced cut: balance of a cut = the heavier of the two new block
 *       weights; a random topological order takes, among the components whose
 *       predecessors are all placed, the one with the smallest key, keys from
 *       SplitMix64; first best wins (earlier sweep, then earlier position);
 *       the sweeps run for any number of remaining components
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int32_t n;
  const int32_t *xadj;
  const int32_t *adjncy;
  const int32_t *vwgt;
  const int32_t *adjwgt;
} or_graph;

typedef struct {
  int32_t area_mode; /* 0 = weight bound (alpha), 1 = BFS depth */
  int32_t depth;
  int32_t alpha;
  int32_t alpha_max;
  int32_t adaptive;
  int32_t max_iters;
  int32_t eps_ppm;
  int32_t mb_reps;  /* 0: smallest source set; > 0: most balanced minimum cut, this many sweeps */
  int32_t mb_seed;  /* seed of the sweeps' random keys (its 32 bits, zero-extended) */
  int32_t fm_limit; /* 0: no FM; > 0: 2-way FM before the flow, stop after this many moves
                       without improvement */
  int32_t fm_seed;  /* seed of the FM keys and tie bits (its 32 bits, zero-extended) */
  int32_t active_blocks; /* sweeps: refine only pairs with a block changed in the previous sweep */
  int32_t cut_side; /* without mb_reps: 0 smallest source set, 1 largest, 2 the smallest unless
                       it is infeasible and the largest is feasible */
  int32_t terminals; /* 0: corridor border pinned to s / t by infinite arcs (Sec. 4.1);
                        1: the blocks' outside parts contracted into s / t (arcs of weight omega) */
  int32_t mt_alpha; /* 0: no multi-try FM; > 0: after the pairwise improvements of a batch, one
                       multi-try round per pair (Sec. 4.2), stopping rule parameter alpha */
  int32_t mt_seed;  /* seed of the multi-try keys (its 32 bits, zero-extended) */
  int32_t restart_alpha; /* 0: none; > 0: the one restart of rule R6b from this factor */
} or_params;

/* one flow solve */
typedef struct {
  int32_t alpha;
  int32_t decision; /* 1 apply, 2 infeasible, 3 feasible not improving, 4 not adjacent */
  int64_t flow;
  int64_t region_vertices;
  int64_t region_edges;
  int64_t source_side;   /* corridor vertices ending on the source side */
  int64_t cut_before;    /* pair cut before this solve */
  int64_t cut_candidate; /* pair cut of the candidate partition */
  int64_t wa, wb;        /* block weights of the candidate */
} or_solve;

typedef struct {
  int32_t status; /* 1 accepted, 2 rejected (imbalance), 3 no improvement, 4 not adjacent */
  int32_t iters;
  int32_t final_alpha;
  int32_t applied;
  int32_t iter_cap; /* 1 if the loop ended only because of max_iters */
  int32_t pad;
  int64_t flow_value;
  int64_t cut_before, cut_after;
  int64_t weight_a, weight_b;
  int64_t region_vertices, region_edges;
  int64_t mt_kept; /* multi-try moves kept (after the pairwise improvement) */
} or_result;

enum { DEC_APPLY = 1, DEC_INFEASIBLE = 2, DEC_EQUAL = 3, DEC_NOT_ADJ = 4 };
enum { ST_ACCEPTED = 1, ST_REJECTED = 2, ST_NO_IMPROVEMENT = 3, ST_NOT_ADJACENT = 4 };

/* ------------------------------------------------------------------------ */
/* graph validation                                                          */

/* 0 ok; -1 bad graph.  Symmetric, positive edge weights, no self loops, no
 * parallel arcs, non-negative vertex weights (Sec. 2.1: omega > 0, c >= 0). */
int32_t or_validate_graph(const or_graph *g) {
  if (g->n < 0 || g->xadj[0] != 0) return -1;
  for (int32_t u = 0; u < g->n; u++) {
    if (g->xadj[u + 1] < g->xadj[u]) return -1;
    if (g->vwgt[u] < 0) return -1;
  }
  int32_t *mark = (int32_t *)malloc(sizeof(int32_t) * (size_t)(g->n ? g->n : 1));
  if (!mark) return -1;
  for (int32_t u = 0; u < g->n; u++) mark[u] = -1;
  int32_t rc = 0;
  for (int32_t u = 0; u < g->n && rc == 0; u++) {
    for (int32_t e = g->xadj[u]; e < g->xadj[u + 1]; e++) {
      int32_t v = g->adjncy[e];
      if (v < 0 || v >= g->n || v == u || g->adjwgt[e] < 1 || mark[v] == u) { rc = -1; break; }
      mark[v] = u;
      /* the reverse arc must exist with the same weight */
      int found = 0;
      for (int32_t f = g->xadj[v]; f < g->xadj[v + 1]; f++)
        if (g->adjncy[f] == u) { found = g->adjwgt[f] == g->adjwgt[e]; break; }
      if (!found) { rc = -1; break; }
    }
  }
  free(mark);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* generic max flow on a small directed network (Dinic)                      */

typedef struct {
  int32_t nn;      /* nodes */
  int64_t na, cap; /* arcs used / allocated; arc i^1 is the reverse of arc i */
  int32_t *tail, *head;
  int64_t *res;    /* residual capacity */
  int64_t *cap0;   /* original capacity */
  int64_t *off;    /* [nn+1] arcs grouped by tail */
  int64_t *byt;    /* arc ids grouped by tail */
} or_net;

static int net_init(or_net *N, int32_t nn, int64_t max_arcs) {
  memset(N, 0, sizeof(*N));
  N->nn = nn;
  N->cap = max_arcs > 0 ? max_arcs : 1;
  N->tail = (int32_t *)malloc(sizeof(int32_t) * (size_t)N->cap);
  N->head = (int32_t *)malloc(sizeof(int32_t) * (size_t)N->cap);
  N->res = (int64_t *)malloc(sizeof(int64_t) * (size_t)N->cap);
  N->cap0 = (int64_t *)malloc(sizeof(int64_t) * (size_t)N->cap);
  return (N->tail && N->head && N->res && N->cap0) ? 0 : -1;
}

static void net_free(or_net *N) {
  free(N->tail); free(N->head); free(N->res); free(N->cap0); free(N->off); free(N->byt);
  memset(N, 0, sizeof(*N));
}

/* add arc u->v with capacity c and its reverse v->u with capacity rc */
static void net_add(or_net *N, int32_t u, int32_t v, int64_t c, int64_t rc) {
  int64_t i = N->na;
  if (i + 2 > N->cap) abort(); /* sized too small by the caller: a bug, never data */
  N->tail[i] = u; N->head[i] = v; N->res[i] = c; N->cap0[i] = c;
  N->tail[i + 1] = v; N->head[i + 1] = u; N->res[i + 1] = rc; N->cap0[i + 1] = rc;
  N->na += 2;
}

static int net_finish(or_net *N) {
  N->off = (int64_t *)calloc((size_t)N->nn + 1, sizeof(int64_t));
  N->byt = (int64_t *)malloc(sizeof(int64_t) * (size_t)(N->na ? N->na : 1));
  if (!N->off || !N->byt) return -1;
  for (int64_t i = 0; i < N->na; i++) N->off[N->tail[i] + 1]++;
  for (int32_t v = 0; v < N->nn; v++) N->off[v + 1] += N->off[v];
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ((size_t)N->nn + 1));
  if (!fill) return -1;
  memcpy(fill, N->off, sizeof(int64_t) * ((size_t)N->nn + 1));
  for (int64_t i = 0; i < N->na; i++) N->byt[fill[N->tail[i]]++] = i;
  free(fill);
  return 0;
}

/* Dinic: repeat { BFS level graph from s over residual arcs; if t is not
 * reached stop; find augmenting s-t paths along level-increasing residual
 * arcs with current-arc pointers until none is left }.  Returns the flow. */
static int64_t net_dinic(or_net *N, int32_t s, int32_t t) {
  int32_t nn = N->nn;
  int32_t *level = (int32_t *)malloc(sizeof(int32_t) * (size_t)nn);
  int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)nn);
  int64_t *it = (int64_t *)malloc(sizeof(int64_t) * (size_t)nn);
  int64_t *path = (int64_t *)malloc(sizeof(int64_t) * (size_t)nn);
  int64_t flow = 0;
  if (!level || !queue || !it || !path) { flow = -1; goto done; }
  if (s == t) goto done;
  for (;;) {
    for (int32_t v = 0; v < nn; v++) level[v] = -1;
    int32_t qh = 0, qt = 0;
    level[s] = 0;
    queue[qt++] = s;
    while (qh < qt) {
      int32_t v = queue[qh++];
      for (int64_t j = N->off[v]; j < N->off[v + 1]; j++) {
        int64_t a = N->byt[j];
        if (N->res[a] > 0 && level[N->head[a]] < 0) {
          level[N->head[a]] = level[v] + 1;
          queue[qt++] = N->head[a];
        }
      }
    }
    if (level[t] < 0) break;
    for (int32_t v = 0; v < nn; v++) it[v] = N->off[v];
    /* blocking flow: depth-first search for s-t paths in the level graph */
    int32_t v = s;
    int64_t plen = 0;
    for (;;) {
      if (v == t) {
        int64_t b = N->res[path[0]];
        for (int64_t i = 1; i < plen; i++) if (N->res[path[i]] < b) b = N->res[path[i]];
        for (int64_t i = 0; i < plen; i++) { N->res[path[i]] -= b; N->res[path[i] ^ 1] += b; }
        flow += b;
        v = s;
        plen = 0;
        continue;
      }
      int advanced = 0;
      while (it[v] < N->off[v + 1]) {
        int64_t a = N->byt[it[v]];
        int32_t w = N->head[a];
        if (N->res[a] > 0 && level[w] == level[v] + 1) {
          path[plen++] = a;
          v = w;
          advanced = 1;
          break;
        }
        it[v]++;
      }
      if (advanced) continue;
      /* dead end: v leaves the level graph; retreat one arc */
      level[v] = -1;
      if (v == s) break;
      plen--;
      v = N->tail[path[plen]];
      it[v]++;
    }
  }
done:
  free(level); free(queue); free(it); free(path);
  return flow;
}

/* T-side closure: reach[v] = 1 iff t is reachable from v over arcs with
 * positive residual (a BFS from t over the reverses of residual arcs) */
static void net_reach_to(const or_net *N, int32_t t, uint8_t *reach, int32_t *queue) {
  memset(reach, 0, (size_t)N->nn);
  int32_t qh = 0, qt = 0;
  reach[t] = 1;
  queue[qt++] = t;
  while (qh < qt) {
    int32_t w = queue[qh++];
    for (int64_t j = N->off[w]; j < N->off[w + 1]; j++) {
      int64_t a = N->byt[j] ^ 1; /* the arc v -> w */
      int32_t v = N->tail[a];
      if (N->res[a] > 0 && !reach[v]) { reach[v] = 1; queue[qt++] = v; }
    }
  }
}

/* reach[v] = 1 iff v is reachable from s over arcs with positive residual */
static void net_reach(const or_net *N, int32_t s, uint8_t *reach, int32_t *queue) {
  memset(reach, 0, (size_t)N->nn);
  int32_t qh = 0, qt = 0;
  reach[s] = 1;
  queue[qt++] = s;
  while (qh < qt) {
    int32_t v = queue[qh++];
    for (int64_t j = N->off[v]; j < N->off[v + 1]; j++) {
      int64_t a = N->byt[j];
      if (N->res[a] > 0 && !reach[N->head[a]]) { reach[N->head[a]] = 1; queue[qt++] = N->head[a]; }
    }
  }
}

/* Max flow on an explicit network given as arcs (tail, head, cap); every arc
 * gets a zero-capacity reverse.  Writes the flow value and, if reach != NULL,
 * the smallest source set (nodes reachable from s in the final residual
 * graph).  Returns 0, or -1 on bad input. */
int32_t or_maxflow(int32_t nn, int64_t narcs, const int32_t *tails, const int32_t *heads,
                   const int64_t *caps, int32_t s, int32_t t, int64_t *flow_out,
                   uint8_t *reach) {
  if (nn <= 0 || s < 0 || s >= nn || t < 0 || t >= nn || s == t) return -1;
  or_net N;
  if (net_init(&N, nn, 2 * narcs) != 0) { net_free(&N); return -1; }
  for (int64_t i = 0; i < narcs; i++) {
    if (tails[i] < 0 || tails[i] >= nn || heads[i] < 0 || heads[i] >= nn || caps[i] < 0) {
      net_free(&N);
      return -1;
    }
    net_add(&N, tails[i], heads[i], caps[i], 0);
  }
  if (net_finish(&N) != 0) { net_free(&N); return -1; }
  *flow_out = net_dinic(&N, s, t);
  if (reach) {
    int32_t *q = (int32_t *)malloc(sizeof(int32_t) * (size_t)nn);
    net_reach(&N, s, reach, q);
    free(q);
  }
  net_free(&N);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* most balanced minimum cut (Sec. 4.1.1)                                    */

/* SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014): the generator started at `seed` adds the golden
 * gamma to its state per call and returns the state through a 64-bit finaliser
 * (xor-shift 30, multiply, xor-shift 27, multiply, xor-shift 31).  Output
 * number n >= 1 is therefore a function of seed + n * gamma alone. */
static uint64_t splitmix64_out(uint64_t seed, uint64_t n) {
  uint64_t z = seed + n * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint64_t or_splitmix64(uint64_t seed, uint64_t n) { return splitmix64_out(seed, n); }

/* key of a component with identifier id (its smallest global vertex id) in
 * sweep r: output number r * 2^32 + id + 1 of the generator */
static uint64_t mb_key(uint64_t seed, int32_t r, int32_t id) {
  return splitmix64_out(seed, (((uint64_t)(uint32_t)r << 32) | (uint32_t)id) + 1);
}

/* Strongly connected components of the directed graph formed by the arcs with
 * positive residual capacity (Tarjan 1972): depth-first search keeping the
 * visit index and the lowest index reachable through the search tree and the
 * vertices still on the component stack; a vertex whose lowest index is its
 * own closes a component.  Recursion replaced by an explicit stack of (vertex,
 * next arc).  comp[v] in [0, nc), components numbered in closing order.
 * Returns nc, or -1 when out of memory. */
static int32_t net_scc(const or_net *N, int32_t *comp) {
  int32_t nn = N->nn;
  int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)nn);
  int32_t *low = (int32_t *)malloc(sizeof(int32_t) * (size_t)nn);
  int32_t *stk = (int32_t *)malloc(sizeof(int32_t) * (size_t)nn);
  int32_t *cv = (int32_t *)malloc(sizeof(int32_t) * (size_t)nn);
  int64_t *cp = (int64_t *)malloc(sizeof(int64_t) * (size_t)nn);
  uint8_t *on = (uint8_t *)calloc((size_t)nn, 1);
  int32_t nc = 0;
  if (!idx || !low || !stk || !cv || !cp || !on) { nc = -1; goto done; }
  for (int32_t v = 0; v < nn; v++) idx[v] = -1;
  int32_t next = 0, ns = 0;
  for (int32_t root = 0; root < nn; root++) {
    if (idx[root] >= 0) continue;
    int32_t depth = 0;
    cv[0] = root;
    cp[0] = N->off[root];
    idx[root] = low[root] = next++;
    stk[ns++] = root;
    on[root] = 1;
    while (depth >= 0) {
      int32_t v = cv[depth];
      if (cp[depth] < N->off[v + 1]) {
        int64_t a = N->byt[cp[depth]++];
        if (N->res[a] <= 0) continue;
        int32_t w = N->head[a];
        if (idx[w] < 0) {  /* tree arc: descend */
          idx[w] = low[w] = next++;
          stk[ns++] = w;
          on[w] = 1;
          depth++;
          cv[depth] = w;
          cp[depth] = N->off[w];
        } else if (on[w] && idx[w] < low[v]) {
          low[v] = idx[w];
        }
        continue;
      }
      /* all arcs of v done */
      if (low[v] == idx[v]) {
        int32_t x;
        do {
          x = stk[--ns];
          on[x] = 0;
          comp[x] = nc;
        } while (x != v);
        nc++;
      }
      depth--;
      if (depth >= 0 && low[v] < low[cv[depth]]) low[cv[depth]] = low[v];
    }
  }
done:
  free(idx); free(low); free(stk); free(cv); free(cp); free(on);
  return nc;
}

typedef struct {
  int32_t ncomp;      /* components of the residual graph */
  int32_t reduced;    /* components left after removing the s and t closures */
  int32_t reduced_arcs;
  int32_t best_rep;   /* sweep and position of the chosen cut (-1: none) */
  int32_t best_pos;
  int64_t best_bal;   /* max(source side weight, sink side weight) of the chosen cut */
} or_mbinfo;

/* Most balanced minimum cut on a network that holds a maximum s-t flow.
 * Node weights w (s and t included), key identifiers gid, fixed weights base_s
 * and base_t of the two sides outside the network; the balance of a source
 * side C is max(base_s + w(C), base_t + w(V \ C)), smaller is better.
 * Writes src[v] = 1 for the source side of the chosen cut and, if not NULL,
 * cls[v] = 0 (with s), 1 (remaining), 2 (with t) and comp[v].  Returns 0, or
 * -1 when out of memory. */
static int32_t net_mb_cut(const or_net *N, int32_t s, int32_t t, const int64_t *w,
                          const int32_t *gid, int64_t base_s, int64_t base_t, int32_t reps,
                          uint64_t seed, uint8_t *src, int8_t *cls_out, int32_t *comp_out,
                          or_mbinfo *info) {
  int32_t nn = N->nn;
  memset(info, 0, sizeof(*info));
  info->best_rep = info->best_pos = -1;
  int32_t *comp = (int32_t *)malloc(sizeof(int32_t) * (size_t)nn);
  if (!comp) return -1;
  int32_t nc = net_scc(N, comp);
  if (nc < 0) { free(comp); return -1; }
  info->ncomp = nc;
  /* the contracted graph: one arc per residual arc between two components,
   * as forward and backward adjacency lists */
  int64_t na = 0;
  for (int64_t a = 0; a < N->na; a++)
    if (N->res[a] > 0 && comp[N->tail[a]] != comp[N->head[a]]) na++;
  int64_t *fo = (int64_t *)calloc((size_t)nc + 1, sizeof(int64_t));
  int64_t *bo = (int64_t *)calloc((size_t)nc + 1, sizeof(int64_t));
  int32_t *fa = (int32_t *)malloc(sizeof(int32_t) * (size_t)(na ? na : 1));
  int32_t *ba = (int32_t *)malloc(sizeof(int32_t) * (size_t)(na ? na : 1));
  int8_t *cl = (int8_t *)malloc((size_t)nc);
  int32_t *q = (int32_t *)malloc(sizeof(int32_t) * (size_t)nc);
  int64_t *wc = (int64_t *)calloc((size_t)nc, sizeof(int64_t));
  int32_t *kid = (int32_t *)malloc(sizeof(int32_t) * (size_t)nc);
  int32_t *indeg = (int32_t *)malloc(sizeof(int32_t) * (size_t)nc);
  uint8_t *placed = (uint8_t *)malloc((size_t)nc);
  int rc = 0;
  if (!fo || !bo || !fa || !ba || !cl || !q || !wc || !kid || !indeg || !placed) { rc = -1; goto done; }
  for (int64_t a = 0; a < N->na; a++) {
    int32_t x = comp[N->tail[a]], y = comp[N->head[a]];
    if (N->res[a] > 0 && x != y) { fo[x + 1]++; bo[y + 1]++; }
  }
  for (int32_t c = 0; c < nc; c++) { fo[c + 1] += fo[c]; bo[c + 1] += bo[c]; }
  {
    int64_t *fp = (int64_t *)malloc(sizeof(int64_t) * (size_t)nc);
    int64_t *bp = (int64_t *)malloc(sizeof(int64_t) * (size_t)nc);
    if (!fp || !bp) { free(fp); free(bp); rc = -1; goto done; }
    memcpy(fp, fo, sizeof(int64_t) * (size_t)nc);
    memcpy(bp, bo, sizeof(int64_t) * (size_t)nc);
    for (int64_t a = 0; a < N->na; a++) {
      int32_t x = comp[N->tail[a]], y = comp[N->head[a]];
      if (N->res[a] > 0 && x != y) { fa[fp[x]++] = y; ba[bp[y]++] = x; }
    }
    free(fp); free(bp);
  }
  /* remove the sink's component with all its predecessors (class 2) and the
   * source's component with all its successors (class 0), by BFS */
  for (int32_t c = 0; c < nc; c++) cl[c] = 1;
  {
    int32_t qh = 0, qt = 0;
    cl[comp[t]] = 2;
    q[qt++] = comp[t];
    while (qh < qt) {
      int32_t c = q[qh++];
      for (int64_t j = bo[c]; j < bo[c + 1]; j++)
        if (cl[ba[j]] != 2) { cl[ba[j]] = 2; q[qt++] = ba[j]; }
    }
    qh = qt = 0;
    if (cl[comp[s]] == 2) { rc = -1; goto done; } /* s reaches t: the flow is not maximal */
    cl[comp[s]] = 0;
    q[qt++] = comp[s];
    while (qh < qt) {
      int32_t c = q[qh++];
      for (int64_t j = fo[c]; j < fo[c + 1]; j++) {
        if (cl[fa[j]] == 2) { rc = -1; goto done; }
        if (cl[fa[j]] != 0) { cl[fa[j]] = 0; q[qt++] = fa[j]; }
      }
    }
  }
  /* weights and key identifiers of the remaining components; the two fixed sides */
  int64_t w_src = base_s, w_snk = base_t;
  for (int32_t c = 0; c < nc; c++) kid[c] = INT32_MAX;
  for (int32_t v = 0; v < nn; v++) {
    int32_t c = comp[v];
    if (cl[c] == 2) w_snk += w[v];
    else w_src += w[v];  /* the sweeps start with every remaining component on the source side */
    if (cl[c] == 1) {
      wc[c] += w[v];
      if (gid[v] < kid[c]) kid[c] = gid[v];
    }
  }
  int32_t nrem = 0;
  for (int32_t c = 0; c < nc; c++) nrem += cl[c] == 1;
  info->reduced = nrem;
  for (int32_t c = 0; c < nc; c++)
    if (cl[c] == 1)
      for (int64_t j = fo[c]; j < fo[c + 1]; j++) info->reduced_arcs += cl[fa[j]] == 1;
  int32_t best_r = -1, best_j = 0;
  int64_t best = 0;
  if (nrem > 0 && reps > 0) {
    /* sweeps: a random topological order of the remaining components moves
     * them one by one to the sink side; the first most balanced cut wins */
    for (int32_t r = 0; r < reps; r++) {
      for (int32_t c = 0; c < nc; c++) {
        indeg[c] = 0;
        placed[c] = 0;
      }
      for (int32_t c = 0; c < nc; c++)
        if (cl[c] == 1)
          for (int64_t j = fo[c]; j < fo[c + 1]; j++)
            if (cl[fa[j]] == 1) indeg[fa[j]]++;
      int64_t ws = w_src, wt = w_snk;
      for (int32_t j = 0; j <= nrem; j++) {
        if (j > 0) {
          int32_t pick = -1;
          uint64_t kp = 0;
          for (int32_t c = 0; c < nc; c++) {
            if (cl[c] != 1 || placed[c] || indeg[c] != 0) continue;
            uint64_t kc = mb_key(seed, r, kid[c]);
            if (pick < 0 || kc < kp) { pick = c; kp = kc; }
          }
          if (pick < 0) { rc = -1; goto done; } /* a cycle: cannot happen after contraction */
          placed[pick] = 1;
          ws -= wc[pick];
          wt += wc[pick];
          for (int64_t e = fo[pick]; e < fo[pick + 1]; e++)
            if (cl[fa[e]] == 1) indeg[fa[e]]--;
        }
        int64_t bal = ws > wt ? ws : wt;
        if (best_r < 0 || bal < best) { best = bal; best_r = r; best_j = j; }
      }
    }
    /* the chosen cut: the first best_j components of sweep best_r's order */
    for (int32_t c = 0; c < nc; c++) { indeg[c] = 0; placed[c] = 0; }
    for (int32_t c = 0; c < nc; c++)
      if (cl[c] == 1)
        for (int64_t j = fo[c]; j < fo[c + 1]; j++)
          if (cl[fa[j]] == 1) indeg[fa[j]]++;
    for (int32_t j = 0; j < best_j; j++) {
      int32_t pick = -1;
      uint64_t kp = 0;
      for (int32_t c = 0; c < nc; c++) {
        if (cl[c] != 1 || placed[c] || indeg[c] != 0) continue;
        uint64_t kc = mb_key(seed, best_r, kid[c]);
        if (pick < 0 || kc < kp) { pick = c; kp = kc; }
      }
      placed[pick] = 1;
      for (int64_t e = fo[pick]; e < fo[pick + 1]; e++)
        if (cl[fa[e]] == 1) indeg[fa[e]]--;
    }
    info->best_rep = best_r;
    info->best_pos = best_j;
    info->best_bal = best;
    for (int32_t v = 0; v < nn; v++) {
      int32_t c = comp[v];
      src[v] = (uint8_t)(cl[c] == 0 || (cl[c] == 1 && !placed[c]));
    }
  } else {
    for (int32_t v = 0; v < nn; v++) src[v] = (uint8_t)(cl[comp[v]] == 0);
  }
  if (cls_out) for (int32_t v = 0; v < nn; v++) cls_out[v] = cl[comp[v]];
  if (comp_out) memcpy(comp_out, comp, sizeof(int32_t) * (size_t)nn);
done:
  free(comp); free(fo); free(bo); free(fa); free(ba); free(cl); free(q); free(wc); free(kid);
  free(indeg); free(placed);
  return rc;
}

/* Strongly connected components of a plain directed graph (tails -> heads).
 * comp: [nn].  Returns the number of components, or -1 on bad input. */
int32_t or_scc(int32_t nn, int64_t narcs, const int32_t *tails, const int32_t *heads,
               int32_t *comp) {
  if (nn <= 0) return -1;
  or_net N;
  if (net_init(&N, nn, 2 * narcs) != 0) { net_free(&N); return -1; }
  for (int64_t i = 0; i < narcs; i++) {
    if (tails[i] < 0 || tails[i] >= nn || heads[i] < 0 || heads[i] >= nn) { net_free(&N); return -1; }
    net_add(&N, tails[i], heads[i], 1, 0);
  }
  if (net_finish(&N) != 0) { net_free(&N); return -1; }
  int32_t nc = net_scc(&N, comp);
  net_free(&N);
  return nc;
}

/* Max flow, then the most balanced minimum cut, on an explicit network (arcs
 * with zero-capacity reverses).  w, gid: [nn] node weights and key ids.
 * Outputs (each [nn]): src (chosen source side), smin (smallest source set),
 * cls, comp; info[6] = ncomp, reduced, reduced_arcs, best_rep, best_pos,
 * best_bal.  Returns 0, or -1 on bad input. */
int32_t or_mbcut(int32_t nn, int64_t narcs, const int32_t *tails, const int32_t *heads,
                 const int64_t *caps, int32_t s, int32_t t, const int64_t *w, const int32_t *gid,
                 int64_t base_s, int64_t base_t, int32_t reps, uint32_t seed, int64_t *flow_out,
                 uint8_t *src, uint8_t *smin, int8_t *cls, int32_t *comp, int64_t *info) {
  if (nn <= 0 || s < 0 || s >= nn || t < 0 || t >= nn || s == t || reps < 0) return -1;
  or_net N;
  if (net_init(&N, nn, 2 * narcs) != 0) { net_free(&N); return -1; }
  for (int64_t i = 0; i < narcs; i++) {
    if (tails[i] < 0 || tails[i] >= nn || heads[i] < 0 || heads[i] >= nn || caps[i] < 0) {
      net_free(&N);
      return -1;
    }
    net_add(&N, tails[i], heads[i], caps[i], 0);
  }
  if (net_finish(&N) != 0) { net_free(&N); return -1; }
  *flow_out = net_dinic(&N, s, t);
  int32_t *qq = (int32_t *)malloc(sizeof(int32_t) * (size_t)nn);
  if (!qq) { net_free(&N); return -1; }
  net_reach(&N, s, smin, qq);
  free(qq);
  or_mbinfo mi;
  int32_t rc = net_mb_cut(&N, s, t, w, gid, base_s, base_t, reps, (uint64_t)seed, src, cls,
                          comp, &mi);
  info[0] = mi.ncomp; info[1] = mi.reduced; info[2] = mi.reduced_arcs;
  info[3] = mi.best_rep; info[4] = mi.best_pos; info[5] = mi.best_bal;
  net_free(&N);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* pair refinement                                                           */

static int cmp_i32(const void *x, const void *y) {
  int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
  return (a > b) - (a < b);
}

/* pair cut omega(E_ab), each undirected edge counted once */
static int64_t pair_cut(const or_graph *g, const int32_t *part, int32_t a, int32_t b) {
  int64_t c = 0;
  for (int32_t u = 0; u < g->n; u++) {
    if (part[u] != a) continue;
    for (int32_t e = g->xadj[u]; e < g->xadj[u + 1]; e++)
      if (part[g->adjncy[e]] == b) c += g->adjwgt[e];
  }
  return c;
}

/* One bounded BFS (Sec. 4.1): seeds = boundary of block `blk` towards
 * `other`, expanded only inside `blk`.  Vertices are taken level by level,
 * each level in ascending id, while the running weight stays <= bound
 * (FACTOR mode); the walk stops for good at the first vertex that would
 * exceed it.  DEPTH mode takes every vertex at distance <= depth.
 * Marks inB[v] = tag for every taken vertex. */
static void area_bfs(const or_graph *g, const int32_t *part, int32_t blk, int32_t other,
                     int32_t mode, int32_t depth, int64_t bound, uint8_t *inB, uint8_t tag,
                     uint8_t *seen, int32_t *cur, int32_t *next) {
  int32_t ncur = 0;
  for (int32_t u = 0; u < g->n; u++) {
    if (part[u] != blk) continue;
    for (int32_t e = g->xadj[u]; e < g->xadj[u + 1]; e++)
      if (part[g->adjncy[e]] == other) { cur[ncur++] = u; break; }
  }
  for (int32_t i = 0; i < ncur; i++) seen[cur[i]] = 1;
  int64_t weight = 0;
  int32_t lev = 0;
  while (ncur > 0) {
    qsort(cur, (size_t)ncur, sizeof(int32_t), cmp_i32);
    if (mode == 1) {
      if (lev > depth) return;
      for (int32_t i = 0; i < ncur; i++) inB[cur[i]] = tag;
    } else {
      for (int32_t i = 0; i < ncur; i++) {
        int32_t v = cur[i];
        if (weight + g->vwgt[v] > bound) return; /* stop the whole search */
        weight += g->vwgt[v];
        inB[v] = tag;
      }
    }
    int32_t nnext = 0;
    for (int32_t i = 0; i < ncur; i++) {
      int32_t u = cur[i];
      for (int32_t e = g->xadj[u]; e < g->xadj[u + 1]; e++) {
        int32_t v = g->adjncy[e];
        if (part[v] == blk && !seen[v]) { seen[v] = 1; next[nnext++] = v; }
      }
    }
    int32_t *t = cur; cur = next; next = t;
    ncur = nnext;
    lev++;
  }
}

/* One flow solve for the pair (a = source side, b = sink side) at factor
 * alpha.  Fills rec; if apply is set and the candidate is accepted, writes it
 * into part.  side_out (optional, length n): -1 outside the corridor, 0/1
 * corridor vertex ending in a / b, 2/3 border vertex pinned to s / t (only
 * with pinned terminals). */
static int32_t solve_once(const or_graph *g, int32_t *part, int32_t k, int32_t a, int32_t b,
                          const or_params *p, int32_t alpha, or_solve *rec, int8_t *side_out) {
  int32_t n = g->n;
  memset(rec, 0, sizeof(*rec));
  rec->alpha = alpha;
  /* Sec. 2.1: c(V), max c(v), block weights, L_max = (1+eps) c(V)/k + max c */
  int64_t cV = 0, maxc = 0, cA = 0, cB = 0;
  for (int32_t u = 0; u < n; u++) {
    cV += g->vwgt[u];
    if (g->vwgt[u] > maxc) maxc = g->vwgt[u];
    if (part[u] == a) cA += g->vwgt[u];
    if (part[u] == b) cB += g->vwgt[u];
  }
  int64_t lmax = (int64_t)(((__int128)(1000000 + (int64_t)p->eps_ppm) * cV) /
                           ((__int128)1000000 * k)) + maxc;
  int64_t cut = pair_cut(g, part, a, b);
  rec->cut_before = cut;
  if (side_out) for (int32_t u = 0; u < n; u++) side_out[u] = -1;
  if (cut == 0) {
    rec->decision = DEC_NOT_ADJ;
    rec->cut_candidate = cut;
    rec->wa = cA;
    rec->wb = cB;
    return 0;
  }
  /* R4: U_x(alpha) = floor((1 + alpha eps) c(V) / k) - c(other block) */
  int64_t base = (int64_t)(((__int128)(1000000 + (int64_t)alpha * p->eps_ppm) * cV) /
                           ((__int128)1000000 * k));
  int64_t UA = base - cB, UB = base - cA;
  if (UA < 0) UA = 0;
  if (UB < 0) UB = 0;

  uint8_t *inB = (uint8_t *)calloc((size_t)n, 1);
  uint8_t *seen = (uint8_t *)calloc((size_t)n, 1);
  int32_t *q1 = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t *q2 = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t *loc = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  if (!inB || !seen || !q1 || !q2 || !loc) { free(inB); free(seen); free(q1); free(q2); free(loc); return -1; }
  area_bfs(g, part, a, b, p->area_mode, p->depth, UA, inB, 1, seen, q1, q2);
  area_bfs(g, part, b, a, p->area_mode, p->depth, UB, inB, 2, seen, q1, q2);

  /* corridor vertices in ascending id -> local ids; s = nb, t = nb + 1 */
  int32_t nb = 0;
  for (int32_t u = 0; u < n; u++) loc[u] = inB[u] ? nb++ : -1;
  int32_t S = nb, T = nb + 1;
  /* R2: border within G[A u B]: a corridor vertex with a neighbour in A u B
   * outside the corridor.  cin: the old a-b edges whose cut state the solve
   * decides (both ends in the corridor; with contracted terminals also those
   * with one end outside).  R30: cs / ct = weight from a corridor vertex into
   * a / b outside the corridor. */
  uint8_t *border = (uint8_t *)calloc((size_t)(nb ? nb : 1), 1);
  int64_t *cs = (int64_t *)calloc((size_t)(nb ? nb : 1), sizeof(int64_t));
  int64_t *ct = (int64_t *)calloc((size_t)(nb ? nb : 1), sizeof(int64_t));
  if (!border || !cs || !ct) { free(cs); free(ct); goto oom; }
  int64_t nedges = 0, sumw = 0, cin = 0;
  for (int32_t u = 0; u < n; u++) {
    if (!inB[u]) continue;
    for (int32_t e = g->xadj[u]; e < g->xadj[u + 1]; e++) {
      int32_t v = g->adjncy[e];
      if (inB[v]) {
        if (u < v) {
          nedges++;
          sumw += g->adjwgt[e];
          if (inB[u] != inB[v]) cin += g->adjwgt[e];
        }
      } else if (part[v] == a || part[v] == b) {
        border[loc[u]] = 1;
        if (part[v] == a) cs[loc[u]] += g->adjwgt[e];
        else ct[loc[u]] += g->adjwgt[e];
        if (p->terminals && part[v] != part[u]) cin += g->adjwgt[e];
      }
    }
  }
  if (p->terminals) memset(border, 0, (size_t)(nb ? nb : 1)); /* nothing is pinned */
  rec->region_vertices = nb;
  rec->region_edges = nedges;
  int64_t INF = 2 * sumw + 1; /* exceeds every finite cut */
  or_net N;
  /* two arcs per corridor edge, and an s or t arc with its reverse at most twice per vertex */
  if (net_init(&N, nb + 2, 2 * nedges + 4 * (int64_t)nb) != 0) { free(cs); free(ct); goto oom; }
  for (int32_t u = 0; u < n; u++) {
    if (!inB[u]) continue;
    for (int32_t e = g->xadj[u]; e < g->xadj[u + 1]; e++) {
      int32_t v = g->adjncy[e];
      if (inB[v] && u < v) net_add(&N, loc[u], loc[v], g->adjwgt[e], g->adjwgt[e]);
    }
    if (p->terminals) {
      /* R30: arcs from the contracted outside of a, into that of b */
      if (cs[loc[u]] > 0) net_add(&N, S, loc[u], cs[loc[u]], 0);
      if (ct[loc[u]] > 0) net_add(&N, loc[u], T, ct[loc[u]], 0);
    } else if (border[loc[u]]) {
      if (inB[u] == 1) net_add(&N, S, loc[u], INF, 0); /* s -> left border */
      else net_add(&N, loc[u], T, INF, 0);             /* right border -> t */
    }
  }
  free(cs);
  free(ct);
  if (net_finish(&N) != 0) { net_free(&N); goto oom; }
  int64_t flow = net_dinic(&N, S, T);
  rec->flow = flow;
  uint8_t *reach = (uint8_t *)malloc((size_t)nb + 2);
  int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * ((size_t)nb + 2));
  if (!reach || !queue) { free(reach); free(queue); net_free(&N); goto oom; }
  net_reach(&N, S, reach, queue);
  if (p->mb_reps > 0) {
    /* Sec. 4.1.1: the most balanced minimum cut replaces the smallest source
     * set; the blocks keep their vertices outside the corridor */
    int64_t *w = (int64_t *)calloc((size_t)nb + 2, sizeof(int64_t));
    int32_t *gid = (int32_t *)malloc(sizeof(int32_t) * ((size_t)nb + 2));
    if (!w || !gid) { free(w); free(gid); free(reach); free(queue); net_free(&N); goto oom; }
    int64_t base_s = cA, base_t = cB;
    for (int32_t u = 0; u < n; u++) {
      if (!inB[u]) continue;
      w[loc[u]] = g->vwgt[u];
      gid[loc[u]] = u;
      if (inB[u] == 1) base_s -= g->vwgt[u];
      else base_t -= g->vwgt[u];
    }
    gid[S] = gid[T] = INT32_MAX;
    or_mbinfo mi;
    int32_t mrc = net_mb_cut(&N, S, T, w, gid, base_s, base_t, p->mb_reps,
                             (uint64_t)(uint32_t)p->mb_seed, reach, NULL, NULL, &mi);
    free(w);
    free(gid);
    if (mrc != 0) { free(reach); free(queue); net_free(&N); goto oom; }
  } else if (p->cut_side != 0) {
    /* the largest minimum source side: every node that cannot reach t
     * (Sec. 4.1.1: the closed sets between the two closures are the minimum
     * cuts); cut_side 2 takes it only when the smallest source set is
     * infeasible and it is feasible */
    uint8_t *tr = (uint8_t *)malloc((size_t)nb + 2);
    if (!tr) { free(reach); free(queue); net_free(&N); goto oom; }
    net_reach_to(&N, T, tr, queue);
    int64_t wa1 = cA, wb1 = cB, wa2 = cA, wb2 = cB;
    for (int32_t u = 0; u < n; u++) {
      if (!inB[u]) continue;
      int in1 = reach[loc[u]], in2 = !tr[loc[u]];
      if (inB[u] == 1 && !in1) { wa1 -= g->vwgt[u]; wb1 += g->vwgt[u]; }
      if (inB[u] == 2 && in1) { wb1 -= g->vwgt[u]; wa1 += g->vwgt[u]; }
      if (inB[u] == 1 && !in2) { wa2 -= g->vwgt[u]; wb2 += g->vwgt[u]; }
      if (inB[u] == 2 && in2) { wb2 -= g->vwgt[u]; wa2 += g->vwgt[u]; }
    }
    int take = p->cut_side == 1 ||
               (!(wa1 <= lmax && wb1 <= lmax) && (wa2 <= lmax && wb2 <= lmax));
    if (take)
      for (int32_t v = 0; v < nb + 2; v++) reach[v] = (uint8_t)!tr[v];
    free(tr);
  }

  /* candidate: corridor vertex -> a iff on the source side of the cut */
  int64_t wa = cA, wb = cB, src = 0;
  for (int32_t u = 0; u < n; u++) {
    if (!inB[u]) continue;
    int in_s = reach[loc[u]];
    src += in_s;
    if (inB[u] == 1 && !in_s) { wa -= g->vwgt[u]; wb += g->vwgt[u]; }
    if (inB[u] == 2 && in_s) { wb -= g->vwgt[u]; wa += g->vwgt[u]; }
    if (side_out) side_out[u] = (int8_t)((border[loc[u]] ? 2 : 0) + (in_s ? 0 : 1));
  }
  rec->source_side = src;
  rec->wa = wa;
  rec->wb = wb;
  /* the decided edges: C_in before, flow after */
  int64_t cand = cut - cin + flow;
  rec->cut_candidate = cand;
  int feasible = wa <= lmax && wb <= lmax;
  if (!feasible) rec->decision = DEC_INFEASIBLE;
  else if (cand < cut) rec->decision = DEC_APPLY;
  else rec->decision = DEC_EQUAL;
  if (rec->decision == DEC_APPLY) {
    for (int32_t u = 0; u < n; u++)
      if (inB[u]) part[u] = reach[loc[u]] ? a : b;
  }
  free(reach);
  free(queue);
  net_free(&N);
  free(border); free(inB); free(seen); free(q1); free(q2); free(loc);
  return 0;
oom:
  free(border); free(inB); free(seen); free(q1); free(q2); free(loc);
  return -1;
}

/* ------------------------------------------------------------------------ */
/* 2-way FM local search with TopGain (Sec. 2.2)                             */

/* FM key of vertex v: output number v + 1 of SplitMix64 started at the seed;
 * the tie bit of move step t: bit 0 of output number 2^32 + t + 1 */
static uint64_t fm_key(uint64_t seed, int32_t v) { return splitmix64_out(seed, (uint64_t)(uint32_t)v + 1); }
static int fm_bit(uint64_t seed, int64_t t) {
  return (int)(splitmix64_out(seed, (1ull << 32) + (uint64_t)t + 1) & 1ull);
}

typedef struct {
  int64_t cut0, cut;   /* pair cut before and after */
  int64_t steps;       /* moves made */
  int64_t kept;        /* moves kept after the rollback */
  int64_t wa, wb;      /* block weights after */
} or_fminfo;

/* one pass of 2-way FM on blocks a, b of part (in place).  lmax: the balance
 * bound.  Returns 0 or -1 (out of memory).  move_log (optional, n): the
 * vertices in move order, info->steps of them. */
static int32_t pair_fm(const or_graph *g, int32_t *part, int32_t a, int32_t b, int64_t lmax,
                       int32_t limit, uint64_t seed, or_fminfo *info, int32_t *move_log) {
  int32_t n = g->n;
  int64_t *gain = (int64_t *)calloc((size_t)n, sizeof(int64_t));
  int8_t *st = (int8_t *)calloc((size_t)n, 1); /* 0 out, 1 queued, 2 moved */
  int32_t *log = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
  int32_t *qa = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
  if (!gain || !st || !log || !qa) { free(gain); free(st); free(log); free(qa); return -1; }
  memset(info, 0, sizeof(*info));
  int64_t wa = 0, wb = 0, cut = 0;
  /* gains: weight to the other block of the pair minus weight to the own */
  for (int32_t v = 0; v < n; v++) {
    if (part[v] != a && part[v] != b) continue;
    int32_t other = part[v] == a ? b : a;
    int64_t ext = 0, in = 0;
    for (int32_t e = g->xadj[v]; e < g->xadj[v + 1]; e++) {
      int32_t u = g->adjncy[e];
      if (part[u] == other) ext += g->adjwgt[e];
      else if (part[u] == part[v]) in += g->adjwgt[e];
    }
    gain[v] = ext - in;
    if (ext > 0) st[v] = 1; /* boundary vertex: queued */
    if (part[v] == a) { wa += g->vwgt[v]; cut += ext; }
    else wb += g->vwgt[v];
  }
  int32_t nq = 0; /* the queued vertices, scanned for the top of each block */
  for (int32_t v = 0; v < n; v++) if (st[v] == 1) qa[nq++] = v;
  info->cut0 = cut;
  /* quality of a state: (infeasible, feasible ? cut : max(wa, wb)) */
  int best_inf = !(wa <= lmax && wb <= lmax);
  int64_t best_val = best_inf ? (wa > wb ? wa : wb) : cut;
  int64_t best_step = 0, steps = 0, since = 0;
  for (;;) {
    if (since >= limit) break;
    /* tops of the two queues: largest gain, then largest key */
    int32_t top[2] = {-1, -1};
    uint64_t tk[2] = {0, 0};
    for (int32_t i = 0; i < nq; i++) {
      int32_t v = qa[i];
      if (st[v] != 1) continue;
      int side = part[v] == a ? 0 : 1;
      uint64_t kv = fm_key(seed, v);
      int32_t t = top[side];
      if (t < 0 || gain[v] > gain[t] || (gain[v] == gain[t] && kv > tk[side])) {
        top[side] = v;
        tk[side] = kv;
      }
    }
    if (top[0] < 0 && top[1] < 0) break;
    int side;
    if ((wa > lmax || wb > lmax) && wa != wb) side = wa > wb ? 0 : 1;  /* move out of the heavier */
    else if (top[0] < 0 || top[1] < 0) side = top[0] < 0 ? 1 : 0;
    else if (gain[top[0]] != gain[top[1]]) side = gain[top[0]] > gain[top[1]] ? 0 : 1;
    else side = fm_bit(seed, steps);
    if (top[side] < 0) side = 1 - side;
    int32_t v = top[side];
    int32_t from = part[v], to = from == a ? b : a;
    /* move */
    part[v] = to;
    st[v] = 2;
    cut -= gain[v];
    if (from == a) { wa -= g->vwgt[v]; wb += g->vwgt[v]; }
    else { wb -= g->vwgt[v]; wa += g->vwgt[v]; }
    log[steps++] = v;
    for (int32_t e = g->xadj[v]; e < g->xadj[v + 1]; e++) {
      int32_t u = g->adjncy[e];
      if ((part[u] != a && part[u] != b) || st[u] == 2) continue;
      /* the edge turns from internal to cut for u in `from`, and back for u in `to` */
      gain[u] += part[u] == from ? 2 * (int64_t)g->adjwgt[e] : -2 * (int64_t)g->adjwgt[e];
      if (st[u] == 0) { st[u] = 1; qa[nq++] = u; }
    }
    int inf = !(wa <= lmax && wb <= lmax);
    int64_t val = inf ? (wa > wb ? wa : wb) : cut;
    if (inf < best_inf || (inf == best_inf && val < best_val)) {
      best_inf = inf;
      best_val = val;
      best_step = steps;
      since = 0;
    } else {
      since++;
    }
  }
  /* roll back the moves after the best state */
  for (int64_t i = steps - 1; i >= best_step; i--) {
    int32_t v = log[i];
    int32_t to = part[v], from = to == a ? b : a;
    part[v] = from;
    if (from == a) { wa += g->vwgt[v]; wb -= g->vwgt[v]; }
    else { wb += g->vwgt[v]; wa -= g->vwgt[v]; }
  }
  info->steps = steps;
  info->kept = best_step;
  info->wa = wa;
  info->wb = wb;
  info->cut = pair_cut(g, part, a, b);
  if (move_log) memcpy(move_log, log, sizeof(int32_t) * (size_t)steps);
  free(gain); free(st); free(log); free(qa);
  return 0;
}

/* 2-way FM on one pair alone (for tests).  info[6] = cut before, cut after,
 * moves made, moves kept, weight a, weight b; move_log (optional, n). */
int32_t or_pair_fm(const or_graph *g, int32_t *part, int32_t k, int32_t a, int32_t b,
                   int32_t eps_ppm, int32_t limit, uint32_t seed, int64_t *info,
                   int32_t *move_log) {
  if (a < 0 || b < 0 || a >= k || b >= k || a == b || limit < 0) return -3;
  int64_t cV = 0, maxc = 0;
  for (int32_t u = 0; u < g->n; u++) {
    cV += g->vwgt[u];
    if (g->vwgt[u] > maxc) maxc = g->vwgt[u];
  }
  int64_t lmax = (int64_t)(((__int128)(1000000 + (int64_t)eps_ppm) * cV) /
                           ((__int128)1000000 * k)) + maxc;
  or_fminfo fi;
  if (pair_fm(g, part, a, b, lmax, limit, (uint64_t)seed, &fi, move_log) != 0) return -7;
  info[0] = fi.cut0; info[1] = fi.cut; info[2] = fi.steps; info[3] = fi.kept;
  info[4] = fi.wa; info[5] = fi.wb;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* multi-try FM (Sec. 4.2): rounds of localized k-way searches               */

/* Keys of the multi-try searches, SplitMix64 outputs from the seed:
 *   todo order of vertex v       output number 2^40 + v + 1
 *   queue order of vertex v      output number 2^41 + v + 1
 *   tie key of target block P    output number 2^42 + v * k + P + 1        */
static uint64_t mt_key(uint64_t seed, int which, uint64_t x) {
  return splitmix64_out(seed, (1ull << (40 + which)) + x + 1);
}

static int cmp_u64(const void *x, const void *y) {
  uint64_t a = *(const uint64_t *)x, b = *(const uint64_t *)y;
  return (a > b) - (a < b);
}

/* The k-way gain of v (Sec. 2.2, k-way local search): over the blocks P other
 * than v's own that hold a neighbour of v, the largest omega(v, P) minus
 * omega(v, own block); the block reaching it is the target, equal gains going
 * to the smaller tie key.  Returns the target, or -1 when every neighbour is
 * in v's block (v is not a boundary vertex).  wsum: [k], zero on entry and
 * on return. */
static int32_t mt_gain(const or_graph *g, const int32_t *part, int32_t k, uint64_t seed,
                       int32_t v, int64_t *wsum, int64_t *gain_out) {
  int32_t own = part[v];
  for (int32_t e = g->xadj[v]; e < g->xadj[v + 1]; e++) wsum[part[g->adjncy[e]]] += g->adjwgt[e];
  int32_t best = -1;
  int64_t bg = 0;
  uint64_t bk = 0;
  for (int32_t e = g->xadj[v]; e < g->xadj[v + 1]; e++) {
    int32_t P = part[g->adjncy[e]];
    if (P == own) continue;
    int64_t gP = wsum[P] - wsum[own];
    uint64_t kP = mt_key(seed, 2, (uint64_t)v * (uint64_t)k + (uint64_t)P);
    if (best < 0 || gP > bg || (gP == bg && kP < bk)) { best = P; bg = gP; bk = kP; }
  }
  for (int32_t e = g->xadj[v]; e < g->xadj[v + 1]; e++) wsum[part[g->adjncy[e]]] = 0;
  *gain_out = bg;
  return best;
}

/* KaSPar's stopping rule (Sec. 2.2): with p moves since the last best state
 * and S1, S2 the sum and the sum of squares of their gains, mean mu = S1/p and
 * variance sigma^2 = S2/p - mu^2; stop when p mu^2 > alpha sigma^2 + beta,
 * beta = ln n.  Multiplied by p^2 and with beta as the fixed-point
 * beta_fx = floor(ln n * 2^16):  2^16 (p S1^2 - alpha (p S2 - S1^2)) > beta_fx p^2. */
static int mt_stop(int64_t p, __int128 S1, __int128 S2, int32_t alpha, int64_t beta_fx) {
  __int128 lhs = ((__int128)p * S1 * S1 - (__int128)alpha * ((__int128)p * S2 - S1 * S1)) * 65536;
  return lhs > (__int128)beta_fx * p * p;
}

typedef struct {
  const or_graph *g;
  int32_t *part;
  int32_t k;
  uint64_t seed;
  int64_t lmax, beta_fx, over; /* over: blocks heavier than lmax */
  int32_t alpha;
  int64_t *bw;                 /* [k] block weights */
  int64_t *wsum;               /* [k] scratch of mt_gain */
  int32_t *touched;            /* [n] number of the round that last touched the vertex */
  uint8_t *inq;                /* [n] queued in the current search */
  int64_t *gain;               /* [n] gain and target of queued vertices */
  int32_t *tgt;
  int32_t *q;                  /* [n] queued vertices (with popped ones) */
  int32_t *mv, *mfrom;         /* [n] moves of the current search */
  int64_t *ev;                 /* optional event log */
  int64_t nev, evcap;
} mt_ctx;

static void mt_event(mt_ctx *C, int64_t a, int64_t b, int64_t c, int64_t d, int64_t e) {
  if (C->ev && C->nev + 5 <= C->evcap) {
    int64_t *x = C->ev + C->nev;
    x[0] = a; x[1] = b; x[2] = c; x[3] = d; x[4] = e;
  }
  C->nev += 5;
}

/* Queues y when it is a boundary vertex; a queued vertex counts as touched by
 * this round from then on. */
static int32_t mt_insert(mt_ctx *C, int32_t y, int32_t round, int32_t *nq) {
  int32_t t = mt_gain(C->g, C->part, C->k, C->seed, y, C->wsum, &C->gain[y]);
  if (t < 0) return 0;
  C->touched[y] = round;
  C->tgt[y] = t;
  C->inq[y] = 1;
  C->q[(*nq)++] = y;
  return 1;
}

/* One multi-try round (Sec. 4.2) over a todo list in its order: each entry
 * that is still a boundary vertex and was not touched by an earlier search of
 * this round starts a k-way search from itself and its untouched boundary
 * neighbours.  A search repeatedly takes the queued vertex with the largest
 * gain (equal gains: the larger queue key), moves it to its target block
 * unless that block would exceed lmax, and queues the untouched boundary
 * neighbours of a moved vertex (recomputing the gains of queued ones; a queued
 * vertex left without a target leaves the queue); it ends when the queue is
 * empty or the stopping rule fires, and rolls back to its best state: fewest
 * blocks above lmax, then lowest cut, earliest on ties.  Vertices touched by a
 * search (queued or moved) are not queued again in this round.  chg (optional,
 * [k]): the blocks a kept move left or entered get 1. */
static void mt_round(mt_ctx *C, const int32_t *todo, int32_t ntodo, int32_t round,
                     int64_t *searches, int64_t *moves, int64_t *kept, uint8_t *chg) {
  const or_graph *g = C->g;
  int32_t *part = C->part;
  for (int32_t i = 0; i < ntodo; i++) {
    int32_t v = todo[i];
    if (C->touched[v] == round) continue;
    int64_t gv;
    if (mt_gain(g, part, C->k, C->seed, v, C->wsum, &gv) < 0) continue; /* no longer boundary */
    /* the search's start set: v and its untouched boundary neighbours */
    int32_t nq = 0;
    mt_insert(C, v, round, &nq);
    for (int32_t e = g->xadj[v]; e < g->xadj[v + 1]; e++) {
      int32_t y = g->adjncy[e];
      if (C->touched[y] != round) mt_insert(C, y, round, &nq);
    }
    (*searches)++;
    mt_event(C, 1, round, v, nq, 0);
    int64_t delta = 0, best = 0, best_over = C->over;
    int64_t nmv = 0, best_n = 0, pcount = 0;
    __int128 S1 = 0, S2 = 0;
    for (;;) {
      int32_t x = -1;
      uint64_t kx = 0;
      for (int32_t j = 0; j < nq; j++) {
        int32_t y = C->q[j];
        if (!C->inq[y]) continue;
        uint64_t ky = mt_key(C->seed, 1, (uint64_t)y);
        if (x < 0 || C->gain[y] > C->gain[x] || (C->gain[y] == C->gain[x] && ky > kx)) { x = y; kx = ky; }
      }
      if (x < 0) break;
      C->inq[x] = 0;
      int32_t to = C->tgt[x], from = part[x];
      int64_t gx = C->gain[x], cx = g->vwgt[x];
      if (C->bw[to] + cx > C->lmax) continue; /* the move would overload its target */
      if (C->bw[from] > C->lmax && C->bw[from] - cx <= C->lmax) C->over--;
      C->bw[from] -= cx;
      C->bw[to] += cx;
      part[x] = to;
      delta -= gx;
      C->mv[nmv] = x;
      C->mfrom[nmv] = from;
      nmv++;
      mt_event(C, 2, x, from, to, gx);
      if (C->over < best_over || (C->over == best_over && delta < best)) {
        best = delta;
        best_over = C->over;
        best_n = nmv;
        pcount = 0;
        S1 = S2 = 0;
      } else {
        pcount++;
        S1 += gx;
        S2 += (__int128)gx * gx;
        if (mt_stop(pcount, S1, S2, C->alpha, C->beta_fx)) break;
      }
      for (int32_t e = g->xadj[x]; e < g->xadj[x + 1]; e++) {
        int32_t y = g->adjncy[e];
        if (C->inq[y]) {
          int32_t t = mt_gain(g, part, C->k, C->seed, y, C->wsum, &C->gain[y]);
          if (t < 0) C->inq[y] = 0;
          else C->tgt[y] = t;
        } else if (C->touched[y] != round) {
          mt_insert(C, y, round, &nq);
        }
      }
    }
    for (int32_t j = 0; j < nq; j++) C->inq[C->q[j]] = 0;
    /* roll back the moves after the best state */
    for (int64_t j = nmv - 1; j >= best_n; j--) {
      int32_t x = C->mv[j], from = C->mfrom[j], to = part[x];
      int64_t cx = g->vwgt[x];
      C->bw[to] -= cx;
      if (C->bw[from] <= C->lmax && C->bw[from] + cx > C->lmax) C->over++;
      C->bw[from] += cx;
      part[x] = from;
    }
    if (chg)
      for (int64_t j = 0; j < best_n; j++) {
        chg[C->mfrom[j]] = 1;
        chg[part[C->mv[j]]] = 1;
      }
    mt_event(C, 3, nmv, best_n, 0, 0);
    *moves += nmv;
    *kept += best_n;
  }
}

/* The multi-try phase of a batch (after its pairwise improvements): the todo
 * list of each pair, formed from the partition at the start of the phase, is
 * every vertex of its two blocks with a neighbour in another block, ordered
 * by the upper 32 bits of its todo key, then by id; then one round per pair in
 * pair order.  kept: [npairs] moves kept per pair; chg (optional, [k]).
 * ev (optional): events of 5 int64: (1, round, start vertex, start set size,
 * 0) per search, (2, vertex, from, to, gain) per move, (3, moves, kept, 0, 0)
 * at the end of a search; *nev gets their count * 5 (even past evcap). */
static int32_t mt_phase(const or_graph *g, int32_t *part, int32_t k, const int32_t *pairs,
                        int32_t npairs, const or_params *p, int64_t *kept, int64_t *stats3,
                        uint8_t *chg, int64_t *ev, int64_t evcap, int64_t *nev) {
  int32_t n = g->n;
  mt_ctx C;
  memset(&C, 0, sizeof(C));
  C.g = g;
  C.part = part;
  C.k = k;
  C.seed = (uint64_t)(uint32_t)p->mt_seed;
  C.alpha = p->mt_alpha;
  C.beta_fx = (int64_t)floor(log((double)n) * 65536.0);
  C.bw = (int64_t *)calloc((size_t)k, sizeof(int64_t));
  C.wsum = (int64_t *)calloc((size_t)k, sizeof(int64_t));
  C.touched = (int32_t *)calloc((size_t)n, sizeof(int32_t));
  C.inq = (uint8_t *)calloc((size_t)n, 1);
  C.gain = (int64_t *)calloc((size_t)n, sizeof(int64_t));
  C.tgt = (int32_t *)calloc((size_t)n, sizeof(int32_t));
  C.q = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  C.mv = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  C.mfrom = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  uint64_t *tk = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
  int64_t *toff = (int64_t *)calloc((size_t)npairs + 1, sizeof(int64_t));
  int32_t *todo = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t rc = 0;
  if (!C.bw || !C.wsum || !C.touched || !C.inq || !C.gain || !C.tgt || !C.q || !C.mv || !C.mfrom ||
      !tk || !toff || !todo) { rc = -7; goto done; }
  C.ev = ev;
  C.evcap = evcap;
  int64_t cV = 0, maxc = 0;
  for (int32_t u = 0; u < n; u++) {
    cV += g->vwgt[u];
    if (g->vwgt[u] > maxc) maxc = g->vwgt[u];
    C.bw[part[u]] += g->vwgt[u];
  }
  C.lmax = (int64_t)(((__int128)(1000000 + (int64_t)p->eps_ppm) * cV) / ((__int128)1000000 * k)) +
           maxc;
  for (int32_t b = 0; b < k; b++) C.over += C.bw[b] > C.lmax;
  /* the todo lists, all formed before the first round */
  for (int32_t i = 0; i < npairs; i++) {
    int32_t a = pairs[2 * i], b = pairs[2 * i + 1];
    int64_t nt = 0;
    for (int32_t u = 0; u < n; u++) {
      if (part[u] != a && part[u] != b) continue;
      int boundary = 0;
      for (int32_t e = g->xadj[u]; e < g->xadj[u + 1] && !boundary; e++)
        boundary = part[g->adjncy[e]] != part[u];
      if (boundary) tk[nt++] = ((mt_key(C.seed, 0, (uint64_t)u) >> 32) << 32) | (uint32_t)u;
    }
    qsort(tk, (size_t)nt, sizeof(uint64_t), cmp_u64);
    for (int64_t j = 0; j < nt; j++) todo[toff[i] + j] = (int32_t)(uint32_t)tk[j];
    toff[i + 1] = toff[i] + nt;
  }
  for (int32_t i = 0; i < npairs; i++) {
    int64_t s = 0, m = 0, kk = 0;
    mt_round(&C, todo + toff[i], (int32_t)(toff[i + 1] - toff[i]), i + 1, &s, &m, &kk, chg);
    kept[i] = kk;
    if (stats3) { stats3[0] += s; stats3[1] += m; stats3[2] += kk; }
  }
  if (nev) *nev = C.nev;
done:
  free(C.bw); free(C.wsum); free(C.touched); free(C.inq); free(C.gain); free(C.tgt); free(C.q);
  free(C.mv); free(C.mfrom); free(tk); free(toff); free(todo);
  return rc;
}

/* The multi-try phase alone on a partition (for tests): pairs [2*npairs]
 * (block-disjoint), stats[3] = searches, moves made, moves kept; kept
 * [npairs]; chg (optional, [k]); events as for mt_phase. */
int32_t or_multitry(const or_graph *g, int32_t *part, int32_t k, const int32_t *pairs,
                    int32_t npairs, int32_t eps_ppm, int32_t alpha, uint32_t seed,
                    int64_t *stats, int64_t *kept, uint8_t *chg, int64_t *ev, int64_t evcap,
                    int64_t *nev) {
  if (alpha < 1 || eps_ppm < 0 || npairs < 0) return -8;
  or_params p;
  memset(&p, 0, sizeof(p));
  p.eps_ppm = eps_ppm;
  p.mt_alpha = alpha;
  p.mt_seed = (int32_t)seed;
  memset(stats, 0, sizeof(int64_t) * 3);
  return mt_phase(g, part, k, pairs, npairs, &p, kept, stats, chg, ev, evcap, nev);
}

/* Adaptive flow iterations (Sec. 4.1) on one pair, after its 2-way FM when
 * fm_limit > 0: the pairwise improvement.  trace (optional) gets one record
 * per solve, at most p->max_iters.  side_out: of the last solve. */
static int32_t refine_pair_core(const or_graph *g, int32_t *part, int32_t k, int32_t a, int32_t b,
                                const or_params *p, or_result *res, int8_t *side_out,
                                or_solve *trace) {
  memset(res, 0, sizeof(*res));
  if (a < 0 || b < 0 || a >= k || b >= k || a == b) return -3;
  if (p->alpha < 1 || p->alpha_max < 1 || p->max_iters < 1 || p->eps_ppm < 0 ||
      (p->area_mode != 0 && p->area_mode != 1) || p->depth < 0 || p->mb_reps < 0 ||
      p->fm_limit < 0 || p->cut_side < 0 || p->cut_side > 2 ||
      (p->terminals != 0 && p->terminals != 1) || p->mt_alpha < 0 || p->restart_alpha < 0)
    return -8;
  int64_t w_a = 0, w_b = 0;
  for (int32_t u = 0; u < g->n; u++) {
    if (part[u] == a) w_a += g->vwgt[u];
    if (part[u] == b) w_b += g->vwgt[u];
  }
  res->cut_before = pair_cut(g, part, a, b);
  int64_t fm_kept = 0;
  if (p->fm_limit > 0) {
    /* Sec. 2.2 / appendix: the pairwise improvement starts with 2-way FM,
     * followed by the flow-based improvement */
    int64_t cV = 0, maxc = 0;
    for (int32_t u = 0; u < g->n; u++) {
      cV += g->vwgt[u];
      if (g->vwgt[u] > maxc) maxc = g->vwgt[u];
    }
    int64_t lmax = (int64_t)(((__int128)(1000000 + (int64_t)p->eps_ppm) * cV) /
                             ((__int128)1000000 * k)) + maxc;
    or_fminfo fi;
    if (pair_fm(g, part, a, b, lmax, p->fm_limit, (uint64_t)(uint32_t)p->fm_seed, &fi, NULL) != 0)
      return -7;
    fm_kept = fi.kept;
  }
  int32_t alpha = p->alpha < p->alpha_max ? p->alpha : p->alpha_max;
  int32_t last = 0;
  int stopped = 0;
  const int32_t restart = p->restart_alpha < p->alpha_max ? p->restart_alpha : p->alpha_max;
  const int32_t start = alpha;
  int restarted = 0;
  for (int32_t it = 0; it < p->max_iters; it++) {
    or_solve rec;
    if (solve_once(g, part, k, a, b, p, alpha, &rec, side_out) != 0) return -7;
    if (trace) trace[it] = rec;
    res->iters++;
    res->final_alpha = alpha;
    res->flow_value = rec.flow;
    res->region_vertices += rec.region_vertices;
    res->region_edges += rec.region_edges;
    last = rec.decision;
    if (rec.decision == DEC_APPLY) {
      res->applied++;
      if (!p->adaptive) { stopped = 1; break; }
      alpha = 2 * alpha < p->alpha_max ? 2 * alpha : p->alpha_max;
    } else if (rec.decision == DEC_INFEASIBLE) {
      if (!p->adaptive || alpha == 1) { stopped = 1; break; }
      alpha = alpha / 2 > 1 ? alpha / 2 : 1;
    } else if (rec.decision == DEC_EQUAL && res->applied == 0 && !restarted && start < restart) {
      restarted = 1; /* R6b: once, from the plain search's start */
      alpha = restart;
    } else {
      stopped = 1; /* feasible and not improving, or not adjacent */
      break;
    }
  }
  res->iter_cap = !stopped;
  if (last == DEC_NOT_ADJ && res->applied == 0) res->status = ST_NOT_ADJACENT;
  else if (res->applied > 0 || fm_kept > 0) res->status = ST_ACCEPTED;
  else if (last == DEC_INFEASIBLE) res->status = ST_REJECTED;
  else res->status = ST_NO_IMPROVEMENT;
  res->cut_after = pair_cut(g, part, a, b);
  res->weight_a = 0;
  res->weight_b = 0;
  for (int32_t u = 0; u < g->n; u++) {
    if (part[u] == a) res->weight_a += g->vwgt[u];
    if (part[u] == b) res->weight_b += g->vwgt[u];
  }
  (void)w_a; (void)w_b;
  return 0;
}

/* Pairs of one quotient-graph matching: the pairwise improvements one after
 * the other (the pairs must be block-disjoint, so their order does not change
 * the outcome), then with mt_alpha > 0 the multi-try phase over the pairs in
 * their order.  chg (optional, [k]): blocks changed by the multi-try phase. */
static int32_t refine_batch(const or_graph *g, int32_t *part, int32_t k, const int32_t *pairs,
                            int32_t npairs, const or_params *p, or_result *res, or_solve *trace,
                            int8_t *side_out, uint8_t *chg) {
  uint8_t *used = (uint8_t *)calloc((size_t)(k > 0 ? k : 1), 1);
  if (!used) return -7;
  for (int32_t i = 0; i < npairs; i++) {
    int32_t a = pairs[2 * i], b = pairs[2 * i + 1];
    if (a < 0 || b < 0 || a >= k || b >= k || a == b) { free(used); return -3; }
    if (used[a] || used[b]) { free(used); return -4; }
    used[a] = used[b] = 1;
  }
  free(used);
  for (int32_t i = 0; i < npairs; i++) {
    int32_t rc = refine_pair_core(g, part, k, pairs[2 * i], pairs[2 * i + 1], p, &res[i], side_out,
                                  trace ? trace + (size_t)i * p->max_iters : NULL);
    if (rc != 0) return rc;
  }
  if (p->mt_alpha > 0 && npairs > 0) {
    int64_t *kept = (int64_t *)calloc((size_t)npairs, sizeof(int64_t));
    if (!kept) return -7;
    int32_t rc = mt_phase(g, part, k, pairs, npairs, p, kept, NULL, chg, NULL, 0, NULL);
    for (int32_t i = 0; i < npairs && rc == 0; i++) res[i].mt_kept = kept[i];
    free(kept);
    if (rc != 0) return rc;
  }
  return 0;
}

int32_t or_refine_pair(const or_graph *g, int32_t *part, int32_t k, int32_t a, int32_t b,
                       const or_params *p, or_result *res, int8_t *side_out, or_solve *trace) {
  const int32_t pr[2] = {a, b};
  return refine_batch(g, part, k, pr, 1, p, res, trace, side_out, NULL);
}

int32_t or_refine_batch(const or_graph *g, int32_t *part, int32_t k, const int32_t *pairs,
                        int32_t npairs, const or_params *p, or_result *res, or_solve *trace) {
  return refine_batch(g, part, k, pairs, npairs, p, res, trace, NULL, NULL);
}

/* Quotient graph (Sec. 2.1): one edge {a,b}, a < b, per pair of blocks that
 * share a cut edge, sorted by (a,b).  Greedy edge colouring: in that order,
 * each edge takes the smallest colour free at both ends, so every colour
 * class is a matching.  Returns the number of edges (or -1). */
int32_t or_quotient_colouring(const or_graph *g, const int32_t *part, int32_t k,
                              int32_t *edges, int32_t *colour, int32_t max_edges) {
  uint8_t *adj = (uint8_t *)calloc((size_t)k * k, 1);
  if (!adj) return -1;
  for (int32_t u = 0; u < g->n; u++)
    for (int32_t e = g->xadj[u]; e < g->xadj[u + 1]; e++) {
      int32_t x = part[u], y = part[g->adjncy[e]];
      if (x < y) adj[(size_t)x * k + y] = 1;
    }
  int32_t ne = 0;
  for (int32_t x = 0; x < k; x++)
    for (int32_t y = x + 1; y < k; y++)
      if (adj[(size_t)x * k + y]) {
        if (ne >= max_edges) { free(adj); return -1; }
        edges[2 * ne] = x;
        edges[2 * ne + 1] = y;
        ne++;
      }
  free(adj);
  /* used[c*k + block] */
  int32_t maxc = 2 * k + 1;
  uint8_t *used = (uint8_t *)calloc((size_t)maxc * k, 1);
  if (!used) return -1;
  for (int32_t i = 0; i < ne; i++) {
    int32_t x = edges[2 * i], y = edges[2 * i + 1], c = 0;
    while (used[(size_t)c * k + x] || used[(size_t)c * k + y]) c++;
    used[(size_t)c * k + x] = used[(size_t)c * k + y] = 1;
    colour[i] = c;
  }
  free(used);
  return ne;
}

/* Total cut sum_{i<j} omega(E_ij) (Sec. 2.1). */
int64_t or_total_cut(const or_graph *g, const int32_t *part) {
  int64_t c = 0;
  for (int32_t u = 0; u < g->n; u++)
    for (int32_t e = g->xadj[u]; e < g->xadj[u + 1]; e++)
      if (part[u] != part[g->adjncy[e]]) c += g->adjwgt[e];
  return c / 2;
}

/* Refinement sweep: build and colour the quotient graph, refine the pairs of
 * each colour class in colour order, repeat until a sweep changes nothing or
 * max_sweeps is reached.  With active_blocks (Sec. 4.3, active block
 * scheduling): every block starts active; a sweep refines only the pairs with
 * an active block (the colour classes of the whole quotient graph, filtered),
 * and the blocks of the pairs it changed are the active ones of the next
 * sweep.  A pair changed when a flow solve or its FM pass changed the
 * partition, or its multi-try round kept a move; the blocks a kept multi-try
 * move left or entered are active in the next sweep too.  Returns 0; stats[0] = sweeps run, stats[1] = flow solves,
 * stats[2] = changed pairs, stats[3] = region edges. */
int32_t or_sweep(const or_graph *g, int32_t *part, int32_t k, const or_params *p,
                 int32_t max_sweeps, int64_t *total_cut_out, int64_t *stats) {
  int32_t maxe = k * (k - 1) / 2 + 1;
  int32_t *edges = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)maxe);
  int32_t *colour = (int32_t *)malloc(sizeof(int32_t) * (size_t)maxe);
  int32_t *pairs = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)maxe);
  or_result *res = (or_result *)malloc(sizeof(or_result) * (size_t)maxe);
  uint8_t *act = (uint8_t *)malloc((size_t)k), *nact = (uint8_t *)malloc((size_t)k);
  if (!edges || !colour || !pairs || !res || !act || !nact) {
    free(edges); free(colour); free(pairs); free(res); free(act); free(nact);
    return -7;
  }
  memset(act, 1, (size_t)k);
  memset(stats, 0, sizeof(int64_t) * 4);
  int32_t rc = 0;
  for (int32_t s = 0; s < max_sweeps; s++) {
    int32_t ne = or_quotient_colouring(g, part, k, edges, colour, maxe);
    if (ne < 0) { rc = -7; break; }
    int32_t ncol = 0;
    for (int32_t i = 0; i < ne; i++) if (colour[i] + 1 > ncol) ncol = colour[i] + 1;
    int64_t changed = 0;
    memset(nact, 0, (size_t)k);
    for (int32_t c = 0; c < ncol; c++) {
      int32_t np = 0;
      for (int32_t i = 0; i < ne; i++)
        if (colour[i] == c && (!p->active_blocks || act[edges[2 * i]] || act[edges[2 * i + 1]])) {
          pairs[2 * np] = edges[2 * i];
          pairs[2 * np + 1] = edges[2 * i + 1];
          np++;
        }
      if (np == 0) continue;
      rc = refine_batch(g, part, k, pairs, np, p, res, NULL, NULL, nact);
      if (rc != 0) break;
      for (int32_t i = 0; i < np; i++) {
        stats[1] += res[i].iters;
        stats[3] += res[i].region_edges;
        if (res[i].status == ST_ACCEPTED) nact[pairs[2 * i]] = nact[pairs[2 * i + 1]] = 1;
        if (res[i].status == ST_ACCEPTED || res[i].mt_kept > 0) changed++;
      }
    }
    if (rc != 0) break;
    stats[0]++;
    stats[2] += changed;
    if (changed == 0) break;
    memcpy(act, nact, (size_t)k);
  }
  *total_cut_out = or_total_cut(g, part);
  free(edges); free(colour); free(pairs); free(res); free(act); free(nact);
  return rc;
}

/* Per-pair input features for the learned area factor (no counterpart in the
 * paper): boundary sizes, block weights, pair cut, slacks to L_max and the
 * alpha = 1 area bound relative to the boundary weight.  f[0..7]:
 *   log2(1+|dA|), log2(1+|dB|), c(A)/W, c(B)/W, log2(1+cut_AB),
 *   (Lmax-c(A))/W, (Lmax-c(B))/W, log2(1 + U_A(1)/max(1,c(dA)))
 * with W = c(V)/k.  Double precision. */
int32_t or_pair_features(const or_graph *g, const int32_t *part, int32_t k, int32_t a,
                         int32_t b, int32_t eps_ppm, double *f) {
  if (a < 0 || b < 0 || a >= k || b >= k || a == b) return -3;
  int64_t cV = 0, maxc = 0, cA = 0, cB = 0, nda = 0, ndb = 0, wda = 0, cut = 0;
  for (int32_t u = 0; u < g->n; u++) {
    cV += g->vwgt[u];
    if (g->vwgt[u] > maxc) maxc = g->vwgt[u];
    if (part[u] != a && part[u] != b) continue;
    int32_t other = part[u] == a ? b : a;
    int hit = 0;
    for (int32_t e = g->xadj[u]; e < g->xadj[u + 1]; e++)
      if (part[g->adjncy[e]] == other) {
        hit = 1;
        if (part[u] == a) cut += g->adjwgt[e];
      }
    if (part[u] == a) { cA += g->vwgt[u]; if (hit) { nda++; wda += g->vwgt[u]; } }
    else { cB += g->vwgt[u]; if (hit) ndb++; }
  }
  int64_t lmax = (int64_t)(((__int128)(1000000 + (int64_t)eps_ppm) * cV) /
                           ((__int128)1000000 * k)) + maxc;
  int64_t u1 = (int64_t)(((__int128)(1000000 + (int64_t)eps_ppm) * cV) /
                         ((__int128)1000000 * k)) - cB;
  if (u1 < 0) u1 = 0;
  double W = (double)cV / (double)k;
  if (W <= 0) W = 1;
  f[0] = log2(1.0 + (double)nda);
  f[1] = log2(1.0 + (double)ndb);
  f[2] = (double)cA / W;
  f[3] = (double)cB / W;
  f[4] = log2(1.0 + (double)cut);
  f[5] = (double)(lmax - cA) / W;
  f[6] = (double)(lmax - cB) / W;
  f[7] = log2(1.0 + (double)u1 / (double)(wda > 1 ? wda : 1));
  return 0;
}
