/*
 * flowrefine -- max-flow min-cut local refinement between pairs of blocks of a
 * graph partition, on one AMD Instinct MI355X (gfx950).
 *
 * Method: Sanders & Schulz, "Engineering Multilevel Graph Partitioning
 * Algorithms", Section 4.1 ("Using Max-Flow Min-Cut Computations for Local
 * Improvement").  For a pair of adjacent blocks (a, b):
 *   1. boundary nodes of a towards b and of b towards a (Sec. 4.1, delta_l/r);
 *   2. a BFS inside each block from its boundary, stopped once the area would
 *      exceed (1 + alpha*eps) c(V)/k - c(other block) (Sec. 4.1, corridor B,
 *      generalised from k = 2 to k blocks);
 *   3. the corridor network G': G[B] plus s -> left corridor border and right
 *      corridor border -> t with infinite capacity (Sec. 4.1);
 *   4. a maximum s-t flow (push-relabel with global relabelling);
 *   5. the minimum cut with the smallest source set, i.e. the vertices
 *      reachable from s in the residual graph (Sec. 4.1.1, Ford-Fulkerson
 *      labelling), or on request the most balanced minimum cut found by the
 *      heuristic of Sec. 4.1.1 (see fr_params.mb_reps);
 *   6. the balance check c(V_i) <= L_max = (1+eps) c(V)/k + max_v c(v)
 *      (Sec. 2.1) and the adaptive flow iterations on alpha (Sec. 4.1).
 * All arithmetic is integer.  Every output (flow value, smallest source set,
 * partition, cut, block weights, alpha sequence) is unique, so it can be
 * compared bit for bit with any exact reference.
 *
 * Readings of points the paper leaves open:
 *   - only blocks a and b matter: the border is taken within G[A u B];
 *   - BFS levels are walked in ascending vertex id and the walk stops for good
 *     at the first vertex that would exceed the bound;
 *   - area bound U_x(alpha) = floor((1+alpha*eps) c(V)/k) - c(other), >= 0;
 *   - acceptance uses L_max with the original eps;
 *   - adaptive loop: start at alpha (<= alpha_max); accepted => alpha =
 *     min(2 alpha, alpha_max) and repeat; infeasible => alpha = max(alpha/2,1),
 *     stop if it already was 1; feasible but not smaller => stop; at most
 *     max_iters flow solves;
 *   - the first block of a pair is the source side;
 *   - most balanced minimum cut: a cut's balance is the heavier of the two
 *     new block weights; a random topological order of the remaining residual
 *     components takes, among those whose predecessors are all placed, the
 *     one with the smallest key (SplitMix64, see mb_seed); the first most
 *     balanced cut wins (earlier sweep, then earlier position), for any
 *     number of remaining components.
 *
 * Conventions: every entry point returns FR_OK (0) or a negative FR_E_* code,
 * and never throws.  On error the partition is left unchanged.  All buffers
 * are owned by the caller; the library keeps no pointer after a call returns.
 * Calls on one context are serialised by the caller (a context is not
 * thread-safe).  Calls block until their GPU work has finished.
 */
#ifndef FLOWREFINE_H
#define FLOWREFINE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------- */
#define FR_OK 0
#define FR_E_INVALID_GRAPH (-1)      /* CSR malformed, asymmetric, self loop, weight out of range */
#define FR_E_INVALID_PART (-2)       /* part[v] outside [0, k) */
#define FR_E_INVALID_PAIR (-3)       /* block id outside [0, k), or a == b */
#define FR_E_PAIRS_NOT_DISJOINT (-4) /* two pairs of one batch share a block */
#define FR_E_OVERFLOW (-5)           /* capacities of one corridor reach 2^31, or an edge weight >= 2^30 */
#define FR_E_DEVICE (-6)             /* HIP runtime error, or a failed internal consistency check */
#define FR_E_OOM (-7)                /* device or host allocation failed */
#define FR_E_INVALID_ARG (-8)        /* NULL pointer, bad parameter value */
#define FR_E_SOLVER_LIMIT (-9)       /* push-relabel exceeded its sweep safety cap, or a
                                        sliced round ran more than max(256 max_iters,
                                        65,536) launches */
#define FR_E_SCRATCH_LIMIT (-10)     /* flow_refine_pair_static: graph beyond its static scratch */

/* ---- per-pair status (fr_result.status) --------------------------------- */
#define FR_ACCEPTED 1           /* at least one flow solve was applied */
#define FR_REJECTED_IMBALANCE 2 /* nothing applied; the last candidate broke L_max */
#define FR_NO_IMPROVEMENT 3     /* nothing applied; the last candidate was feasible, not smaller */
#define FR_NOT_ADJACENT 4       /* the blocks share no edge */

/* ---- per-solve decision (fr_solve.decision) ----------------------------- */
#define FR_DEC_APPLY 1
#define FR_DEC_INFEASIBLE 2
#define FR_DEC_EQUAL 3
#define FR_DEC_NOT_ADJACENT 4

/* ---- area modes (fr_params.area_mode) ----------------------------------- */
#define FR_AREA_FACTOR 0 /* weight-bounded corridor, U_x(alpha) */
#define FR_AREA_DEPTH 1  /* every vertex within BFS distance <= depth of the boundary */

/* Undirected graph as symmetric CSR.  n vertices; xadj[n+1] with xadj[0] = 0
 * and xadj[n] = 2m < 2^31; adjncy[2m] neighbour ids (no self loops, no
 * repeats, each edge stored in both directions); adjwgt[2m] edge weights in
 * [1, 2^30) equal in both directions (omega: E -> R>0, Sec. 2.1); vwgt[n]
 * vertex weights >= 0 (c: V -> R>=0).  on_device = 1: all five pointers and
 * the partition are device pointers (for example torch tensors); 0: host
 * pointers, copied by the library for the call.  Read-only. */
typedef struct {
  int32_t n;
  int32_t on_device;
  const int32_t *xadj;
  const int32_t *adjncy;
  const int32_t *adjwgt;
  const int32_t *vwgt;
} fr_graph;

/* Parameters of the adaptive flow iterations. */
typedef struct {
  int32_t area_mode; /* FR_AREA_FACTOR or FR_AREA_DEPTH */
  int32_t depth;     /* FR_AREA_DEPTH only, >= 0 */
  int32_t alpha;     /* start factor, >= 1 (clamped to alpha_max) */
  int32_t alpha_max; /* upper bound alpha' of the factor, >= 1 */
  int32_t adaptive;  /* 0: one flow solve; 1: adaptive flow iterations */
  int32_t max_iters; /* flow solves per pair, in [1, 64] */
  int32_t eps_ppm;   /* imbalance eps in parts per million (3 % = 30000), >= 0 */
  int32_t use_mlp;   /* start each pair at the learned factor (needs loaded weights) */
  /* Most balanced minimum cut (Sec. 4.1.1; "balanced adaptive flow
   * iterations" when adaptive = 1).  0: the candidate is the smallest source
   * set.  r > 0: after each max flow, the strongly connected components of
   * the residual graph that lie neither with s (its component and successors)
   * nor with t (its component and predecessors) are swept r times: sweep j
   * moves them to the sink side one by one in a random topological order,
   * starting from the largest minimum source side; the candidate is the
   * minimum cut with the smallest max(c'(a), c'(b)) seen.  Flow value and
   * candidate cut are those of any minimum cut; only the balance changes.
   * At most FR_MB_MAX_REPS. */
  int32_t mb_reps;
  /* Keys of the sweeps: component x (identified by its smallest vertex id
   * g) in sweep j gets output number j * 2^32 + g + 1 of SplitMix64 started
   * at mb_seed (the 32 bits, zero-extended to 64). */
  int32_t mb_seed;
  /* Pairwise 2-way FM local search with TopGain before the flow (Sec. 2.2 and
   * the pairwise improvement of active block scheduling: FM, then max-flow
   * min-cut).  0: off.  f > 0: one FM pass on each pair before its adaptive
   * flow iterations, stopped after f moves without a better state (or when
   * no vertex is left to move), rolled back to the best state.  Queues: one
   * per block, ordered by gain, equal gains by the key SplitMix64(fm_seed)
   * output number v + 1 of vertex v (larger first); boundary vertices start
   * queued, a vertex joins when a neighbour moves, each moves at most once.
   * TopGain: the block with the larger top gain moves, the heavier block
   * while one is overloaded (c > L_max), ties by bit 0 of output number
   * 2^32 + t + 1 for move t (1: block b).  Best state: feasible before
   * infeasible, then the smaller pair cut (feasible) or the lighter heavier
   * block (infeasible), the earliest on ties.  Each vertex's weighted degree
   * within the pair must stay below 2^31 (else FR_E_OVERFLOW). */
  int32_t fm_limit;
  int32_t fm_seed;
  /* Sweeps only (Sec. 4.3, active block scheduling): 1 = every block starts
   * active, a sweep refines only the pairs with an active block (the colour
   * classes of the whole quotient graph, filtered) and the blocks of the
   * pairs it changed (a flow solve applied or FM moves kept) are the active
   * ones of the next sweep; 0 = every pair every sweep. */
  int32_t active_blocks;
  /* Candidate cut without most balanced cuts (mb_reps = 0; with them the
   * sweeps already include both): 0 = the smallest source set (Sec. 4.1.1);
   * 1 = the largest minimum source side, every corridor vertex that cannot
   * reach t in the residual graph; 2 = the smallest, or the largest when the
   * smallest breaks L_max and the largest does not.  Both have the minimum
   * cut's value, so only the balance differs. */
  int32_t cut_side;
  /* Terminals of the corridor network.  FR_TERM_PINNED (0, Sec. 4.1): the
   * corridor border is tied to s / t by infinite arcs, so it never moves.
   * FR_TERM_CONTRACTED (1): the parts of blocks a and b outside the corridor
   * are contracted into s and t; a corridor vertex gets an arc s -> u of the
   * weight of its edges into a outside the corridor and an arc u -> t of the
   * weight of its edges into b outside.  Every corridor vertex may then
   * change sides: the minimum cut is the best reassignment of the corridor
   * (balance aside), never worse than the pinned one.  Those arc capacities
   * count toward the 2^31 capacity bound. */
  int32_t terminals;
  /* Multi-try FM (Sec. 4.2; "localized k-way searches"), after the pairwise
   * improvements of a batch or of each round of a sweep.  0: off.  a > 0:
   * one multi-try round per pair, in pair order (the searches of a round
   * may move vertices into any block, so they run one after the other): the
   * round's todo list is every vertex of the pair's two blocks with a
   * neighbour in another block, taken when the phase starts, in the order of
   * key SplitMix64(mt_seed) output number 2^40 + v + 1 (its upper 32 bits,
   * then v); an entry that is still a boundary vertex and was not touched by
   * an earlier search of the round starts a k-way search from itself and
   * its untouched boundary neighbours.  The search keeps one queue ordered by
   * the k-way gain (the largest weight to another adjacent block minus the
   * weight to the own block; target ties by the smaller key of output
   * 2^42 + v*k + P + 1), equal gains by the larger key of output 2^41 + v +
   * 1; a popped vertex moves unless its target would exceed L_max; a moved
   * vertex's untouched boundary neighbours join, queued ones are updated (and
   * leave without a target); it stops when the queue is empty or when
   * p mu^2 > a sigma^2 + ln n over the p moves since the last best state
   * (KaSPar's rule, evaluated exactly with ln n as floor(ln n * 2^16) /
   * 2^16), then rolls back to the first state with the fewest blocks above
   * L_max, then the lowest cut.  Vertices a search queued are not queued
   * again in the round.  Each vertex's weighted degree must stay below 2^31
   * (else FR_E_OVERFLOW).  The paper uses a = 10. */
  int32_t mt_alpha;
  int32_t mt_seed;
  /* With use_mlp, 1: a pair that started below alpha, has applied nothing and
   * meets a feasible cut without improvement continues once from alpha (the
   * plain search's start) within the same max_iters, so the learned start
   * never ends a pair's search that the plain search would have continued
   * from a larger corridor; 0: it stops there (the adaptive rule of
   * Sec. 4.1 as is).  Must be 0 or 1. */
  int32_t mlp_restart;
} fr_params;

#define FR_TERM_PINNED 0
#define FR_TERM_CONTRACTED 1

#define FR_MB_MAX_REPS 256

/* Outcome of one pair. */
typedef struct {
  int32_t status;      /* FR_ACCEPTED, FR_REJECTED_IMBALANCE, FR_NO_IMPROVEMENT, FR_NOT_ADJACENT */
  int32_t iters;       /* flow solves run */
  int32_t final_alpha; /* factor of the last solve */
  int32_t applied;     /* solves whose candidate was applied */
  int32_t iter_cap;    /* 1 if the loop stopped only because of max_iters */
  int32_t start_alpha; /* factor of the first solve (differs from alpha with use_mlp) */
  int64_t flow_value;  /* max-flow value of the last solve */
  int64_t cut_before, cut_after;         /* pair cut omega(E_ab) before / after the call */
  int64_t weight_a, weight_b;            /* c(V_a), c(V_b) after the call */
  int64_t region_vertices, region_edges; /* corridor vertices / edges summed over the solves */
  int64_t mt_kept;     /* multi-try moves kept after this pair's improvement (status,
                          cut_after and weights are those of the pairwise improvement) */
} fr_result;

/* One flow solve (trace record). */
typedef struct {
  int32_t alpha;
  int32_t decision;        /* FR_DEC_* */
  int64_t flow;            /* max-flow value */
  int64_t region_vertices; /* |B| */
  int64_t region_edges;    /* edges of G[B] */
  int64_t source_side;     /* corridor vertices on the source side of the candidate cut */
  int64_t cut_before;      /* pair cut before the solve */
  int64_t cut_candidate;   /* pair cut of the candidate partition */
  int64_t wa, wb;          /* block weights of the candidate */
} fr_solve;

/* Kernel launch parameters; any valid setting gives identical results. */
typedef struct {
  int32_t block_threads;   /* threads per workgroup of the per-pair kernels: 256, 512 or 1024 */
  int32_t blocks_per_cu;   /* persistent per-pair workgroups per compute unit: 1..8 */
  int32_t tpv;             /* lanes per vertex in push/relabel sweeps: 1, 2, 4, 8 or 16
                              (1 runs as 2, 16 as 8) */
  int32_t relabel_period;  /* global relabel interval, 1..10^6: after a global relabel
                              whose search took L levels, the next one follows after
                              L/2 push/relabel sweeps, clamped to [period/4 (at least
                              1), 2 period], or when the active list runs dry */
  int32_t mb_lds;          /* most balanced cut: 1 = component graph in LDS when it fits,
                              0 = always in device memory */
  int32_t slice_us;        /* sliced rounds, 0..10^7 us (0 = off): a flow-kernel launch
                              gives each solve this much device time, then stops it at
                              the next global relabel that is due anyway, if by then at
                              most a quarter of the launch's solves still run; it
                              continues in the next launch of the chain, while the pairs
                              whose solves ended start their next adaptive iteration,
                              so they no longer wait for the round's slowest pair; the
                              chain may then run past max_iters launches.  Rounds of
                              one pair, captured sweeps, most balanced cuts, fused
                              rounds and the entry point without device allocation run
                              unsliced.  (Every call that is not captured ends its chain
                              once no pair iterates: the host reads the count back after
                              2, 4 and 8 launches and then every 4.) */
} fr_tuning;

typedef struct fr_context fr_context;

/* Create a context on HIP device `device`.  Calls wait for work already
 * queued on `hip_stream` (a hipStream_t; NULL = the null stream) and run on
 * the context's own stream.  Device scratch is allocated lazily and grows
 * with the largest graph seen: per-pair arenas and corridor marks take
 * (speculative factors per pair) x (n vertices, 2m arcs) slots, at most
 * 2^28 vertex and 2^29 arc slots. */
int32_t fr_create(int32_t device, void *hip_stream, fr_context **ctx);
int32_t fr_destroy(fr_context *ctx);
const char *fr_strerror(int32_t code);

/* The imbalance eps as a fraction (0.03 = 3 %) in parts per million, rounded
 * to the nearest, for fr_params.eps_ppm; FR_E_INVALID_ARG outside [0, 100] or
 * for NaN.  No GPU work. */
int32_t fr_eps_to_ppm(double eps, int32_t *ppm);

/* Adaptive flow refinement of one pair (a = source side, b = sink side):
 * Sec. 4.1 (boundary, corridor by bounded BFS, network with the border tied
 * to s and t, maximum flow, minimum cut, adaptive flow iterations) and Sec.
 * 4.1.1 (the smallest source set, or the most balanced minimum cut), preceded
 * by 2-way FM (Sec. 2.2) with fm_limit and followed by a multi-try round
 * (Sec. 4.2) with mt_alpha.
 * part: [n] in/out, block ids in [0, k).  res: host, one record.
 * side_out (optional, host int8 [n]): per vertex of the LAST solve, -1 outside
 * the corridor, 0 / 1 corridor vertex ending in a / b, 2 / 3 border vertex
 * pinned to s (block a) / t (block b; pinned terminals only).
 * trace (optional, host, p->max_iters records): one record per solve. */
int32_t flow_refine_pair(fr_context *ctx, const fr_graph *g, int32_t *part, int32_t k,
                         int32_t a, int32_t b, const fr_params *p, fr_result *res,
                         int8_t *side_out, fr_solve *trace);

/* flow_refine_pair for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same computation and results, with every vertex-, arc-
 * and block-sized buffer taken from a static device array of 64 MiB that
 * the library holds on each GPU it runs on until the process ends (its
 * address is resolved by fr_create); no hipMalloc, hipFree or other
 * allocating call is made.  Limits: the graph and part must be device
 * pointers (g->on_device = 1); mb_reps, fm_limit and use_mlp must be 0;
 * no side output; the adaptive iterations run one solve at a time (no
 * speculative factors).  The buffers need about 49 bytes per vertex plus
 * 16 per arc (each undirected edge twice) plus 28 per block, each piece
 * rounded to 256 bytes: a graph beyond 64 MiB of that returns
 * FR_E_SCRATCH_LIMIT before any device work, with part unchanged (2D RGG
 * n = 2^18, mean degree 8, takes 47 MB).  Calls on one GPU share the array
 * and keep no state in it between calls (it is cleared where needed), so
 * calls that overlap on one GPU -- from several contexts or threads -- race
 * and must be serialised by the caller.  res / trace as for
 * flow_refine_pair. */
int32_t flow_refine_pair_static(fr_context *ctx, const fr_graph *g, int32_t *part, int32_t k,
                                int32_t a, int32_t b, const fr_params *p, fr_result *res,
                                fr_solve *trace);

/* All pairs of one quotient-graph matching in one batched solve (Sec. 4.3:
 * the pairs of a matching touch disjoint blocks, so their pairwise
 * improvements are independent; with mt_alpha the multi-try rounds of the
 * pairs follow in pair order).  pairs: host
 * int32 [2*npairs] (a_i, b_i), blocks pairwise disjoint.  res: host
 * [npairs]; trace (optional): host [npairs * p->max_iters], record j of pair i
 * at i*max_iters + j.  With p->use_mlp = 1 each pair starts at the factor the
 * loaded area-factor network predicts (see fr_mlp_*). */
int32_t flow_refine_batch(fr_context *ctx, const fr_graph *g, int32_t *part, int32_t k,
                          const int32_t *pairs, int32_t npairs, const fr_params *p,
                          fr_result *res, fr_solve *trace);

/* Quotient graph of the partition (an edge {a, b}, a < b, per pair of blocks
 * sharing a cut edge; Sec. 2.1) in (a, b) order, greedily edge-coloured (each
 * edge takes the smallest colour free at both ends), so every colour class is
 * a matching.  edges: host int32 [2*max_edges]; colour: host int32
 * [max_edges].  *nedges gets the edge count (FR_E_INVALID_ARG if > max_edges). */
int32_t fr_quotient_matchings(fr_context *ctx, const fr_graph *g, const int32_t *part, int32_t k,
                              int32_t *edges, int32_t *colour, int32_t max_edges,
                              int32_t *nedges);

/* Repeated rounds (Sec. 4.3): build and colour the quotient graph, run one
 * batched solve per colour class in colour order (all rounds of a sweep
 * recorded into one hipGraph and launched once), until a sweep changes
 * nothing or max_sweeps sweeps ran (p->active_blocks: only pairs with a block
 * changed in the previous sweep, or entered or left by a kept multi-try
 * move).  stats (optional, host int64 [4]): sweeps, flow solves, changed
 * pairs (a flow solve applied, or FM or multi-try moves kept), region
 * edges.  total_cut_out: the cut
 * sum_{i<j} omega(E_ij) after the sweep. */
int32_t flow_refine_sweep(fr_context *ctx, const fr_graph *g, int32_t *part, int32_t k,
                          const fr_params *p, int32_t max_sweeps, int64_t *total_cut_out,
                          int64_t *stats);

/* Launch parameters (fr_tuning); FR_E_INVALID_ARG for values out of range. */
int32_t fr_set_tuning(fr_context *ctx, const fr_tuning *t);
int32_t fr_get_tuning(fr_context *ctx, fr_tuning *t);

/* Speculative adaptive iterations (Sec. 4.1, the adaptive factor) on (1, the
 * default) or off (0).  An infeasible candidate halves alpha and solves the
 * same partition again, so each pair can solve its halving chain alpha,
 * alpha/2, ..., 1 at once, one workgroup per factor, and the rule then walks
 * the finished solves in order: the recorded solves, the trace, the result
 * and the partition are those of the sequential loop; solves past the walk
 * are discarded (counted in the work counters, not in region_vertices /
 * region_edges).  Used for pair, batch and sweep calls with adaptive
 * iterations (the chain starts at the learned factor when use_mlp is set), as
 * far as every factor of every pair gets a workgroup slot; fr_last_stats
 * counters[7] reports the factors per pair of the last pair / batch call. */
int32_t fr_set_speculation(fr_context *ctx, int32_t on);

/* Rounds as one launch (1) or as one launch chain per adaptive iteration (0,
 * the default).  With 1, each workgroup takes a pair of the round and runs
 * its whole adaptive loop (Sec. 4.1: boundary, corridor, network, flow, the
 * factor rule) in one persistent kernel, so a pair never waits for the
 * round's other pairs between its iterations; every solve is then one factor
 * (no speculative factors, fr_set_speculation has no effect).  With 0, every
 * iteration of the round is a chain of launches over all pairs, and a pair's
 * next iteration waits for the slowest pair's current one unless its solves
 * are sliced (fr_tuning.slice_us).  Calls with the
 * most balanced cut (mb_reps > 0) always run the launch chains.  Results are
 * identical either way.  The launch chains are the faster choice wherever
 * measured: they keep the speculative factors, and their boundary and
 * network passes spread over the whole chip instead of one workgroup. */
int32_t fr_set_fused(fr_context *ctx, int32_t on);

/* Input checks of every call on (1, the default) or off (0; malformed input
 * then gives undefined results): CSR shape, ids and weights in range, no self
 * loop or repeated neighbour, symmetry with equal weights.  Vertices of more
 * than 16 arcs are checked through hash tables of their neighbours (device
 * memory grown on demand), so the work is O(m) expected; the entry point
 * that allocates nothing scans their lists instead (O(sum of deg^2) over
 * those vertices). */
int32_t fr_set_validation(fr_context *ctx, int32_t on);

/* Per-phase timing of sweeps on (1) or off (0, the default).  On: the rounds
 * of each sweep are launched one by one instead of as one recorded hipGraph,
 * with HIP events around the phases of every adaptive iteration, so
 * fr_last_stats reports the corridor, network-build and flow-kernel times
 * summed over the whole sweep call (results are identical either way).
 * Pair and batch calls always time their phases. */
int32_t fr_set_timing(fr_context *ctx, int32_t on);

/* Statistics of the last pair, batch or sweep call (host arrays, either may
 * be NULL; a sweep sums its rounds, and reports event times only with
 * fr_set_timing on).
 * ms[8]: [0] setup (validation, weights, arenas), [1] the round (setup
 *   kernels and every flow iteration), [2] corridor kernels (boundary and
 *   BFS), [3] network-build kernels, [4] whole call on the device, [5]
 *   global relabels and [6] push/relabel sweeps (device clock time summed
 *   over the pairs' workgroups), [7] flow kernel (relabels, sweeps,
 *   closure, decision), or with fused rounds the round kernel (every phase;
 *   [2] and [3] are then 0); [1..3], [7] are HIP event times.
 * counters[32]: [0] push/relabel sweeps, [1] global relabels, [2] corridor
 *   BFS levels, [3] relabel BFS levels, [4] closure levels, [5] workgroups
 *   of the per-pair kernels, [6] internal check that failed (0 = none),
 *   [7] speculative factors per pair (1 = none); [8] most-balanced-cut
 *   kernels time in ns, [9] free vertices, [10] their residual components,
 *   [11] solves whose component graph (more than 2,048 components) was kept
 *   in device memory instead of LDS; [12] FM moves made, [13] FM moves kept;
 *   [14] flow-kernel launches (one per launch of a round's chain: the chain
 *   ends once no pair iterates, a captured sweep runs max_iters per round),
 *   or round-kernel launches (one per round) with fused rounds; [15] pairs
 *   whose learned start was restarted from alpha (use_mlp);
 *   [28] multi-try searches, [29] multi-try moves made, [30] kept; [31]
 *   solves continued in a later launch (sliced rounds);
 *   [16..27] vertices and arcs touched: boundary scan, corridor BFS, network
 *   build, push/relabel sweeps, global relabels, residual closure (vertices
 *   then arcs for each); the rest 0. */
int32_t fr_last_stats(fr_context *ctx, double *ms, int64_t *counters);

/* ---- learned area factor (no counterpart in the paper) -----------------
 * A small network (8 features -> 64 -> 64 -> 5 classes, ReLU, softmax;
 * FP32) proposes the start factor alpha in {1, 2, 4, 8, 16} of each pair;
 * the adaptive flow iterations then run as usual from that factor, so every
 * flow result stays exact.  Parameters: one float array of
 * fr_mlp_num_params() values, W1[8][64], b1[64], W2[64][64], b2[64],
 * W3[64][5], b3[5] (row-major [in][out]).  All arrays below are host arrays. */
int32_t fr_mlp_num_params(void);
/* He-normal initialisation from a seed; the network counts as loaded. */
int32_t fr_mlp_init(fr_context *ctx, uint64_t seed);
int32_t fr_mlp_set_weights(fr_context *ctx, const float *w, int32_t count);
int32_t fr_mlp_get_weights(fr_context *ctx, float *w, int32_t count);
/* probs[n*5] = softmax output for features x[n*8]. */
int32_t fr_mlp_forward(fr_context *ctx, const float *x, int32_t n, float *probs);
/* Mean cross-entropy of (x, labels in [0,5)) and its gradient grad[num_params]
 * (either output may be NULL). */
int32_t fr_mlp_loss_grad(fr_context *ctx, const float *x, const int32_t *labels, int32_t n,
                         float *loss, float *grad);
/* Mean expected cost of (x, costs) and its gradient (either output may be
 * NULL): costs[n*5] holds every sample's cost of each class (finite), the loss
 * is the mean over the samples of sum_c p_c costs_c with the softmax
 * probabilities p (cost-sensitive classification: the class of least cost
 * is the target, and near misses cost what the costs say). */
int32_t fr_mlp_loss_grad_cost(fr_context *ctx, const float *x, const float *costs, int32_t n,
                              float *loss, float *grad);
/* Start factors alpha[n] in {1, 2, 4, 8, 16} for features x[n*8]: 2^c for the
 * most probable class c (the first on ties), as batch and sweep calls with
 * use_mlp take them. */
int32_t fr_mlp_predict(fr_context *ctx, const float *x, int32_t n, int32_t *alpha);
/* Minibatch Adam (beta 0.9 / 0.999) on the device; epoch_loss[epochs]
 * (optional) = mean cross-entropy over all n samples after each epoch. */
int32_t fr_mlp_train(fr_context *ctx, const float *x, const int32_t *labels, int32_t n,
                     int32_t epochs, int32_t batch, float lr, uint64_t seed, float *epoch_loss);
/* fr_mlp_train on the mean expected cost of per-class costs[n*5] (see
 * fr_mlp_loss_grad_cost); epoch_loss gets that loss. */
int32_t fr_mlp_train_cost(fr_context *ctx, const float *x, const float *costs, int32_t n,
                          int32_t epochs, int32_t batch, float lr, uint64_t seed,
                          float *epoch_loss);
/* Features feats[npairs*8] of block-disjoint pairs: log2(1+|boundary a|),
 * log2(1+|boundary b|), c(a)/W, c(b)/W, log2(1+pair cut), (L_max-c(a))/W,
 * (L_max-c(b))/W, log2(1 + U_a(1)/c(boundary a)); W = c(V)/k. */
int32_t fr_pair_features(fr_context *ctx, const fr_graph *g, const int32_t *part, int32_t k,
                         const int32_t *pairs, int32_t npairs, int32_t eps_ppm, float *feats);

/* ---- autotuner -----------------------------------------------------------
 * Runs one batched round of `pairs` (graph and partition on the device; the
 * partition is not modified) under each candidate tuning, reps timed runs
 * after one warm-up, checks that all candidates give identical results
 * (FR_E_DEVICE otherwise), stores the mean solve time per candidate in
 * ms_out[ncand] (optional) and keeps the fastest as the context's tuning. */
int32_t fr_autotune(fr_context *ctx, const fr_graph *g, const int32_t *part, int32_t k,
                    const int32_t *pairs, int32_t npairs, const fr_params *p,
                    const fr_tuning *candidates, int32_t ncand, int32_t reps, double *ms_out,
                    int32_t *best);

#ifdef __cplusplus
}
#endif
#endif /* FLOWREFINE_H */
