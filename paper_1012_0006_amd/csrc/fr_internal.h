// Internal layout shared by the kernels and the host driver of libflowrefine.
#pragma once
#include <stdint.h>

#include "flowrefine.h"

#define FR_MAX_ALPHA 1024
#define FR_MAX_ITERS 64

// A corridor arc: local head, index of its reverse arc, and the residual
// pair -- the arc's own residual capacity in the low 32 bits, the reverse
// arc's in the high 32 bits.  One record is one 16-byte load.
struct __attribute__((aligned(16))) Arc {
  int32_t lh;
  int32_t lr;
  unsigned long long rc;
};

// Per-pair state of the adaptive flow iterations, kept in device memory
// across the solves of one call.
struct PairState {
  int32_t a, b;
  int32_t alpha;
  int32_t iters, applied, last_dec, iter_cap;
  int32_t start_alpha, final_alpha;
  int32_t last_nr;      // corridor vertices of the last solve
  int32_t nr;           // corridor vertices of the current solve
  int32_t done;         // the adaptive loop has stopped (a slot: not solved this launch)
  int32_t last_slot;    // slot of the pair's last recorded solve
  int32_t restarted;    // the one restart of a learned start has happened
  int64_t cA, cB;       // current block weights
  int64_t cut;          // current pair cut
  int64_t cut0;         // pair cut at call start
  int64_t flow_last;
  int64_t rv_sum, re_sum;
  int64_t sweeps, relabels, bfs_levels, gr_levels, cl_levels;
  int64_t t_corridor, t_build, t_relabel, t_push, t_closure, t_finish;  // wall-clock ticks
  int64_t work[12];     // vertices / arcs touched per phase (W_*), summed over solves
  // most balanced cut, summed over solves: free vertices, residual components
  // among them, solves whose component graph was too large for LDS (kept in
  // device memory), wall-clock ticks
  int64_t mb_free, mb_comp, mb_big, t_mb;
  // 2-way FM before the flow: moves made, moves kept after the rollback
  int64_t fm_steps, fm_kept;
  // multi-try FM after the round (kept on the pair's first entry): searches
  // started, moves made, moves kept after the rollbacks
  int64_t mt_searches, mt_moves, mt_kept;
  // sliced rounds: the phase of the entry's current iteration (0 corridor
  // due, 1 flow under way, 2 solved, waiting for the pair's other slots),
  // the iterations it started (its corridor marks' stamp), the sweeps and
  // relabel interval of a solve that spans launches, and how often its
  // solves continued in a later launch
  int32_t phase, iter;
  int64_t solve_sweeps;
  int32_t rp_eff, slices;
};

// work counters: the data each phase of a solve touches
enum {
  W_BND_VERTS = 0,  // vertices of A u B scanned for the boundary
  W_BND_ARCS,       // their arcs
  W_BFS_ITEMS,      // corridor BFS frontier vertices expanded
  W_BFS_ARCS,       // their arcs
  W_NET_VERTS,      // corridor vertices (network build)
  W_NET_ARCS,       // global arcs of corridor vertices scanned by the build
  W_SWEEP_ITEMS,    // active vertices processed by push/relabel sweeps
  W_SWEEP_ARCS,     // their corridor arcs
  W_GR_ITEMS,       // vertices expanded by global relabels
  W_GR_ARCS,        // their corridor arcs
  W_CL_ITEMS,       // vertices expanded by the residual closure
  W_CL_ARCS,        // their corridor arcs
  W_COUNT
};

// per-pair sums of the current solve (int64 [P][PA_N]), cleared for the next
enum {
  PA_CUT = 0,  // pair cut
  PA_BW0,      // boundary weight, side a / side b
  PA_BW1,
  PA_BC0,      // boundary vertex count, side a / side b
  PA_BC1,
  PA_RARCS,    // corridor arcs
  PA_RCAP,     // their capacity sum
  PA_RCIN,     // weight of the old a-b edges the solve decides
  PA_CS,       // contracted terminals: capacity out of s (the initial excess)
  PA_N
};

struct Ctl {
  int32_t queue;        // next entry of the pair order to take
  int32_t err;          // first FR_E_* seen on the device (0 = none)
  int32_t diag;         // which internal check raised err (DIAG_*)
  int32_t bad_part;     // part[] holds an id outside [0, k)
  int32_t bad_graph;    // set by the validation kernel
  int32_t live;         // entries still iterating (sliced rounds, read by the host)
  int64_t cV;           // total vertex weight
  int64_t maxc;         // max vertex weight
};

enum { DIAG_NONE = 0, DIAG_LIST = 1, DIAG_CLOSURE = 2, DIAG_REV = 3, DIAG_SWEEPS = 4,
       DIAG_OVERFLOW = 5, DIAG_MB = 6, DIAG_FM = 7, DIAG_MT = 8 };

struct KArgs {
  // graph (device)
  int32_t n, k;
  const int32_t *xadj, *adjncy, *adjwgt, *vwgt;
  int32_t *part;
  // pairs of this round (one matching)
  int32_t P;
  const int32_t *pairs;     // [2P]
  int32_t *order;           // [P] pairs in the order workgroups take them
  int32_t *blk2pair;        // [k]
  int32_t *binfo;           // [2k] per block in the round: first entry of its pair while a
                            // slot still iterates (else -1), (other block << 1) | (block is b)
  int32_t *alpha0;          // [P] start factor per pair
  PairState *ps;            // [P]
  fr_solve *trace;          // [P * max_iters] or null
  int64_t *bstat;           // [3k] weight, vertex count, arc count per block
  int32_t *queue;           // [2 * max_iters] pair-queue counters: corridor and flow kernels
  int64_t *pacc;            // [P * PA_N] per-pair sums of the current solve
  int32_t *pcnt;            // [2P] boundary-list and sink-list counters
  // Speculative slots: every pair of the round owns W consecutive entries
  // (pair p, slot s at index p * W + s) that solve the same partition at the
  // factors alpha, alpha/2, ... of its halving chain at once; each slot has
  // its own corridor marks (mark/vmap + (index % W) * mstride).  W = 1: one
  // entry per pair, shared marks (mstride 0).
  int32_t W;
  int64_t mstride;
  fr_solve *srec;           // [P] record of each entry's solve in the current launch
  // pairs still iterating in the current launch, compacted: act[0..nact),
  // prefix sums of their union sizes (vpre) and corridor sizes (cpre)
  int32_t *act, *nact;
  int64_t *vpre, *cpre;
  int64_t *fstat;           // [4P] boundary statistics for the learned factor
  const int64_t *base;      // floor((1 + alpha eps) c(V) / k), alpha = 0..alpha_max
  int64_t lmax;
  // parameters
  int32_t area_mode, depth, alpha_max, adaptive, max_iters, eps_ppm;
  // learned start: a search that started below this factor, applied nothing
  // and met a feasible cut without improvement continues once from it (the
  // plain search's start; 0 = never)
  int32_t restart_alpha;
  int32_t stamp0;           // corridor mark of the first solve (even)
  // most balanced minimum cut: sweeps (0 = smallest source set), key seed,
  // component graph in LDS when it fits, quotient arcs (one slot per arc slot)
  int32_t mb_reps, mb_seed, mb_lds;
  int32_t *mbq;
  int32_t *mbc;             // large component graphs: 4 words per arena vertex slot
  int64_t *mpre;            // [P + 1] prefix sums of the entries' free-vertex counts
  // 2-way FM before the flow: non-improving moves before it stops (0 = off),
  // key seed, per-vertex gains and queue positions (-1 not queued, -2 moved)
  int32_t fm_limit, fm_seed;
  int32_t *fmg, *fmq;
  // candidate without the most balanced cut: 0 smallest source set, 1 largest,
  // 2 the largest only when the smallest is infeasible and it is feasible
  int32_t cut_side;
  // multi-try FM after the round (0 = off): stopping-rule alpha, key seed,
  // beta = floor(ln n 2^16), touched stamp of the round's first pair minus 1;
  // block weights [k], todo keys and their sort buffer (arena slots),
  // per-vertex touched stamps, targets and heap slots (-1 none), heap slots
  // beyond LDS [2n], move log of a search [n] x 2, changed blocks [k]
  int32_t mt_alpha, mt_seed;
  int64_t mt_beta;
  int32_t mt_stamp0;
  int64_t *mtw;
  unsigned long long *mtk, *mtk2;
  int32_t *mtt, *mtb, *mtq, *mth, *mtv, *mtf;
  uint8_t *mtchg;
  // terminals of the corridor network: 0 border pinned by infinite arcs,
  // 1 the blocks' outside parts contracted into s / t (per-vertex capacities:
  // s -> u as the initial excess, u -> t in the sink-list array SNK)
  int32_t terminals;
  // per vertex [n]
  int32_t *mark, *vmap;
  // per-pair arenas: vertex slots [voff[p], voff[p+1]), arc slots [aoff[p], aoff[p+1])
  int64_t *voff, *aoff;
  int32_t *ucnt;            // [P] fill counters of the union lists
  int32_t *uvert;           // vertices of blocks a and b of each pair
  int32_t *lg;              // corridor: local id -> global id
  int32_t *lo;              // local CSR offsets (n + P slots: nv_p + 1 per pair)
  int32_t *ex, *lab, *ins, *LA, *LB, *SNK;
  uint8_t *lflag;
  Arc *arc;                 // local arcs (one 16-byte record each)
  Ctl *ctl;
  // launch
  int32_t tpv, relabel_period;
  // sliced rounds: device-clock ticks an entry's flow may run in one launch
  // before it stops at the next due global relabel (0: run to the end)
  int64_t slice_ticks;
  int64_t max_sweeps;
  int8_t *side_out;
};

// corridor vertex flags
#define LF_SIDE_B 1u   // vertex of block b (sink side)
#define LF_BORDER 2u   // has a neighbour in A u B outside the corridor
#define LF_SRC(f) (((f) & 3u) == LF_BORDER)
#define LF_SNK(f) (((f) & 3u) == (LF_BORDER | LF_SIDE_B))
