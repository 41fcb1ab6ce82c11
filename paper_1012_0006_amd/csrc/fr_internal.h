// Internal layout shared by the kernels and the host driver of libflowrefine.
#pragma once
#include <stdint.h>

#include "flowrefine.h"

#define FR_MAX_ALPHA 1024
#define FR_MAX_ITERS 64
#define FR_MAX_PAIRS 1024  // pairs of one batched launch (LDS holds 2 sides each)
#define FR_NACC 12

// accumulator slots per pair (int64), zeroed before every round
enum {
  ACC_CUT = 0,    // pair cut measured by the boundary pass
  ACC_CIN,        // weight of old a-b edges with both ends in the corridor
  ACC_FLOW,       // excess collected at the sink border
  ACC_MOVAB,      // weight moving a -> b
  ACC_MOVBA,      // weight moving b -> a
  ACC_SRC,        // corridor vertices in the smallest source set
  ACC_RVERT,      // corridor vertices
  ACC_RARCS,      // corridor arcs (2 per edge)
  ACC_CAP,        // sum of corridor arc capacities
  ACC_NDA,        // boundary vertices of side a
  ACC_NDB,        // boundary vertices of side b
  ACC_WDA         // boundary weight of side a
};

// BFS side states
enum { SIDE_EXPAND = 0, SIDE_DONE = 1, SIDE_CROSS = 2 };

struct PairState {
  int32_t a, b;
  int32_t alpha, active;
  int32_t iters, applied, last_dec, iter_cap;
  int32_t start_alpha, final_alpha;
  int32_t stopped, pad;
  int64_t cA, cB;       // current block weights
  int64_t cut;          // current pair cut (after the last applied solve)
  int64_t cut0;         // pair cut at call start (-1 until measured)
  int64_t flow_last;
  int64_t rv_sum, re_sum;
  int64_t U[2];         // area bound per side for the coming solve
};

struct Ctl {
  int32_t stamp;        // corridor mark of the current round (even, grows by 2)
  int32_t err;          // first FR_E_* seen on the device (0 = none)
  int32_t nr;           // corridor vertices of the round (all pairs)
  int32_t na;           // corridor arcs of the round
  int32_t nsink;        // sink-border vertices
  int32_t active_pairs; // pairs that need another solve
  int32_t cnt[3];       // frontier counters, rotating
  int32_t pad;
  int64_t sweeps;       // push/relabel sweeps (all rounds of the call)
  int64_t relabels;     // global relabels
  int64_t bfs_levels;   // corridor BFS levels
  int64_t gr_levels;    // global-relabel BFS levels
  int64_t cl_levels;    // closure BFS levels
  int64_t cV;           // total vertex weight
  int64_t maxc;         // max vertex weight
  int32_t bad_part;     // set when part[] holds an id outside [0, k)
  int32_t bad_graph;    // set by the validation kernel
  int32_t diag;         // which internal check raised err (DIAG_*)
  int32_t pad2;
};

enum { DIAG_NONE = 0, DIAG_LIST = 1, DIAG_CLOSURE = 2, DIAG_REV = 3, DIAG_SWEEPS = 4 };

struct GridBar {
  uint32_t count;
  uint32_t gen;
  int32_t abort;
  int32_t pad;
};

struct KArgs {
  // graph (device)
  int32_t n, k;
  const int32_t *xadj, *adjncy, *adjwgt, *vwgt;
  int32_t *part;
  // pairs
  int32_t P;
  const int32_t *blk2pair, *blk2side;
  PairState *ps;
  fr_solve *trace;
  const int64_t *base;  // floor((1 + alpha eps) c(V) / k) for alpha = 0..alpha_max
  int64_t lmax;
  // parameters
  int32_t area_mode, depth, alpha_max, adaptive, max_iters, eps_ppm;
  // vertex scratch [n]
  int32_t *mark, *vmap, *f0, *f1;
  // corridor arrays [n] (corridor size <= n)
  int32_t *lglob, *loff, *lpair, *ldeg, *excess, *label, *ins, *fa, *fb, *sinks;
  uint8_t *lflag;
  // corridor arcs [2m]
  int32_t *lhead, *lrev, *rcap;
  // per pair
  int64_t *acc;   // [P][FR_NACC]
  int64_t *lvlw;  // [3][P][2]
  int32_t *lvlc;  // [3][P][2]
  // scan scratch
  int64_t *bsum;  // [nblocks + 1]
  Ctl *ctl;
  GridBar *bar;
  int8_t *side_out;
  // launch
  int32_t tpv, relabel_period;
  int64_t max_sweeps;
  uint64_t spin_limit;  // wall-clock ticks a barrier may wait
};

// corridor vertex flags
#define LF_SIDE_B 1u   // vertex of block b (sink side)
#define LF_BORDER 2u   // has a neighbour in A u B outside the corridor
#define LF_SRC(f) (((f) & 3u) == LF_BORDER)
#define LF_SNK(f) (((f) & 3u) == (LF_BORDER | LF_SIDE_B))
