// libflowrefine: host driver and C ABI (declared in include/flowrefine.h).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <numeric>
#include <random>
#include <vector>

#include "fr_internal.h"
#include "fr_kernels.h"
#include "fr_mb.h"
#include "fr_fm.h"
#include "fr_mlp.h"
#include "fr_mt.h"

#define HIPCHK(x)                        \
  do {                                   \
    hipError_t _e = (x);                 \
    if (_e != hipSuccess) {              \
      last_hip_error = _e;               \
      return FR_E_DEVICE;                \
    }                                    \
  } while (0)

static thread_local hipError_t last_hip_error = hipSuccess;

#define FR_MAX_PAIRS 4096  // pairs of one round (one launch)
#define FR_MAX_K 8192
#define FR_MAX_BLOCKS_PER_CU 8

struct DevBufs {
  int64_t ncap = 0, acap = 0, kcap = 0, pcap = 0;  // graph copies: n, arcs
  int64_t sncap = 0, sacap = 0;                      // arenas and marks: slots * n, slots * arcs
  // per vertex
  int32_t *mark = nullptr, *vmap = nullptr, *uvert = nullptr, *lg = nullptr, *lo = nullptr,
          *ex = nullptr, *lab = nullptr, *ins = nullptr, *LA = nullptr, *LB = nullptr,
          *SNK = nullptr, *partw = nullptr, *parts = nullptr, *gx = nullptr, *gv = nullptr;
  uint8_t *lflag = nullptr;
  int8_t *side = nullptr;
  int32_t *mbq = nullptr;  // most balanced cut: quotient arcs, one per arc slot (lazy)
  int64_t mbqcap = 0;
  // input checks: hub table offsets [n], table keys and weights
  int64_t *vhdir = nullptr;
  int32_t *vkey = nullptr, *vw = nullptr;
  int64_t vhcap = 0, vtcap = 0;
  int32_t *mbc = nullptr;  // most balanced cut: large component graphs, 4 per vertex slot (lazy)
  int64_t mbccap = 0;
  int32_t *fmg = nullptr, *fmq = nullptr;  // 2-way FM: per-vertex gains, queue positions (lazy)
  int64_t fmcap = 0;
  // multi-try FM (lazy): per vertex touched stamps, targets, heap slots, heap
  // overflow [2n], move log [n] x 2; todo keys per arena slot x 2; per block
  // weights and changed flags
  int32_t *mtt = nullptr, *mtb = nullptr, *mtq = nullptr, *mth = nullptr, *mtv = nullptr,
          *mtf = nullptr;
  unsigned long long *mtk = nullptr, *mtk2 = nullptr;
  int64_t *mtw = nullptr;
  uint8_t *mtchg = nullptr;
  int64_t mtncap = 0, mtscap = 0, mtkcap = 0;
  // per arc
  int32_t *ga = nullptr, *gw = nullptr;
  Arc *arc = nullptr;  // corridor arcs
  // per block
  int32_t *blk2pair = nullptr;
  int64_t *bstat = nullptr;  // [3k]
  uint8_t *qadj = nullptr;   // [k*k]
  // per pair of a call (all rounds of a sweep): grows with pcap
  PairState *ps = nullptr;
  int32_t *pairs = nullptr, *alpha0 = nullptr, *order = nullptr;
  // per round (at most FR_MAX_PAIRS pairs)
  fr_solve *trace = nullptr, *srec = nullptr;
  int32_t *ucnt = nullptr, *qctr = nullptr, *pcnt = nullptr, *act = nullptr, *nact = nullptr;
  int64_t *voff = nullptr, *aoff = nullptr, *fstat = nullptr, *pacc = nullptr, *vpre = nullptr,
          *cpre = nullptr, *mpre = nullptr;
  float *feats = nullptr, *probs = nullptr;
  int64_t *base = nullptr, *scal = nullptr;
  Ctl *ctl = nullptr;
  // learned factor: parameters, Adam moments, gradient
  float *mlp = nullptr, *mlp_m = nullptr, *mlp_v = nullptr, *mlp_g = nullptr;
};

struct fr_context {
  int device = 0;
  hipStream_t user_stream = nullptr;
  hipStream_t cs = nullptr;  // the library's own stream (graph capture needs a non-null one)
  int num_cus = 0;
  // grids of the whole-graph passes: every workgroup resident at once (each
  // wave walks one contiguous run of vertex chunks)
  int g_bnd = 0, g_bstat = 0, g_fstat = 0, g_union = 0;
  fr_tuning tune{1024, 2, 8, 100, 1, 8000};
  int validate = 1;
  int mlp_loaded = 0;
  DevBufs d;
  Ctl *h_ctl = nullptr;  // pinned
  int32_t stamp = 2;
  double wall_khz = 100000.0;  // device constant-rate clock
  int64_t graph_launches = 0;
  std::vector<hipEvent_t> itev;  // five per launch of the per-iteration chain (timed calls)
  int32_t timed_iters = 0;
  int speculate = 1;
  int fused = 0;  // rounds as one persistent launch (k_round) where possible
  int timing = 0;  // sweeps: uncaptured rounds with per-phase events
  int32_t mt_stamp = 0;  // multi-try: touched stamps used so far
  // stats of the last call
  double ms[8] = {0};
  int64_t counters[32] = {0};
  hipEvent_t ev[4] = {};
};

static bool verbose() {
  static int v = -1;
  if (v < 0) {
    const char *e = getenv("FR_VERBOSE");
    v = (e && *e && *e != '0') ? 1 : 0;
  }
  return v == 1;
}

static void dfree(void *p) {
  if (p) (void)hipFree(p);
}

template <typename T>
static hipError_t dalloc(T **p, int64_t count) {
  return hipMalloc((void **)p, sizeof(T) * (size_t)(count > 0 ? count : 1));
}

static void free_vertex_arc(DevBufs &d) {
  int32_t **v32[] = {&d.mark, &d.vmap, &d.uvert, &d.lg, &d.lo, &d.ex, &d.lab, &d.ins, &d.LA,
                     &d.LB, &d.SNK, &d.partw, &d.parts, &d.gx, &d.gv,
                     &d.ga, &d.gw};
  for (auto pp : v32) {
    dfree(*pp);
    *pp = nullptr;
  }
  dfree(d.arc);
  d.arc = nullptr;
  dfree(d.mbq);
  d.mbq = nullptr;
  d.mbqcap = 0;
  dfree(d.mbc);
  d.mbc = nullptr;
  d.mbccap = 0;
  dfree(d.fmg);
  dfree(d.fmq);
  d.fmg = d.fmq = nullptr;
  d.fmcap = 0;
  for (int32_t **pp : {&d.mtt, &d.mtb, &d.mtq, &d.mth, &d.mtv, &d.mtf}) {
    dfree(*pp);
    *pp = nullptr;
  }
  dfree(d.mtk);
  dfree(d.mtk2);
  d.mtk = d.mtk2 = nullptr;
  d.mtncap = d.mtscap = 0;
  dfree(d.lflag);
  d.lflag = nullptr;
  dfree(d.side);
  d.side = nullptr;
  d.ncap = d.acap = d.sncap = d.sacap = 0;
}

// Graph-sized buffers (staged copies, partitions, side codes) for n vertices
// and narcs arcs; arena-sized ones (per-entry slices, corridor marks) for
// `slots` entries per vertex and per arc.
static int32_t ensure_capacity(fr_context *c, int64_t n, int64_t narcs, int64_t k,
                               int64_t slots = 1) {
  DevBufs &d = c->d;
  const int64_t sn = slots * n, sa = slots * narcs;
  if (n > d.ncap || narcs > d.acap || sn > d.sncap || sa > d.sacap) {
    const int64_t nc = std::max(n, d.ncap), ac = std::max(narcs, d.acap);
    const int64_t snc = std::max(sn, d.sncap), sac = std::max(sa, d.sacap);
    free_vertex_arc(d);
    hipError_t e = hipSuccess;
#define A_(p, cnt) \
  if (e == hipSuccess) e = dalloc(&d.p, cnt)
    A_(mark, snc); A_(vmap, snc); A_(uvert, snc); A_(lg, snc); A_(lo, snc + FR_MAX_PAIRS + 1);
    A_(ex, snc); A_(lab, snc); A_(ins, snc); A_(LA, snc); A_(LB, snc); A_(SNK, snc);
    A_(lflag, snc); A_(arc, sac);
    A_(partw, nc); A_(parts, nc); A_(gx, nc + 1); A_(gv, nc); A_(side, nc);
    A_(ga, ac); A_(gw, ac);
#undef A_
    if (e != hipSuccess) {
      free_vertex_arc(d);
      return FR_E_OOM;
    }
    if (hipMemset(d.mark, 0, sizeof(int32_t) * (size_t)snc) != hipSuccess) return FR_E_DEVICE;
    d.ncap = nc;
    d.acap = ac;
    d.sncap = snc;
    d.sacap = sac;
    c->stamp = 2;
  }
  if (k > d.kcap) {
    dfree(d.blk2pair); dfree(d.bstat); dfree(d.qadj); dfree(d.mtw); dfree(d.mtchg);
    d.blk2pair = nullptr;
    d.bstat = nullptr;
    d.qadj = nullptr;
    d.mtw = nullptr;
    d.mtchg = nullptr;
    d.mtkcap = 0;
    if (dalloc(&d.blk2pair, 3 * k) != hipSuccess || dalloc(&d.bstat, 3 * k) != hipSuccess ||
        dalloc(&d.qadj, k * k) != hipSuccess)
      return FR_E_OOM;
    d.kcap = k;
  }
  return FR_OK;
}

static int32_t ensure_pairs(fr_context *c, int64_t npairs) {
  DevBufs &d = c->d;
  if (npairs <= d.pcap) return FR_OK;
  const int64_t pc = std::max<int64_t>(npairs, 2 * d.pcap);
  dfree(d.ps); dfree(d.pairs); dfree(d.alpha0); dfree(d.order);
  d.ps = nullptr;
  d.pairs = d.alpha0 = d.order = nullptr;
  if (dalloc(&d.ps, pc) != hipSuccess || dalloc(&d.pairs, 2 * pc) != hipSuccess ||
      dalloc(&d.alpha0, pc) != hipSuccess || dalloc(&d.order, pc) != hipSuccess)
    return FR_E_OOM;
  d.pcap = pc;
  return FR_OK;
}

// Corridor marks are compared against a stamp that grows by 2 per solve;
// clear them well before int32 wraps.
static int32_t reserve_stamps(fr_context *c, int64_t count, int32_t *first) {
  if ((int64_t)c->stamp + 2 * count + 4 > (1 << 30)) {
    HIPCHK(hipMemsetAsync(c->d.mark, 0, sizeof(int32_t) * (size_t)c->d.sncap, c->cs));
    c->stamp = 2;
  }
  *first = c->stamp;
  c->stamp += (int32_t)(2 * count + 2);
  return FR_OK;
}

// ---- device scratch of flow_refine_pair_static (callers that cannot
// allocate): one array per GPU, resolved once per device by fr_create.  In
// host code the array's name is only a stand-in; kernels get the address
// from scratch_ptr.
#define FR_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
#define FR_MAX_DEVICES 64
static __device__ __align__(256) unsigned char scratch[FR_STATIC_SCRATCH_BYTES];
static void *scratch_ptr[FR_MAX_DEVICES];
static std::mutex scratch_mu;

// With `device` current: its copy of the scratch array.
static int32_t scratch_address(int device) {
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (device < 0 || device >= FR_MAX_DEVICES) return FR_E_DEVICE;
  if (scratch_ptr[device]) return FR_OK;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    last_hip_error = e;
    return FR_E_DEVICE;
  }
  scratch_ptr[device] = ptr;
  return FR_OK;
}

// Multi-try touched stamps: count rounds of pairs need count + 1 stamps;
// the stamp array is cleared well before int32 wraps.
static int32_t reserve_mt(fr_context *c, int64_t count, int32_t *first) {
  if ((int64_t)c->mt_stamp + count + 2 > (1 << 30)) {
    HIPCHK(hipMemsetAsync(c->d.mtt, 0, sizeof(int32_t) * (size_t)c->d.mtncap, c->cs));
    c->mt_stamp = 0;
  }
  *first = c->mt_stamp;
  c->mt_stamp += (int32_t)(count + 1);
  return FR_OK;
}

extern "C" const char *fr_strerror(int32_t code) {
  switch (code) {
    case FR_OK: return "ok";
    case FR_E_INVALID_GRAPH: return "invalid graph";
    case FR_E_INVALID_PART: return "invalid partition";
    case FR_E_INVALID_PAIR: return "invalid block pair";
    case FR_E_PAIRS_NOT_DISJOINT: return "pairs of a batch share a block";
    case FR_E_OVERFLOW: return "capacity overflow";
    case FR_E_DEVICE: return "HIP device error";
    case FR_E_OOM: return "out of memory";
    case FR_E_INVALID_ARG: return "invalid argument";
    case FR_E_SOLVER_LIMIT: return "push/relabel sweep limit or round launch limit reached";
    case FR_E_SCRATCH_LIMIT: return "graph too large for the static scratch of flow_refine_pair_static";
    default: return "unknown error";
  }
}

extern "C" int32_t fr_create(int32_t device, void *hip_stream, fr_context **out) {
  if (!out) return FR_E_INVALID_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return FR_E_DEVICE;
  if (hipSetDevice(device) != hipSuccess) return FR_E_DEVICE;
  if (scratch_address(device) != FR_OK) return FR_E_DEVICE;
  fr_context *c = new (std::nothrow) fr_context();
  if (!c) return FR_E_OOM;
  c->device = device;
  c->user_stream = (hipStream_t)hip_stream;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
    delete c;
    return FR_E_DEVICE;
  }
  c->num_cus = prop.multiProcessorCount;
  {
    auto resident = [&](const void *fn) {
      int nb = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, 256, 0) != hipSuccess || nb < 1)
        nb = 4;
      return std::min(nb * c->num_cus, 8192);
    };
    c->g_bnd = resident((const void *)k_bnd);
    c->g_bstat = resident((const void *)k_block_stats);
    c->g_fstat = resident((const void *)k_feature_stats);
    c->g_union = resident((const void *)k_union);
  }
  int rate = 0;
  if (hipDeviceGetAttribute(&rate, hipDeviceAttributeWallClockRate, device) == hipSuccess && rate > 0)
    c->wall_khz = rate;
  DevBufs &d = c->d;
  hipError_t e = hipStreamCreateWithFlags(&c->cs, hipStreamNonBlocking);
#define A_(p, cnt) \
  if (e == hipSuccess) e = dalloc(&d.p, cnt)
  A_(trace, (int64_t)FR_MAX_PAIRS * FR_MAX_ITERS); A_(ucnt, FR_MAX_PAIRS);
  A_(qctr, 4 * FR_MAX_ITERS); A_(pcnt, 2 * FR_MAX_PAIRS); A_(pacc, (int64_t)PA_N * FR_MAX_PAIRS);
  A_(act, FR_MAX_PAIRS); A_(nact, 1); A_(vpre, FR_MAX_PAIRS + 1); A_(cpre, FR_MAX_PAIRS + 1);
  A_(mpre, FR_MAX_PAIRS + 1);
  A_(srec, FR_MAX_PAIRS);
  A_(voff, FR_MAX_PAIRS + 1); A_(aoff, FR_MAX_PAIRS + 1); A_(fstat, 4 * FR_MAX_PAIRS);
  A_(feats, MLP_IN * FR_MAX_PAIRS); A_(probs, MLP_OUT * FR_MAX_PAIRS);
  A_(base, FR_MAX_ALPHA + 1); A_(scal, 8); A_(ctl, 1);
  A_(mlp, MLP_NPARAMS); A_(mlp_m, MLP_NPARAMS); A_(mlp_v, MLP_NPARAMS); A_(mlp_g, MLP_NPARAMS);
#undef A_
  if (e == hipSuccess) e = hipHostMalloc((void **)&c->h_ctl, sizeof(Ctl), hipHostMallocDefault);
  for (int i = 0; i < 4 && e == hipSuccess; i++) e = hipEventCreate(&c->ev[i]);
  c->itev.assign(5 * FR_MAX_ITERS, nullptr);
  for (size_t i = 0; i < c->itev.size() && e == hipSuccess; i++) e = hipEventCreate(&c->itev[i]);
  if (e != hipSuccess) {
    fr_destroy(c);
    return FR_E_OOM;
  }
  if (ensure_pairs(c, FR_MAX_PAIRS) != FR_OK) {
    fr_destroy(c);
    return FR_E_OOM;
  }
  *out = c;
  return FR_OK;
}

extern "C" int32_t fr_destroy(fr_context *c) {
  if (!c) return FR_E_INVALID_ARG;
  (void)hipSetDevice(c->device);
  if (c->cs) (void)hipStreamSynchronize(c->cs);
  free_vertex_arc(c->d);
  DevBufs &d = c->d;
  void *ptrs[] = {d.mtw,      d.mtchg, d.vhdir, d.vkey, d.vw,
                  d.blk2pair, d.bstat, d.qadj, d.ps,    d.pairs, d.alpha0, d.order,
                  d.trace,    d.ucnt,  d.voff, d.aoff,  d.fstat, d.feats,  d.probs,
                  d.base,     d.scal,  d.ctl,  d.mlp,   d.mlp_m, d.mlp_v,  d.mlp_g,
                  d.qctr,     d.pcnt,  d.pacc, d.act,   d.nact,  d.vpre,   d.cpre, d.mpre,
                  d.srec};
  for (void *q : ptrs) dfree(q);
  if (c->h_ctl) (void)hipHostFree(c->h_ctl);
  for (int i = 0; i < 4; i++)
    if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
  for (hipEvent_t ev : c->itev)
    if (ev) (void)hipEventDestroy(ev);
  if (c->cs) (void)hipStreamDestroy(c->cs);
  delete c;
  return FR_OK;
}

extern "C" int32_t fr_set_tuning(fr_context *c, const fr_tuning *t) {
  if (!c || !t) return FR_E_INVALID_ARG;
  const int bt = t->block_threads;
  if (!(bt == 256 || bt == 512 || bt == 1024)) return FR_E_INVALID_ARG;
  if (t->blocks_per_cu < 1 || t->blocks_per_cu > FR_MAX_BLOCKS_PER_CU) return FR_E_INVALID_ARG;
  if (!(t->tpv == 1 || t->tpv == 2 || t->tpv == 4 || t->tpv == 8 || t->tpv == 16))
    return FR_E_INVALID_ARG;
  if (t->relabel_period < 1 || t->relabel_period > 1000000) return FR_E_INVALID_ARG;
  if (t->mb_lds != 0 && t->mb_lds != 1) return FR_E_INVALID_ARG;
  if (t->slice_us < 0 || t->slice_us > 10000000) return FR_E_INVALID_ARG;
  c->tune = *t;
  return FR_OK;
}

extern "C" int32_t fr_get_tuning(fr_context *c, fr_tuning *t) {
  if (!c || !t) return FR_E_INVALID_ARG;
  *t = c->tune;
  return FR_OK;
}

extern "C" int32_t fr_set_speculation(fr_context *c, int32_t on) {
  if (!c) return FR_E_INVALID_ARG;
  c->speculate = on ? 1 : 0;
  return FR_OK;
}

extern "C" int32_t fr_set_fused(fr_context *c, int32_t on) {
  if (!c) return FR_E_INVALID_ARG;
  c->fused = on ? 1 : 0;
  return FR_OK;
}

extern "C" int32_t fr_set_timing(fr_context *c, int32_t on) {
  if (!c) return FR_E_INVALID_ARG;
  c->timing = on ? 1 : 0;
  return FR_OK;
}

extern "C" int32_t fr_set_validation(fr_context *c, int32_t on) {
  if (!c) return FR_E_INVALID_ARG;
  c->validate = on ? 1 : 0;
  return FR_OK;
}

extern "C" int32_t fr_last_stats(fr_context *c, double *ms, int64_t *counters) {
  if (!c) return FR_E_INVALID_ARG;
  if (ms) memcpy(ms, c->ms, sizeof(c->ms));
  if (counters) memcpy(counters, c->counters, sizeof(c->counters));
  return FR_OK;
}

// ---------------------------------------------------------------------------

static int64_t floor_div_u128(unsigned __int128 num, unsigned __int128 den) {
  return (int64_t)(num / den);
}

static int32_t check_params(const fr_params *p) {
  if (!p) return FR_E_INVALID_ARG;
  if (p->area_mode != FR_AREA_FACTOR && p->area_mode != FR_AREA_DEPTH) return FR_E_INVALID_ARG;
  if (p->depth < 0 || p->alpha < 1 || p->alpha_max < 1 || p->alpha_max > FR_MAX_ALPHA ||
      p->max_iters < 1 || p->max_iters > FR_MAX_ITERS || p->eps_ppm < 0 || p->eps_ppm > 100000000 ||
      p->mb_reps < 0 || p->mb_reps > FR_MB_MAX_REPS || p->fm_limit < 0 || p->cut_side < 0 ||
      p->cut_side > 2 || (p->terminals != FR_TERM_PINNED && p->terminals != FR_TERM_CONTRACTED) ||
      p->mt_alpha < 0 || (p->mlp_restart != 0 && p->mlp_restart != 1))
    return FR_E_INVALID_ARG;
  return FR_OK;
}

typedef void (*iter_fn)(KArgs, int32_t);

static iter_fn corr_kernel(int tpb) {
  switch (tpb) {
    case 256: return k_corr<256>;
    case 512: return k_corr<512>;
    default: return k_corr<1024>;
  }
}

static iter_fn flow_kernel(int tpb) {
  switch (tpb) {
    case 256: return k_flow<256>;
    case 512: return k_flow<512>;
    default: return k_flow<1024>;
  }
}

typedef void (*round_fn)(KArgs);

static round_fn round_kernel(int tpb) {
  switch (tpb) {
    case 256: return k_round<256>;
    case 512: return k_round<512>;
    default: return k_round<1024>;
  }
}

// Rounds of these parameters run as one launch (k_round): one entry per
// pair, and no most balanced cut (its kernels run between the flow and the
// adaptive rule of every iteration).
static bool fused_rounds(const fr_context *c, const fr_params *p) {
  return c->fused && p->mb_reps == 0;
}

static int32_t graph_narcs(fr_context *c, const fr_graph *g, int64_t *narcs) {
  int32_t na = 0;
  if (g->on_device) {
    HIPCHK(hipMemcpyAsync(&na, g->xadj + g->n, sizeof(int32_t), hipMemcpyDeviceToHost, c->cs));
    HIPCHK(hipStreamSynchronize(c->cs));
  } else {
    na = g->xadj[g->n];
  }
  if (na < 0) return FR_E_INVALID_GRAPH;
  *narcs = na;
  return FR_OK;
}

// Kernel arguments common to every round of a call: graph, partition,
// parameters, scratch.  Per-round fields are set by round_args.
static KArgs call_args(fr_context *c, const DevBufs &d, const fr_graph *g, int32_t *dpart,
                       int32_t k, const fr_params *p) {
  KArgs A;
  memset(&A, 0, sizeof(A));
  A.n = g->n;
  A.k = k;
  A.xadj = g->xadj;
  A.adjncy = g->adjncy;
  A.adjwgt = g->adjwgt;
  A.vwgt = g->vwgt;
  A.part = dpart;
  A.blk2pair = d.blk2pair;
  A.binfo = d.blk2pair + k;  // the same allocation: [k] then [2k]
  A.bstat = d.bstat;
  A.queue = d.qctr;
  A.pacc = d.pacc;
  A.pcnt = d.pcnt;
  A.act = d.act;
  A.W = 1;
  A.mstride = 0;
  A.srec = d.srec;
  A.nact = d.nact;
  A.vpre = d.vpre;
  A.cpre = d.cpre;
  A.mpre = d.mpre;
  A.base = d.base;
  if (p) {
    A.area_mode = p->area_mode;
    A.depth = p->depth;
    A.alpha_max = p->alpha_max;
    A.restart_alpha = p->use_mlp && p->mlp_restart ? std::min(p->alpha, p->alpha_max) : 0;
    A.adaptive = p->adaptive;
    A.max_iters = p->max_iters;
    A.eps_ppm = p->eps_ppm;
    A.mb_reps = p->mb_reps;
    A.mb_seed = p->mb_seed;
    A.fm_limit = p->fm_limit;
    A.fm_seed = p->fm_seed;
    A.cut_side = p->cut_side;
    A.terminals = p->terminals;
  }
  A.mb_lds = c->tune.mb_lds;
  if (p && p->mt_alpha > 0) {
    A.mt_alpha = p->mt_alpha;
    A.mt_seed = p->mt_seed;
    A.mt_beta = (int64_t)std::floor(std::log((double)g->n) * 65536.0);
    A.mtw = d.mtw;
    A.mtk = d.mtk;
    A.mtk2 = d.mtk2;
    A.mtt = d.mtt;
    A.mtb = d.mtb;
    A.mtq = d.mtq;
    A.mth = d.mth;
    A.mtv = d.mtv;
    A.mtf = d.mtf;
    A.mtchg = d.mtchg;
  }
  A.mbq = d.mbq;
  A.mbc = d.mbc;
  A.fmg = d.fmg;
  A.fmq = d.fmq;
  A.mark = d.mark;
  A.vmap = d.vmap;
  A.voff = d.voff;
  A.aoff = d.aoff;
  A.ucnt = d.ucnt;
  A.uvert = d.uvert;
  A.lg = d.lg;
  A.lo = d.lo;
  A.ex = d.ex;
  A.lab = d.lab;
  A.ins = d.ins;
  A.LA = d.LA;
  A.LB = d.LB;
  A.SNK = d.SNK;
  A.lflag = d.lflag;
  A.arc = d.arc;
  A.ctl = d.ctl;
  A.tpv = c->tune.tpv;
  A.relabel_period = c->tune.relabel_period;
  A.slice_ticks = (int64_t)((double)c->tune.slice_us * c->wall_khz / 1000.0);
  A.max_sweeps = 4 * ((int64_t)g->n + 16) + 1000000;
  A.side_out = d.side;
  return A;
}

// Per-call constants: input checks, c(V), max c(v), L_max and the area
// bases floor((1 + alpha eps) c(V) / k) for alpha = 0..alpha_max (exact, in
// 128-bit arithmetic on the host).  One host synchronisation.
// Sets n int32 words to v on the stream (a kernel, not a memset node, so the
// work stays correct inside captured graphs).
__global__ void __launch_bounds__(256) k_fill32(int32_t *x, int64_t n, int32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = v;
}

// Input checks (k_validate).  With may_alloc, vertices of more than
// FR_VAL_HUB arcs get hash tables of their neighbours first (device buffers
// grown on demand); without it (the entry point that allocates nothing)
// their lists are scanned instead.
static int32_t validate_graph(fr_context *c, const KArgs &A, int64_t narcs, bool may_alloc) {
  DevBufs &d = c->d;
  hipStream_t st = c->cs;
  const int sblocks = std::min(4 * c->num_cus, 8192);
  const int64_t *hdir = nullptr;
  const int32_t *tkey = nullptr, *tw = nullptr;
  if (may_alloc) {
    unsigned long long *ctr = (unsigned long long *)(d.scal + 2);
    HIPCHK(hipMemsetAsync(ctr, 0, 2 * sizeof(unsigned long long), st));
    hipLaunchKernelGGL(k_val_hub_size, dim3(sblocks), dim3(256), 0, st, A, narcs, ctr);
    HIPCHK(hipGetLastError());
    int64_t slots = 0;
    HIPCHK(hipMemcpyAsync(&slots, ctr, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (slots > 0) {
      if (d.vhcap < A.n) {
        dfree(d.vhdir);
        d.vhdir = nullptr;
        d.vhcap = 0;
        if (dalloc(&d.vhdir, A.n) != hipSuccess) return FR_E_OOM;
        d.vhcap = A.n;
      }
      if (d.vtcap < slots) {
        dfree(d.vkey);
        dfree(d.vw);
        d.vkey = d.vw = nullptr;
        d.vtcap = 0;
        if (dalloc(&d.vkey, slots) != hipSuccess || dalloc(&d.vw, slots) != hipSuccess)
          return FR_E_OOM;
        d.vtcap = slots;
      }
      hipLaunchKernelGGL(k_fill32, dim3(std::min<int64_t>((slots + 255) / 256, 4 * c->num_cus)),
                         dim3(256), 0, st, d.vkey, slots, -1);
      hipLaunchKernelGGL(k_val_hub_alloc, dim3(sblocks), dim3(256), 0, st, A, narcs, d.vhdir, ctr);
      hipLaunchKernelGGL(k_val_hub_insert, dim3(sblocks), dim3(256), 0, st, A,
                         (const int64_t *)d.vhdir, d.vkey, d.vw);
      HIPCHK(hipGetLastError());
      hdir = d.vhdir;
      tkey = d.vkey;
      tw = d.vw;
    }
  }
  hipLaunchKernelGGL(k_validate, dim3(sblocks), dim3(256), 0, st, A, narcs, hdir, tkey, tw);
  HIPCHK(hipGetLastError());
  return FR_OK;
}

static int32_t call_constants(fr_context *c, KArgs &A, int64_t narcs, const fr_params *p,
                              bool may_alloc = true) {
  DevBufs &d = c->d;
  hipStream_t st = c->cs;
  memset(c->h_ctl, 0, sizeof(Ctl));
  HIPCHK(hipMemcpyAsync(d.ctl, c->h_ctl, sizeof(Ctl), hipMemcpyHostToDevice, st));
  const int sblocks = std::min(4 * c->num_cus, 8192);
  if (c->validate) {
    int32_t rc = validate_graph(c, A, narcs, may_alloc);
    if (rc) return rc;
  }
  hipLaunchKernelGGL(k_graph_stats, dim3(sblocks), dim3(256), 0, st, A);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(c->h_ctl, d.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (c->h_ctl->bad_graph) return FR_E_INVALID_GRAPH;
  if (c->h_ctl->bad_part) return FR_E_INVALID_PART;
  const int64_t cV = c->h_ctl->cV, maxc = c->h_ctl->maxc;
  const unsigned __int128 den = (unsigned __int128)1000000 * (unsigned)A.k;
  // L_max = (1 + eps) c(V) / k + max c(v)  (Sec. 2.1)
  A.lmax = floor_div_u128((unsigned __int128)(1000000 + (int64_t)p->eps_ppm) * (uint64_t)cV, den) +
           maxc;
  int64_t base[FR_MAX_ALPHA + 1];
  const int nb = std::max(p->alpha_max, 1) + 1;
  for (int al = 0; al < nb; al++)
    base[al] = floor_div_u128(
        (unsigned __int128)(1000000 + (int64_t)al * p->eps_ppm) * (uint64_t)cV, den);
  HIPCHK(hipMemcpyAsync(d.base, base, sizeof(int64_t) * nb, hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  return FR_OK;
}

// Per-round view: pairs [off, off + P) of the call's pair arrays.
static KArgs round_args(fr_context *c, const KArgs &base, int64_t off, int32_t P, int32_t stamp0,
                        bool with_trace) {
  DevBufs &d = c->d;
  KArgs A = base;
  A.P = P;
  A.pairs = d.pairs + 2 * off;
  A.alpha0 = d.alpha0 + off;
  A.order = d.order + off;
  A.ps = d.ps + off;
  A.trace = with_trace ? d.trace : nullptr;
  A.stamp0 = stamp0;
  return A;
}

// workgroups of the per-pair kernels for a round of P entries
static int blocks_of(const fr_context *c, int32_t P) {
  const int64_t slots = (int64_t)c->num_cus * c->tune.blocks_per_cu;
  return (int)std::max<int64_t>(1, std::min<int64_t>(P, slots));
}

// All kernels of one matching round: setup kernels, then the launches of
// the per-iteration chain (pairs that stopped are skipped inside).  With
// captured set, device-only work (max_iters launches, no host read-back),
// so a sequence of rounds can be captured into a graph; otherwise the host
// ends the chain once no pair iterates and may slice long solves.  With
// timed set, events around the phases of each launch give the per-phase
// times.
static int32_t enqueue_round(fr_context *c, KArgs A, bool use_mlp, hipStream_t st, bool timed,
                             bool captured) {
  DevBufs &d = c->d;
  const int sblocks = std::min(4 * c->num_cus, 8192);
  A.fstat = use_mlp ? d.fstat : nullptr;
  hipLaunchKernelGGL(k_round_init, dim3(1), dim3(1024), 0, st, A);
  hipLaunchKernelGGL(k_block_stats, dim3(c->g_bstat), dim3(256), 0, st, A);
  if (use_mlp) {
    hipLaunchKernelGGL(k_feature_stats, dim3(c->g_fstat), dim3(256), 0, st, A, d.fstat);
    hipLaunchKernelGGL(k_features, dim3((A.P + 255) / 256), dim3(256), 0, st, A,
                       (const int64_t *)d.fstat, d.feats);
    hipLaunchKernelGGL(k_mlp_forward,
                       dim3((A.P + MLP_SAMPLES_PER_BLOCK - 1) / MLP_SAMPLES_PER_BLOCK), dim3(1024),
                       0, st, (const float *)d.mlp, (const float *)d.feats, A.P, d.probs,
                       (float *)nullptr);
    hipLaunchKernelGGL(k_alpha_from_probs, dim3((A.P + 255) / 256), dim3(256), 0, st,
                       (const float *)d.probs, A.P, A.alpha0);
  }
  hipLaunchKernelGGL(k_arena, dim3(1), dim3(1024), 0, st, A);
  hipLaunchKernelGGL(k_union, dim3(c->g_union), dim3(256), 0, st, A);
  // pairwise FM before the flow iterations: gains grid-wide, then one
  // workgroup per pair
  if (A.fm_limit > 0) {
    hipLaunchKernelGGL(k_fm_gain, dim3(sblocks), dim3(256), 0, st, A);
    hipLaunchKernelGGL(k_fm, dim3(A.P / A.W), dim3(FM_TPB), 0, st, A);
  }
  const int tpb = c->tune.block_threads;
  const int blocks = blocks_of(c, A.P);
  const iter_fn corr = corr_kernel(tpb), flow = flow_kernel(tpb);
  const bool fused = c->fused && A.mb_reps == 0 && A.W == 1;
  // sliced rounds need the host between launches (how many follow is read
  // back), so a captured round passes slice_ticks = 0; a round of one pair
  // has no other pair to wait for
  const bool sliced = A.slice_ticks > 0 && !fused && A.mb_reps == 0 && A.P / A.W > 1;
  if (!sliced) A.slice_ticks = 0;
  if (fused) {
    // every pair's whole adaptive loop in one launch; the events put its
    // time in the flow-kernel slot
    hipEvent_t *ev = c->itev.data();
    if (timed)
      for (int j = 0; j < 3; j++) HIPCHK(hipEventRecord(ev[j], st));
    hipLaunchKernelGGL(round_kernel(tpb), dim3(blocks), dim3(tpb), 0, st, A);
    if (timed)
      for (int j = 3; j < 5; j++) HIPCHK(hipEventRecord(ev[j], st));
  }
  // launches of the per-iteration chain.  Unsliced, each is one adaptive
  // iteration of every pair still iterating, at most max_iters of them; a
  // captured round runs all max_iters (a stopped pair skips the rest).  Not
  // captured, the host reads the number of entries still iterating back
  // after 2, 4 and 8 launches and then every 4, and the chain ends at 0;
  // sliced, a pair's iteration may span launches, so it may run past
  // max_iters.
  const bool host = !captured && !fused;
  int32_t launches = fused ? 0 : (host ? std::min(2, A.max_iters) : A.max_iters);
  // a backstop only: every slice but a solve's last makes at least one sweep,
  // so the solves' sweep cap already bounds the chain
  const int32_t max_launches = std::max(256 * A.max_iters, 1 << 16);
  for (int32_t it = 0;; it++) {
    if (it >= launches) {
      if (!host || (!sliced && it >= A.max_iters)) break;
      hipLaunchKernelGGL(k_live, dim3(1), dim3(1024), 0, st, A);
      HIPCHK(hipMemcpyAsync(&c->h_ctl->live, &c->d.ctl->live, sizeof(int32_t),
                            hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      if (c->h_ctl->live == 0) break;
      if (it >= max_launches) {
        c->timed_iters = timed ? it : 0;
        return FR_E_SOLVER_LIMIT;
      }
      launches = it < 8 ? 2 * it : it + 4;
      if (!sliced) launches = std::min(launches, A.max_iters);
    }
    if (timed && (size_t)(5 * it + 5) > c->itev.size()) {
      const size_t n0 = c->itev.size();
      c->itev.resize(n0 + 5 * FR_MAX_ITERS, nullptr);
      for (size_t i = n0; i < c->itev.size(); i++) HIPCHK(hipEventCreate(&c->itev[i]));
    }
    hipEvent_t *ev = timed ? c->itev.data() + 5 * it : nullptr;
    if (timed) HIPCHK(hipEventRecord(ev[0], st));
    hipLaunchKernelGGL(k_iter_begin, dim3(1), dim3(1024), 0, st, A, it);
    hipLaunchKernelGGL(k_bnd, dim3(c->g_bnd), dim3(256), 0, st, A, it);
    hipLaunchKernelGGL(corr, dim3(blocks), dim3(tpb), 0, st, A, it);
    hipLaunchKernelGGL(k_iter_mid, dim3(1), dim3(1024), 0, st, A, it);
    if (timed) HIPCHK(hipEventRecord(ev[1], st));
    hipLaunchKernelGGL(k_net_count, dim3(sblocks), dim3(256), 0, st, A, it);
    hipLaunchKernelGGL(k_net_scan, dim3(A.P), dim3(1024), 0, st, A, it);
    hipLaunchKernelGGL(k_net_fill, dim3(sblocks), dim3(256), 0, st, A, it);
    hipLaunchKernelGGL(k_net_rev, dim3(sblocks), dim3(256), 0, st, A, it);
    if (timed) HIPCHK(hipEventRecord(ev[2], st));
    hipLaunchKernelGGL(flow, dim3(blocks), dim3(tpb), 0, st, A, it);
    if (timed) HIPCHK(hipEventRecord(ev[3], st));
    if (A.mb_reps > 0) {
      hipLaunchKernelGGL(k_mb_scan, dim3(1), dim3(1024), 0, st, A, it);
      hipLaunchKernelGGL(k_mb_union, dim3(sblocks), dim3(256), 0, st, A, it);
      hipLaunchKernelGGL(k_mb, dim3(A.P), dim3(MB_TPB), 0, st, A, it);
    }
    if (timed) HIPCHK(hipEventRecord(ev[4], st));
    hipLaunchKernelGGL(k_select, dim3(A.P / A.W), dim3(1024), 0, st, A, it);
  }
  // multi-try FM (Sec. 4.2) after the pairwise improvements of the round
  if (A.mt_alpha > 0) {
    hipLaunchKernelGGL(k_mt_clear, dim3(1), dim3(1024), 0, st, A);
    hipLaunchKernelGGL(k_mt_weights, dim3(sblocks), dim3(256), 0, st, A);
    hipLaunchKernelGGL(k_mt_todo, dim3(sblocks), dim3(256), 0, st, A);
    hipLaunchKernelGGL(k_mt_sort, dim3(A.P / A.W), dim3(MT_SORT_TPB), 0, st, A);
    hipLaunchKernelGGL(k_mt, dim3(1), dim3(WAVE), 0, st, A);
  }
  HIPCHK(hipGetLastError());
  c->timed_iters = timed ? (fused ? 1 : launches) : 0;
  return FR_OK;
}

// per-phase event times of the last timed round: corridor, build, flow
// kernel, most balanced cut kernel
static void iteration_times(fr_context *c, double out[4]) {
  out[0] = out[1] = out[2] = out[3] = 0.0;
  for (int it = 0; it < c->timed_iters; it++) {
    float t = 0.f;
    hipEvent_t *ev = c->itev.data() + 5 * it;
    for (int j = 0; j < 4; j++)
      if (hipEventElapsedTime(&t, ev[j], ev[j + 1]) == hipSuccess) out[j] += t;
  }
}

static void fill_result(const PairState &s, fr_result &r) {
  memset(&r, 0, sizeof(r));
  r.iters = s.iters;
  r.final_alpha = s.final_alpha;
  r.start_alpha = s.start_alpha;
  r.applied = s.applied;
  r.iter_cap = s.iter_cap;
  r.flow_value = s.flow_last;
  r.cut_before = s.cut0;
  r.cut_after = s.cut;
  r.weight_a = s.cA;
  r.weight_b = s.cB;
  r.region_vertices = s.rv_sum;
  r.region_edges = s.re_sum;
  r.mt_kept = s.mt_kept;
  if (s.applied > 0) r.status = FR_ACCEPTED;
  else if (s.last_dec == FR_DEC_NOT_ADJACENT) r.status = FR_NOT_ADJACENT;
  else if (s.fm_kept > 0) r.status = FR_ACCEPTED;  // FM moved vertices, the flow did not
  else if (s.last_dec == FR_DEC_INFEASIBLE) r.status = FR_REJECTED_IMBALANCE;
  else r.status = FR_NO_IMPROVEMENT;
}

// Statistics of a call (fr_last_stats): cleared at its start, then every
// round adds its entries' work counters and, when its iterations were timed,
// the per-phase event times.
static void reset_stats(fr_context *c) {
  memset(c->ms, 0, sizeof(c->ms));
  memset(c->counters, 0, sizeof(c->counters));
}

static void add_entry_stats(fr_context *c, const PairState *ps, size_t count) {
  int64_t *C = c->counters;
  double ph[3] = {0, 0, 0};
  for (size_t i = 0; i < count; i++) {
    const PairState &s = ps[i];
    C[0] += s.sweeps;
    C[1] += s.relabels;
    C[2] += s.bfs_levels;
    C[3] += s.gr_levels;
    C[4] += s.cl_levels;
    for (int j = 0; j < W_COUNT; j++) C[16 + j] += s.work[j];
    C[9] += s.mb_free;
    C[10] += s.mb_comp;
    C[11] += s.mb_big;
    C[12] += s.fm_steps;
    C[13] += s.fm_kept;
    C[15] += s.restarted;
    C[31] += s.slices;
    C[28] += s.mt_searches;
    C[29] += s.mt_moves;
    C[30] += s.mt_kept;
    ph[0] += s.t_relabel;
    ph[1] += s.t_push;
  }
  c->ms[5] += ph[0] / c->wall_khz;
  c->ms[6] += ph[1] / c->wall_khz;
}

// the timed iterations of the round just enqueued (after the stream
// synchronised): corridor, build, flow kernel, most balanced cut kernels
static void add_round_times(fr_context *c) {
  double ev[4];
  iteration_times(c, ev);
  c->ms[2] += ev[0];
  c->ms[3] += ev[1];
  c->ms[7] += ev[2];
  c->counters[8] += (int64_t)(ev[3] * 1e6);
  c->counters[14] += c->timed_iters;
}

static int32_t device_error(fr_context *c) {
  HIPCHK(hipMemcpyAsync(c->h_ctl, c->d.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->cs));
  HIPCHK(hipStreamSynchronize(c->cs));
  if (c->h_ctl->err) {
    c->counters[6] = c->h_ctl->diag;
    if (verbose())
      fprintf(stderr, "flowrefine: device error %d (check %d)\n", c->h_ctl->err, c->h_ctl->diag);
    return c->h_ctl->err;
  }
  return FR_OK;
}

// Stage a host graph (and partition) on the device when needed.
struct Staged {
  fr_graph g;
  int32_t *dpart;
  int64_t narcs;
};

// slots: arena and mark arrays for that many entries per vertex / arc
static int32_t stage(fr_context *c, const fr_graph *g, int32_t *part, int32_t k, Staged *s,
                     int32_t slots = 1) {
  int64_t narcs = 0;
  int32_t rc = graph_narcs(c, g, &narcs);
  if (rc) return rc;
  if ((rc = ensure_capacity(c, g->n, narcs, k, slots))) return rc;
  DevBufs &d = c->d;
  hipStream_t st = c->cs;
  s->g = *g;
  s->narcs = narcs;
  s->dpart = part;
  if (!g->on_device) {
    const int64_t n = g->n;
    HIPCHK(hipMemcpyAsync(d.gx, g->xadj, sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d.ga, g->adjncy, sizeof(int32_t) * narcs, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d.gw, g->adjwgt, sizeof(int32_t) * narcs, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d.gv, g->vwgt, sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d.parts, part, sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
    s->g.xadj = d.gx;
    s->g.adjncy = d.ga;
    s->g.adjwgt = d.gw;
    s->g.vwgt = d.gv;
    s->g.on_device = 1;
    s->dpart = d.parts;
  }
  return FR_OK;
}

// Quotient-arc slots of the most balanced cut (one per arena arc slot) and
// the component graphs too large for LDS (four words per arena vertex slot),
// allocated on first use.
static int32_t ensure_mb(fr_context *c, const fr_params *p) {
  DevBufs &d = c->d;
  if (p->fm_limit > 0 && d.fmcap < d.ncap) {  // FM: gains and queue positions per vertex
    dfree(d.fmg);
    dfree(d.fmq);
    d.fmg = d.fmq = nullptr;
    d.fmcap = 0;
    if (dalloc(&d.fmg, d.ncap) != hipSuccess || dalloc(&d.fmq, d.ncap) != hipSuccess)
      return FR_E_OOM;
    d.fmcap = d.ncap;
  }
  if (p->mt_alpha > 0) {  // multi-try FM
    if (d.mtncap < d.ncap) {
      for (int32_t **pp : {&d.mtt, &d.mtb, &d.mtq, &d.mth, &d.mtv, &d.mtf}) {
        dfree(*pp);
        *pp = nullptr;
      }
      d.mtncap = 0;
      if (dalloc(&d.mtt, d.ncap) != hipSuccess || dalloc(&d.mtb, d.ncap) != hipSuccess ||
          dalloc(&d.mtq, d.ncap) != hipSuccess || dalloc(&d.mth, 2 * d.ncap) != hipSuccess ||
          dalloc(&d.mtv, d.ncap) != hipSuccess || dalloc(&d.mtf, d.ncap) != hipSuccess)
        return FR_E_OOM;
      // touched stamps start below every stamp in use, heap slots at -1
      HIPCHK(hipMemset(d.mtt, 0, sizeof(int32_t) * (size_t)d.ncap));
      HIPCHK(hipMemset(d.mtq, 0xff, sizeof(int32_t) * (size_t)d.ncap));
      d.mtncap = d.ncap;
      c->mt_stamp = 0;
    }
    if (d.mtscap < d.sncap) {
      dfree(d.mtk);
      dfree(d.mtk2);
      d.mtk = d.mtk2 = nullptr;
      d.mtscap = 0;
      if (dalloc(&d.mtk, d.sncap) != hipSuccess || dalloc(&d.mtk2, d.sncap) != hipSuccess)
        return FR_E_OOM;
      d.mtscap = d.sncap;
    }
    if (d.mtkcap < d.kcap) {
      dfree(d.mtw);
      dfree(d.mtchg);
      d.mtw = nullptr;
      d.mtchg = nullptr;
      if (dalloc(&d.mtw, d.kcap) != hipSuccess || dalloc(&d.mtchg, d.kcap) != hipSuccess)
        return FR_E_OOM;
      d.mtkcap = d.kcap;
    }
  }
  if (p->mb_reps <= 0) return FR_OK;
  if (d.mbqcap < d.sacap) {
    dfree(d.mbq);
    d.mbq = nullptr;
    d.mbqcap = 0;
    if (dalloc(&d.mbq, d.sacap) != hipSuccess) return FR_E_OOM;
    d.mbqcap = d.sacap;
  }
  if (d.mbccap < d.sncap) {
    dfree(d.mbc);
    d.mbc = nullptr;
    d.mbccap = 0;
    if (dalloc(&d.mbc, 4 * d.sncap) != hipSuccess) return FR_E_OOM;
    d.mbccap = d.sncap;
  }
  return FR_OK;
}

// Make the library stream wait for the caller's stream (inputs it produced).
static int32_t enter(fr_context *c) {
  HIPCHK(hipSetDevice(c->device));
  HIPCHK(hipEventRecord(c->ev[3], c->user_stream));
  HIPCHK(hipStreamWaitEvent(c->cs, c->ev[3], 0));
  c->counters[6] = 0;
  return FR_OK;
}

static int32_t check_batch_args(const fr_context *c, const fr_graph *g, const int32_t *part,
                                int32_t k, const int32_t *pairs, int32_t npairs,
                                const fr_params *p) {
  if (!c || !g || !part || !pairs || npairs < 1 || npairs > FR_MAX_PAIRS || k < 2 || k > FR_MAX_K ||
      g->n < 1 || !g->xadj || !g->adjncy || !g->adjwgt || !g->vwgt)
    return FR_E_INVALID_ARG;
  int32_t rc = check_params(p);
  if (rc) return rc;
  uint8_t used[FR_MAX_K];
  memset(used, 0, (size_t)k);
  for (int i = 0; i < npairs; i++) {
    const int32_t a = pairs[2 * i], b = pairs[2 * i + 1];
    if (a < 0 || b < 0 || a >= k || b >= k || a == b) return FR_E_INVALID_PAIR;
    if (used[a] || used[b]) return FR_E_PAIRS_NOT_DISJOINT;
    used[a] = used[b] = 1;
  }
  return FR_OK;
}

// The pair and batch entry points: one round of disjoint pairs.
// Speculative slots per pair: the length of the halving chain of alpha_max,
// as far as every entry still gets its own workgroup slot and the arenas stay
// within a fixed budget.  One slot without adaptive iterations, with the
// learned factor or when switched off.
static int32_t speculation_slots(const fr_context *c, const fr_params *p, int32_t npairs,
                                 int64_t n, int64_t narcs) {
  if (!c->speculate || !p->adaptive || p->max_iters < 2 || fused_rounds(c, p)) return 1;
  int32_t W = 0;
  for (int32_t a = p->alpha_max; a >= 1; a >>= 1) W++;
  const int64_t slots = (int64_t)c->num_cus * c->tune.blocks_per_cu;
  while (W > 1 && ((int64_t)npairs * W > slots || (int64_t)npairs * W > FR_MAX_PAIRS ||
                   W * n > (1ll << 28) || W * narcs > (1ll << 29)))
    W--;
  return W;
}

// Host-side scratch of a call: inline storage up to N elements, the heap
// beyond (the entry point without device allocation stays within N).
template <typename T, size_t N>
struct HostBuf {
  T inl[N];
  std::vector<T> heap;
  T *p = inl;
  size_t n = 0;
  void resize(size_t m) {
    n = m;
    if (m > N) {
      heap.resize(m);
      p = heap.data();
    } else {
      p = inl;
    }
  }
  T *data() { return p; }
  size_t size() const { return n; }
  T &operator[](size_t i) { return p[i]; }
};


// One batched round of disjoint pairs.  carve = nullptr: the context's
// buffers, grown on demand.  Otherwise the graph must be on the device, the
// call runs one entry per pair (no speculative slots) and every vertex-,
// arc- and block-sized buffer comes from *carve, which the caller sized for
// the graph; nothing is allocated.
static int32_t refine(fr_context *c, const fr_graph *g, int32_t *part, int32_t k,
                      const int32_t *pairs, int32_t npairs, const fr_params *p, fr_result *res,
                      int8_t *side_out, fr_solve *trace, const DevBufs *carve = nullptr) {
  int32_t rc = check_batch_args(c, g, part, k, pairs, npairs, p);
  if (rc) return rc;
  if (!res) return FR_E_INVALID_ARG;
  if (p->use_mlp && !c->mlp_loaded) return FR_E_INVALID_ARG;
  if ((rc = enter(c))) return rc;
  int64_t narcs0 = 0;
  if ((rc = graph_narcs(c, g, &narcs0))) return rc;
  const int32_t W = carve ? 1 : speculation_slots(c, p, npairs, g->n, narcs0);
  Staged s;
  if (carve) {
    if (!g->on_device || (int64_t)npairs > c->d.pcap || side_out) return FR_E_INVALID_ARG;
    s.g = *g;
    s.dpart = part;
    s.narcs = narcs0;
  } else {
    if ((rc = ensure_pairs(c, (int64_t)npairs * W))) return rc;
    if ((rc = stage(c, g, part, k, &s, W))) return rc;
    if ((rc = ensure_mb(c, p))) return rc;
  }
  const DevBufs &d = carve ? *carve : c->d;
  hipStream_t st = c->cs;
  const int64_t n = g->n;
  const int32_t V = npairs * W;
  (void)hipEventRecord(c->ev[0], st);
  HIPCHK(hipMemcpyAsync(d.partw, s.dpart, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st));
  KArgs A = call_args(c, d, &s.g, d.partw, k, p);
  A.W = W;
  A.mstride = W > 1 ? n : 0;
  if ((rc = call_constants(c, A, s.narcs, p, carve == nullptr))) return rc;
  HostBuf<int32_t, 8> a0, vp;
  a0.resize((size_t)V);
  vp.resize((size_t)2 * V);
  for (int32_t i = 0; i < V; i++) {
    a0[i] = p->alpha;
    vp[2 * i] = pairs[2 * (i / W)];
    vp[2 * i + 1] = pairs[2 * (i / W) + 1];
  }
  HIPCHK(hipMemcpyAsync(d.pairs, vp.data(), sizeof(int32_t) * 2 * V, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(d.alpha0, a0.data(), sizeof(int32_t) * V, hipMemcpyHostToDevice, st));
  int32_t mts = 0;
  if (p->mt_alpha > 0) {
    if ((rc = reserve_mt(c, npairs, &mts))) return rc;
    HIPCHK(hipMemsetAsync(d.mtchg, 0, (size_t)k, st));
  }
  int32_t stamp0 = 0;
  if (carve) {
    // the carved marks keep the previous call's stamps: clear them
    hipLaunchKernelGGL(k_fill32, dim3(std::min<int64_t>((n + 255) / 256, 4 * c->num_cus)),
                       dim3(256), 0, st, d.mark, n, 0);
    HIPCHK(hipGetLastError());
    stamp0 = 2;
  } else if ((rc = reserve_stamps(c, p->max_iters, &stamp0))) {
    return rc;
  }
  KArgs R = round_args(c, A, 0, V, stamp0, true);
  R.mt_stamp0 = mts;
  if (carve) R.slice_ticks = 0;
  (void)hipEventRecord(c->ev[1], st);
  if ((rc = enqueue_round(c, R, p->use_mlp != 0, st, true, false))) return rc;
  (void)hipEventRecord(c->ev[2], st);
  if ((rc = device_error(c))) return rc;
  if (side_out) {
    const int sblocks = std::min(4 * c->num_cus, 8192);
    hipLaunchKernelGGL(k_side_fill, dim3(sblocks), dim3(256), 0, st, R);
    hipLaunchKernelGGL(k_side_scatter, dim3(sblocks), dim3(256), 0, st, R);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(side_out, d.side, n, hipMemcpyDeviceToHost, st));
  }
  HostBuf<PairState, 4> ps;
  ps.resize((size_t)V);
  HIPCHK(hipMemcpyAsync(ps.data(), d.ps, sizeof(PairState) * V, hipMemcpyDeviceToHost, st));
  HostBuf<fr_solve, FR_MAX_ITERS> tr;
  if (trace) {
    tr.resize((size_t)npairs * p->max_iters);
    HIPCHK(hipMemcpyAsync(tr.data(), d.trace, sizeof(fr_solve) * tr.size(), hipMemcpyDeviceToHost, st));
  }
  HIPCHK(hipMemcpyAsync(part, d.partw, sizeof(int32_t) * n,
                        g->on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
  (void)hipEventRecord(c->ev[3], st);
  HIPCHK(hipStreamSynchronize(st));
  float t01 = 0.f, t12 = 0.f, t03 = 0.f;
  (void)hipEventElapsedTime(&t01, c->ev[0], c->ev[1]);
  (void)hipEventElapsedTime(&t12, c->ev[1], c->ev[2]);
  (void)hipEventElapsedTime(&t03, c->ev[0], c->ev[3]);
  reset_stats(c);
  add_entry_stats(c, ps.data(), ps.size());
  add_round_times(c);
  c->counters[5] = blocks_of(c, V);
  c->counters[7] = W;
  c->ms[0] = t01;  // validation, graph constants
  c->ms[1] = t12;  // the round: setup kernels and every flow iteration
  c->ms[4] = t03;  // whole call on the device
  for (int i = 0; i < npairs; i++) {
    fill_result(ps[(size_t)i * W], res[i]);
    if (trace)
      for (int j = 0; j < ps[(size_t)i * W].iters; j++)
        trace[(size_t)i * p->max_iters + j] = tr[(size_t)i * p->max_iters + j];
  }
  return FR_OK;
}

extern "C" int32_t flow_refine_pair(fr_context *c, const fr_graph *g, int32_t *part, int32_t k,
                                    int32_t a, int32_t b, const fr_params *p, fr_result *res,
                                    int8_t *side_out, fr_solve *trace) {
  const int32_t pr[2] = {a, b};
  return refine(c, g, part, k, pr, 1, p, res, side_out, trace);
}

// flow_refine_pair without device allocation: the vertex-, arc- and
// block-sized buffers are carved from the device's static scratch array
// (256-byte aligned pieces); the context's fixed per-call buffers were
// allocated by fr_create.
extern "C" int32_t flow_refine_pair_static(fr_context *c, const fr_graph *g, int32_t *part,
                                           int32_t k, int32_t a, int32_t b, const fr_params *p,
                                           fr_result *res, fr_solve *trace) {
  if (!c || !g || !part || !p || !res || g->n < 1 || k < 2 || k > FR_MAX_K) return FR_E_INVALID_ARG;
  if (!g->on_device || p->mb_reps != 0 || p->fm_limit != 0 || p->use_mlp || p->mt_alpha != 0)
    return FR_E_INVALID_ARG;
  int32_t rc = check_params(p);
  if (rc) return rc;
  if (c->device < 0 || c->device >= FR_MAX_DEVICES || !scratch_ptr[c->device]) return FR_E_DEVICE;
  HIPCHK(hipSetDevice(c->device));
  int64_t narcs = 0;
  if ((rc = graph_narcs(c, g, &narcs))) return rc;
  const int64_t n = g->n;
  DevBufs v = c->d;  // the fixed buffers stay; the sized ones are replaced
  unsigned char *const base = (unsigned char *)scratch_ptr[c->device];
  size_t off = 0;
  bool fits = true;
  auto take = [&](auto **ptr, size_t bytes) {
    off = (off + 255) & ~(size_t)255;
    fits = fits && off + bytes <= FR_STATIC_SCRATCH_BYTES;
    *ptr = fits ? reinterpret_cast<std::remove_reference_t<decltype(**ptr)> *>(base + off)
                : nullptr;
    off += bytes;
  };
  const size_t vn = sizeof(int32_t) * (size_t)n;
  take(&v.mark, vn);
  take(&v.vmap, vn);
  take(&v.uvert, vn);
  take(&v.lg, vn);
  take(&v.lo, sizeof(int32_t) * ((size_t)n + 2));
  take(&v.ex, vn);
  take(&v.lab, vn);
  take(&v.ins, vn);
  take(&v.LA, vn);
  take(&v.LB, vn);
  take(&v.SNK, vn);
  take(&v.partw, vn);
  take(&v.lflag, (size_t)n);
  take(&v.arc, sizeof(Arc) * (size_t)narcs);
  take(&v.blk2pair, sizeof(int32_t) * 3 * (size_t)k);
  take(&v.bstat, sizeof(int64_t) * 3 * (size_t)k);
  if (!fits) return FR_E_SCRATCH_LIMIT;
  v.side = nullptr;
  v.mbq = v.mbc = v.fmg = v.fmq = nullptr;
  v.gx = v.gv = v.ga = v.gw = v.parts = nullptr;
  v.qadj = nullptr;
  const int32_t pr[2] = {a, b};
  return refine(c, g, part, k, pr, 1, p, res, nullptr, trace, &v);
}

extern "C" int32_t flow_refine_batch(fr_context *c, const fr_graph *g, int32_t *part, int32_t k,
                                     const int32_t *pairs, int32_t npairs, const fr_params *p,
                                     fr_result *res, fr_solve *trace) {
  return refine(c, g, part, k, pairs, npairs, p, res, nullptr, trace);
}

// ---------------------------------------------------------------------------
// quotient graph, colouring and the refinement sweep

// Quotient edges (a < b, ascending) of a device partition and their greedy
// colours: each edge, in (a, b) order, takes the smallest colour free at
// both of its blocks, so every colour class is a matching.
static int32_t quotient_dev(fr_context *c, const fr_graph *g, const int32_t *dpart, int32_t k,
                            std::vector<int32_t> &edges, std::vector<int32_t> &colour) {
  DevBufs &d = c->d;
  hipStream_t st = c->cs;
  KArgs A;
  memset(&A, 0, sizeof(A));
  A.n = g->n;
  A.k = k;
  A.xadj = g->xadj;
  A.adjncy = g->adjncy;
  A.part = (int32_t *)dpart;
  HIPCHK(hipMemsetAsync(d.qadj, 0, (size_t)k * k, st));
  hipLaunchKernelGGL(k_quotient, dim3(std::min(4 * c->num_cus, 8192)), dim3(256), 0, st, A, d.qadj);
  HIPCHK(hipGetLastError());
  std::vector<uint8_t> q((size_t)k * k);
  HIPCHK(hipMemcpyAsync(q.data(), d.qadj, q.size(), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  edges.clear();
  colour.clear();
  for (int32_t x = 0; x < k; x++)
    for (int32_t y = x + 1; y < k; y++)
      if (q[(size_t)x * k + y]) {
        edges.push_back(x);
        edges.push_back(y);
      }
  std::vector<std::vector<uint8_t>> used;
  for (size_t i = 0; i < edges.size() / 2; i++) {
    const int32_t x = edges[2 * i], y = edges[2 * i + 1];
    int32_t col = 0;
    for (;; col++) {
      if ((size_t)col >= used.size()) used.emplace_back((size_t)k, 0);
      if (!used[col][x] && !used[col][y]) break;
    }
    used[col][x] = used[col][y] = 1;
    colour.push_back(col);
  }
  return FR_OK;
}

extern "C" int32_t fr_quotient_matchings(fr_context *c, const fr_graph *g, const int32_t *part,
                                         int32_t k, int32_t *edges, int32_t *colour,
                                         int32_t max_edges, int32_t *nedges) {
  if (!c || !g || !part || !edges || !colour || !nedges || k < 1 || k > FR_MAX_K || g->n < 1)
    return FR_E_INVALID_ARG;
  int32_t rc = enter(c);
  if (rc) return rc;
  Staged s;
  if ((rc = stage(c, g, const_cast<int32_t *>(part), k, &s))) return rc;
  std::vector<int32_t> e, col;
  if ((rc = quotient_dev(c, &s.g, s.dpart, k, e, col))) return rc;
  *nedges = (int32_t)col.size();
  if ((int64_t)col.size() > max_edges) return FR_E_INVALID_ARG;
  memcpy(edges, e.data(), sizeof(int32_t) * e.size());
  memcpy(colour, col.data(), sizeof(int32_t) * col.size());
  return FR_OK;
}

// One sweep = every colour class of the quotient graph, class after class;
// the rounds are recorded once into a hipGraph and launched as one graph.
extern "C" int32_t flow_refine_sweep(fr_context *c, const fr_graph *g, int32_t *part, int32_t k,
                                     const fr_params *p, int32_t max_sweeps,
                                     int64_t *total_cut_out, int64_t *stats) {
  if (!c || !g || !part || !p || max_sweeps < 1 || k < 2 || k > FR_MAX_K || g->n < 1)
    return FR_E_INVALID_ARG;
  int32_t rc = check_params(p);
  if (rc) return rc;
  if (p->use_mlp && !c->mlp_loaded) return FR_E_INVALID_ARG;
  if ((rc = enter(c))) return rc;
  // arenas for the longest factor chain a round may speculate on
  int64_t narcs0 = 0;
  if ((rc = graph_narcs(c, g, &narcs0))) return rc;
  const int32_t Wmax = speculation_slots(c, p, 1, g->n, narcs0);
  Staged s;
  if ((rc = stage(c, g, part, k, &s, Wmax))) return rc;
  if ((rc = ensure_mb(c, p))) return rc;
  DevBufs &d = c->d;
  hipStream_t st = c->cs;
  // the caller's partition changes only on success: work on a copy
  int32_t *work = d.partw;
  HIPCHK(hipMemcpyAsync(work, s.dpart, sizeof(int32_t) * g->n, hipMemcpyDeviceToDevice, st));
  reset_stats(c);
  (void)hipEventRecord(c->ev[0], st);
  KArgs A = call_args(c, d, &s.g, work, k, p);
  A.mstride = g->n;
  if ((rc = call_constants(c, A, s.narcs, p))) return rc;
  int64_t acc[4] = {0, 0, 0, 0};
  std::vector<int32_t> e, col, pairs, offs;
  std::vector<PairState> ps;
  std::vector<uint8_t> active((size_t)k, 1);  // active block scheduling (Sec. 4.3)
  for (int32_t sw = 0; sw < max_sweeps; sw++) {
    if ((rc = quotient_dev(c, &s.g, work, k, e, col))) return rc;
    if (p->active_blocks) {  // keep the quotient edges with an active block
      size_t m = 0;
      for (size_t i = 0; i < col.size(); i++)
        if (active[(size_t)e[2 * i]] || active[(size_t)e[2 * i + 1]]) {
          e[2 * m] = e[2 * i];
          e[2 * m + 1] = e[2 * i + 1];
          col[m++] = col[i];
        }
      e.resize(2 * m);
      col.resize(m);
    }
    int32_t ncol = 0;
    for (int32_t x : col) ncol = std::max(ncol, x + 1);
    std::vector<int32_t> per_class((size_t)ncol, 0);
    for (int32_t x : col) per_class[x]++;
    int32_t largest = 1;
    for (int32_t v : per_class) largest = std::max(largest, v);
    // speculative factors per pair, sized for the largest round
    const int32_t W = std::min(Wmax, speculation_slots(c, p, largest, g->n, narcs0));
    A.W = W;
    // entries of all rounds (each pair W times), class by class, at most
    // FR_MAX_PAIRS entries per round
    const int32_t per_round = FR_MAX_PAIRS / W;
    pairs.clear();
    offs.assign(1, 0);
    for (int32_t cc = 0; cc < ncol; cc++) {
      int32_t in_round = 0;
      for (size_t i = 0; i < col.size(); i++)
        if (col[i] == cc) {
          for (int32_t sl = 0; sl < W; sl++) {
            pairs.push_back(e[2 * i]);
            pairs.push_back(e[2 * i + 1]);
          }
          if (++in_round == per_round) {
            offs.push_back((int32_t)(pairs.size() / 2));
            in_round = 0;
          }
        }
      if (in_round) offs.push_back((int32_t)(pairs.size() / 2));
    }
    const int64_t total = (int64_t)pairs.size() / 2;
    if (total == 0) break;
    if ((rc = ensure_pairs(c, total))) return rc;
    std::vector<int32_t> a0((size_t)total, p->alpha);
    HIPCHK(hipMemcpyAsync(d.pairs, pairs.data(), sizeof(int32_t) * pairs.size(),
                          hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d.alpha0, a0.data(), sizeof(int32_t) * total, hipMemcpyHostToDevice, st));
    const int32_t nrounds = (int32_t)offs.size() - 1;
    int32_t stamp0 = 0;
    if ((rc = reserve_stamps(c, (int64_t)nrounds * (p->max_iters + 1), &stamp0))) return rc;
    // multi-try: consecutive touched stamps per round, changed blocks cleared
    std::vector<int32_t> mts((size_t)nrounds, 0);
    if (p->mt_alpha > 0) {
      int32_t m0 = 0;
      if ((rc = reserve_mt(c, total / W + nrounds, &m0))) return rc;
      for (int32_t r = 0; r < nrounds; r++) {
        mts[(size_t)r] = m0;
        m0 += (offs[r + 1] - offs[r]) / W + 1;
      }
      HIPCHK(hipMemsetAsync(d.mtchg, 0, (size_t)k, st));
    }
    HIPCHK(hipStreamSynchronize(st));
    if (c->timing) {
      // rounds launched one by one, each iteration's phases between events,
      // read back after every round (the events are reused)
      for (int32_t r = 0; r < nrounds; r++) {
        KArgs R = round_args(c, A, offs[r], offs[r + 1] - offs[r],
                             stamp0 + r * (2 * p->max_iters + 2), false);
        R.mt_stamp0 = mts[(size_t)r];
        if ((rc = enqueue_round(c, R, p->use_mlp != 0, st, true, false))) return rc;
        HIPCHK(hipStreamSynchronize(st));
        add_round_times(c);
      }
    } else {
      hipGraph_t graph = nullptr;
      hipGraphExec_t exec = nullptr;
      HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      int32_t cap_rc = FR_OK;
      for (int32_t r = 0; r < nrounds && cap_rc == FR_OK; r++) {
        KArgs R = round_args(c, A, offs[r], offs[r + 1] - offs[r],
                             stamp0 + r * (2 * p->max_iters + 2), false);
        R.mt_stamp0 = mts[(size_t)r];
        R.slice_ticks = 0;  // captured: no host between the launches
        cap_rc = enqueue_round(c, R, p->use_mlp != 0, st, false, true);
      }
      hipError_t ce = hipStreamEndCapture(st, &graph);
      if (cap_rc != FR_OK || ce != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return cap_rc != FR_OK ? cap_rc : FR_E_DEVICE;
      }
      ce = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      if (ce == hipSuccess) ce = hipGraphLaunch(exec, st);
      if (ce == hipSuccess) ce = hipStreamSynchronize(st);
      if (exec) (void)hipGraphExecDestroy(exec);
      (void)hipGraphDestroy(graph);
      if (ce != hipSuccess) {
        last_hip_error = ce;
        return FR_E_DEVICE;
      }
      c->graph_launches++;
      c->counters[14] += (int64_t)nrounds * p->max_iters;
    }
    if ((rc = device_error(c))) return rc;
    ps.resize((size_t)total);
    HIPCHK(hipMemcpyAsync(ps.data(), d.ps, sizeof(PairState) * total, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    add_entry_stats(c, ps.data(), ps.size());
    c->counters[7] = std::max<int64_t>(c->counters[7], W);
    int64_t changed = 0;
    std::fill(active.begin(), active.end(), 0);
    if (p->mt_alpha > 0) {  // blocks a kept multi-try move left or entered
      HIPCHK(hipMemcpyAsync(active.data(), d.mtchg, (size_t)k, hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
    }
    for (int64_t i = 0; i < total; i += W) {  // the pair's record is its first entry
      const PairState &q = ps[(size_t)i];
      acc[1] += q.iters;
      acc[3] += q.re_sum;
      if (q.applied || q.fm_kept)  // the pairwise improvement changed the partition
        active[(size_t)pairs[2 * i]] = active[(size_t)pairs[2 * i + 1]] = 1;
      if (q.applied || q.fm_kept || q.mt_kept) changed++;
    }
    acc[0]++;
    acc[2] += changed;
    if (changed == 0) break;
  }
  KArgs T = A;
  HIPCHK(hipMemsetAsync(d.scal, 0, sizeof(int64_t), st));
  hipLaunchKernelGGL(k_total_cut, dim3(std::min(4 * c->num_cus, 8192)), dim3(256), 0, st, T, d.scal);
  HIPCHK(hipGetLastError());
  int64_t tc = 0;
  HIPCHK(hipMemcpyAsync(&tc, d.scal, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(part, work, sizeof(int32_t) * g->n,
                        g->on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
  (void)hipEventRecord(c->ev[3], st);
  HIPCHK(hipStreamSynchronize(st));
  float t03 = 0.f;
  (void)hipEventElapsedTime(&t03, c->ev[0], c->ev[3]);
  c->ms[4] = t03;
  if (total_cut_out) *total_cut_out = tc;
  if (stats) memcpy(stats, acc, sizeof(acc));
  return FR_OK;
}

// ---------------------------------------------------------------------------
// learned area factor

extern "C" int32_t fr_mlp_num_params(void) { return MLP_NPARAMS; }

extern "C" int32_t fr_mlp_set_weights(fr_context *c, const float *w, int32_t count) {
  if (!c || !w || count != MLP_NPARAMS) return FR_E_INVALID_ARG;
  HIPCHK(hipSetDevice(c->device));
  HIPCHK(hipMemcpyAsync(c->d.mlp, w, sizeof(float) * MLP_NPARAMS, hipMemcpyHostToDevice, c->cs));
  HIPCHK(hipMemsetAsync(c->d.mlp_m, 0, sizeof(float) * MLP_NPARAMS, c->cs));
  HIPCHK(hipMemsetAsync(c->d.mlp_v, 0, sizeof(float) * MLP_NPARAMS, c->cs));
  HIPCHK(hipStreamSynchronize(c->cs));
  c->mlp_loaded = 1;
  return FR_OK;
}

extern "C" int32_t fr_mlp_get_weights(fr_context *c, float *w, int32_t count) {
  if (!c || !w || count != MLP_NPARAMS || !c->mlp_loaded) return FR_E_INVALID_ARG;
  HIPCHK(hipSetDevice(c->device));
  HIPCHK(hipMemcpyAsync(w, c->d.mlp, sizeof(float) * MLP_NPARAMS, hipMemcpyDeviceToHost, c->cs));
  HIPCHK(hipStreamSynchronize(c->cs));
  return FR_OK;
}

// He-normal weights, zero biases (host RNG, seeded).
extern "C" int32_t fr_mlp_init(fr_context *c, uint64_t seed) {
  if (!c) return FR_E_INVALID_ARG;
  std::vector<float> w(MLP_NPARAMS, 0.f);
  std::mt19937_64 rng(seed);
  auto fill = [&](int off, int fan_in, int count) {
    std::normal_distribution<float> nd(0.f, sqrtf(2.f / (float)fan_in));
    for (int i = 0; i < count; i++) w[off + i] = nd(rng);
  };
  fill(MLP_W1, MLP_IN, MLP_IN * MLP_H);
  fill(MLP_W2, MLP_H, MLP_H * MLP_H);
  fill(MLP_W3, MLP_H, MLP_H * MLP_OUT);
  return fr_mlp_set_weights(c, w.data(), MLP_NPARAMS);
}

// Scratch for n samples: x, labels or per-class costs, probs, activations
// (4*64), backward (5+2*64).
struct MlpScratch {
  float *x = nullptr, *probs = nullptr, *act = nullptr, *dact = nullptr, *loss = nullptr;
  int32_t *labels = nullptr, *idx = nullptr;
  float *xb = nullptr;
  int32_t *lb = nullptr;
  float *costs = nullptr, *cb = nullptr;
  ~MlpScratch() {
    dfree(x); dfree(probs); dfree(act); dfree(dact); dfree(loss); dfree(labels); dfree(idx);
    dfree(xb); dfree(lb); dfree(costs); dfree(cb);
  }
};

static int32_t mlp_alloc(MlpScratch &s, int64_t n, int64_t batch, bool with_costs = false) {
  const int64_t m = std::max(n, batch);
  if (dalloc(&s.x, n * MLP_IN) || dalloc(&s.probs, m * MLP_OUT) || dalloc(&s.act, m * 4 * MLP_H) ||
      dalloc(&s.dact, m * (MLP_OUT + 2 * MLP_H)) || dalloc(&s.loss, 1) || dalloc(&s.labels, n) ||
      dalloc(&s.idx, std::max<int64_t>(batch, 1)) || dalloc(&s.xb, batch * MLP_IN) ||
      dalloc(&s.lb, std::max<int64_t>(batch, 1)))
    return FR_E_OOM;
  if (with_costs && (dalloc(&s.costs, n * MLP_OUT) || dalloc(&s.cb, batch * MLP_OUT)))
    return FR_E_OOM;
  return FR_OK;
}

// labels, or per-class costs when costs is not null
static int32_t mlp_fwd_bwd(fr_context *c, const float *x, const int32_t *labels,
                           const float *costs, int32_t n, MlpScratch &s, bool backward) {
  hipStream_t st = c->cs;
  const int fb = (n + MLP_SAMPLES_PER_BLOCK - 1) / MLP_SAMPLES_PER_BLOCK;
  hipLaunchKernelGGL(k_mlp_forward, dim3(fb), dim3(1024), 0, st, (const float *)c->d.mlp, x, n,
                     s.probs, s.act);
  if (backward) {
    hipLaunchKernelGGL(k_mlp_backward, dim3(fb), dim3(1024), 0, st, (const float *)c->d.mlp,
                       (const float *)s.probs, labels, costs, n, (const float *)s.act, s.dact);
    hipLaunchKernelGGL(k_mlp_grad, dim3((MLP_NPARAMS + 255) / 256), dim3(256), 0, st, x,
                       (const float *)s.act, (const float *)s.dact, n, c->d.mlp_g);
  }
  HIPCHK(hipGetLastError());
  return FR_OK;
}

extern "C" int32_t fr_mlp_forward(fr_context *c, const float *x, int32_t n, float *probs) {
  if (!c || !x || !probs || n < 1 || !c->mlp_loaded) return FR_E_INVALID_ARG;
  HIPCHK(hipSetDevice(c->device));
  MlpScratch s;
  int32_t rc = mlp_alloc(s, n, 1);
  if (rc) return rc;
  HIPCHK(hipMemcpyAsync(s.x, x, sizeof(float) * MLP_IN * n, hipMemcpyHostToDevice, c->cs));
  if ((rc = mlp_fwd_bwd(c, s.x, nullptr, nullptr, n, s, false))) return rc;
  HIPCHK(hipMemcpyAsync(probs, s.probs, sizeof(float) * MLP_OUT * n, hipMemcpyDeviceToHost, c->cs));
  HIPCHK(hipStreamSynchronize(c->cs));
  return FR_OK;
}

extern "C" int32_t fr_mlp_predict(fr_context *c, const float *x, int32_t n, int32_t *alpha) {
  if (!c || !x || !alpha || n < 1 || !c->mlp_loaded) return FR_E_INVALID_ARG;
  HIPCHK(hipSetDevice(c->device));
  MlpScratch s;
  int32_t rc = mlp_alloc(s, n, 1);
  if (rc) return rc;
  HIPCHK(hipMemcpyAsync(s.x, x, sizeof(float) * MLP_IN * n, hipMemcpyHostToDevice, c->cs));
  if ((rc = mlp_fwd_bwd(c, s.x, nullptr, nullptr, n, s, false))) return rc;
  // the start factor of each sample, as the batch and sweep calls take it
  hipLaunchKernelGGL(k_alpha_from_probs, dim3((n + 255) / 256), dim3(256), 0, c->cs,
                     (const float *)s.probs, n, s.labels);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(alpha, s.labels, sizeof(int32_t) * n, hipMemcpyDeviceToHost, c->cs));
  HIPCHK(hipStreamSynchronize(c->cs));
  return FR_OK;
}

extern "C" int32_t fr_eps_to_ppm(double eps, int32_t *ppm) {
  if (!ppm || !(eps >= 0.0) || !(eps <= 100.0)) return FR_E_INVALID_ARG;  // NaN fails both
  *ppm = (int32_t)std::llround(eps * 1e6);
  return FR_OK;
}

// checks of the training targets: labels in [0, 5), or finite costs
static bool mlp_targets_ok(const int32_t *labels, const float *costs, int32_t n) {
  if (costs) {
    for (int64_t i = 0; i < (int64_t)n * MLP_OUT; i++)
      if (!std::isfinite(costs[i])) return false;
    return true;
  }
  if (!labels) return false;
  for (int32_t i = 0; i < n; i++)
    if (labels[i] < 0 || labels[i] >= MLP_OUT) return false;
  return true;
}

static int32_t mlp_loss_grad(fr_context *c, const float *x, const int32_t *labels,
                             const float *costs, int32_t n, float *loss, float *grad) {
  if (!c || !x || n < 1 || !c->mlp_loaded || !mlp_targets_ok(labels, costs, n))
    return FR_E_INVALID_ARG;
  HIPCHK(hipSetDevice(c->device));
  MlpScratch s;
  int32_t rc = mlp_alloc(s, n, 1, costs != nullptr);
  if (rc) return rc;
  HIPCHK(hipMemcpyAsync(s.x, x, sizeof(float) * MLP_IN * n, hipMemcpyHostToDevice, c->cs));
  if (costs)
    HIPCHK(hipMemcpyAsync(s.costs, costs, sizeof(float) * MLP_OUT * n, hipMemcpyHostToDevice, c->cs));
  else
    HIPCHK(hipMemcpyAsync(s.labels, labels, sizeof(int32_t) * n, hipMemcpyHostToDevice, c->cs));
  const float *dc = costs ? s.costs : nullptr;
  if ((rc = mlp_fwd_bwd(c, s.x, s.labels, dc, n, s, true))) return rc;
  hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(256), 0, c->cs, (const float *)s.probs,
                     (const int32_t *)s.labels, dc, n, s.loss);
  if (loss) HIPCHK(hipMemcpyAsync(loss, s.loss, sizeof(float), hipMemcpyDeviceToHost, c->cs));
  if (grad)
    HIPCHK(hipMemcpyAsync(grad, c->d.mlp_g, sizeof(float) * MLP_NPARAMS, hipMemcpyDeviceToHost, c->cs));
  HIPCHK(hipStreamSynchronize(c->cs));
  return FR_OK;
}

extern "C" int32_t fr_mlp_loss_grad(fr_context *c, const float *x, const int32_t *labels, int32_t n,
                                    float *loss, float *grad) {
  if (!labels) return FR_E_INVALID_ARG;
  return mlp_loss_grad(c, x, labels, nullptr, n, loss, grad);
}

extern "C" int32_t fr_mlp_loss_grad_cost(fr_context *c, const float *x, const float *costs,
                                         int32_t n, float *loss, float *grad) {
  if (!costs) return FR_E_INVALID_ARG;
  return mlp_loss_grad(c, x, nullptr, costs, n, loss, grad);
}

// Minibatch Adam on the device; epoch_loss (optional, [epochs]) gets the loss
// over all samples after each epoch (cross-entropy, or expected cost).
static int32_t mlp_train(fr_context *c, const float *x, const int32_t *labels, const float *costs,
                         int32_t n, int32_t epochs, int32_t batch, float lr, uint64_t seed,
                         float *epoch_loss) {
  if (!c || !x || n < 1 || epochs < 1 || batch < 1 || !(lr > 0.f) || !c->mlp_loaded ||
      !mlp_targets_ok(labels, costs, n))
    return FR_E_INVALID_ARG;
  HIPCHK(hipSetDevice(c->device));
  hipStream_t st = c->cs;
  batch = std::min(batch, n);
  MlpScratch s;
  int32_t rc = mlp_alloc(s, n, batch, costs != nullptr);
  if (rc) return rc;
  HIPCHK(hipMemcpyAsync(s.x, x, sizeof(float) * MLP_IN * n, hipMemcpyHostToDevice, st));
  if (costs)
    HIPCHK(hipMemcpyAsync(s.costs, costs, sizeof(float) * MLP_OUT * n, hipMemcpyHostToDevice, st));
  else
    HIPCHK(hipMemcpyAsync(s.labels, labels, sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
  const float *dc = costs ? s.costs : nullptr;
  const float *dcb = costs ? s.cb : nullptr;
  std::vector<int32_t> perm((size_t)n);
  std::iota(perm.begin(), perm.end(), 0);
  std::mt19937_64 rng(seed);
  int32_t t = 0;
  for (int32_t ep = 0; ep < epochs; ep++) {
    std::shuffle(perm.begin(), perm.end(), rng);
    for (int32_t b0 = 0; b0 + batch <= n; b0 += batch) {
      HIPCHK(hipMemcpyAsync(s.idx, perm.data() + b0, sizeof(int32_t) * batch, hipMemcpyHostToDevice, st));
      hipLaunchKernelGGL(k_gather_rows, dim3((batch * MLP_IN + 255) / 256), dim3(256), 0, st,
                         (const float *)s.x, (const int32_t *)s.labels, dc, (const int32_t *)s.idx,
                         batch, s.xb, s.lb, s.cb);
      if ((rc = mlp_fwd_bwd(c, s.xb, s.lb, dcb, batch, s, true))) return rc;
      hipLaunchKernelGGL(k_adam, dim3((MLP_NPARAMS + 255) / 256), dim3(256), 0, st, c->d.mlp,
                         (const float *)c->d.mlp_g, c->d.mlp_m, c->d.mlp_v, lr, 0.9f, 0.999f, 1e-8f,
                         ++t);
      HIPCHK(hipStreamSynchronize(st));  // the host batch indices are reused
    }
    if (epoch_loss) {
      if ((rc = mlp_fwd_bwd(c, s.x, s.labels, dc, n, s, false))) return rc;
      hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(256), 0, st, (const float *)s.probs,
                         (const int32_t *)s.labels, dc, n, s.loss);
      HIPCHK(hipMemcpyAsync(&epoch_loss[ep], s.loss, sizeof(float), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
    }
  }
  return FR_OK;
}

extern "C" int32_t fr_mlp_train(fr_context *c, const float *x, const int32_t *labels, int32_t n,
                                int32_t epochs, int32_t batch, float lr, uint64_t seed,
                                float *epoch_loss) {
  if (!labels) return FR_E_INVALID_ARG;
  return mlp_train(c, x, labels, nullptr, n, epochs, batch, lr, seed, epoch_loss);
}

extern "C" int32_t fr_mlp_train_cost(fr_context *c, const float *x, const float *costs, int32_t n,
                                     int32_t epochs, int32_t batch, float lr, uint64_t seed,
                                     float *epoch_loss) {
  if (!costs) return FR_E_INVALID_ARG;
  return mlp_train(c, x, nullptr, costs, n, epochs, batch, lr, seed, epoch_loss);
}

// The 8 input features of each pair (host [npairs * 8]).
extern "C" int32_t fr_pair_features(fr_context *c, const fr_graph *g, const int32_t *part,
                                    int32_t k, const int32_t *pairs, int32_t npairs,
                                    int32_t eps_ppm, float *feats) {
  fr_params p{FR_AREA_FACTOR, 0, 1, 1, 0, 1, eps_ppm, 0};
  int32_t rc = check_batch_args(c, g, part, k, pairs, npairs, &p);
  if (rc) return rc;
  if (!feats) return FR_E_INVALID_ARG;
  if ((rc = enter(c))) return rc;
  Staged s;
  if ((rc = stage(c, g, const_cast<int32_t *>(part), k, &s))) return rc;
  DevBufs &d = c->d;
  hipStream_t st = c->cs;
  KArgs A = call_args(c, d, &s.g, s.dpart, k, &p);
  if ((rc = call_constants(c, A, s.narcs, &p))) return rc;
  HIPCHK(hipMemcpyAsync(d.pairs, pairs, sizeof(int32_t) * 2 * npairs, hipMemcpyHostToDevice, st));
  KArgs R = round_args(c, A, 0, npairs, 0, false);
  R.fstat = d.fstat;
  const int sblocks = std::min(4 * c->num_cus, 8192);
  hipLaunchKernelGGL(k_round_init, dim3(1), dim3(1024), 0, st, R);
  hipLaunchKernelGGL(k_block_stats, dim3(c->g_bstat), dim3(256), 0, st, R);
  hipLaunchKernelGGL(k_feature_stats, dim3(c->g_fstat), dim3(256), 0, st, R, d.fstat);
  hipLaunchKernelGGL(k_features, dim3((npairs + 255) / 256), dim3(256), 0, st, R,
                     (const int64_t *)d.fstat, d.feats);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(feats, d.feats, sizeof(float) * MLP_IN * npairs, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return FR_OK;
}

// ---------------------------------------------------------------------------
// autotuner: times each candidate tuning on the same round (all must give
// identical results) and keeps the fastest.

extern "C" int32_t fr_autotune(fr_context *c, const fr_graph *g, const int32_t *part, int32_t k,
                               const int32_t *pairs, int32_t npairs, const fr_params *p,
                               const fr_tuning *cand, int32_t ncand, int32_t reps, double *ms_out,
                               int32_t *best_out) {
  if (!c || !g || !part || !pairs || !p || !cand || ncand < 1 || reps < 1) return FR_E_INVALID_ARG;
  if (!g->on_device) return FR_E_INVALID_ARG;  // tune on device-resident inputs
  int32_t rc = FR_OK;
  const fr_tuning keep = c->tune;
  int32_t *dpart = nullptr;
  HIPCHK(hipSetDevice(c->device));
  HIPCHK(hipMalloc((void **)&dpart, sizeof(int32_t) * (size_t)g->n));
  std::vector<fr_result> res((size_t)npairs), ref((size_t)npairs);
  double best_ms = 1e300;
  int32_t best = -1;
  for (int32_t i = 0; i < ncand && rc == FR_OK; i++) {
    if ((rc = fr_set_tuning(c, &cand[i]))) break;
    double tot = 0;
    for (int32_t r = 0; r < reps + 1 && rc == FR_OK; r++) {
      if (hipMemcpy(dpart, part, sizeof(int32_t) * (size_t)g->n, hipMemcpyDeviceToDevice) != hipSuccess) {
        rc = FR_E_DEVICE;
        break;
      }
      rc = refine(c, g, dpart, k, pairs, npairs, p, res.data(), nullptr, nullptr);
      if (rc) break;
      if (r > 0) tot += c->ms[1];  // the first run warms up
    }
    if (rc) break;
    if (i == 0) ref = res;
    for (int32_t j = 0; j < npairs; j++)
      if (memcmp(&res[j], &ref[j], sizeof(fr_result)) != 0) rc = FR_E_DEVICE;  // must not happen
    const double ms = tot / reps;
    if (ms_out) ms_out[i] = ms;
    if (ms < best_ms) {
      best_ms = ms;
      best = i;
    }
  }
  (void)hipFree(dpart);
  if (rc) {
    c->tune = keep;
    return rc;
  }
  c->tune = cand[best];
  if (best_out) *best_out = best;
  return FR_OK;
}
