// libflowrefine: host driver and C ABI (declared in include/flowrefine.h).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "fr_internal.h"
#include "fr_kernels.h"

#define HIPCHK(x)                        \
  do {                                   \
    hipError_t _e = (x);                 \
    if (_e != hipSuccess) {              \
      last_hip_error = _e;               \
      return FR_E_DEVICE;                \
    }                                    \
  } while (0)

static thread_local hipError_t last_hip_error = hipSuccess;

struct DevBufs {
  int64_t ncap = 0, acap = 0, kcap = 0;
  // per vertex
  int32_t *mark = nullptr, *vmap = nullptr, *f0 = nullptr, *f1 = nullptr, *lglob = nullptr,
          *loff = nullptr, *lpair = nullptr, *ldeg = nullptr, *excess = nullptr, *label = nullptr,
          *ins = nullptr, *fa = nullptr, *fb = nullptr, *sinks = nullptr, *partw = nullptr;
  uint8_t *lflag = nullptr;
  int8_t *side = nullptr;
  // host-graph staging
  int32_t *gx = nullptr, *gv = nullptr;
  // per arc
  int32_t *lhead = nullptr, *lrev = nullptr, *rcap = nullptr, *ga = nullptr, *gw = nullptr;
  // per block
  int32_t *blk2pair = nullptr, *blk2side = nullptr;
  int64_t *bw = nullptr;
  uint8_t *qadj = nullptr;  // k*k
  int32_t *parts = nullptr; // sweep working partition [n]
  int64_t *scal = nullptr;  // scalar results
  // per pair (fixed maximum)
  PairState *ps = nullptr;
  fr_solve *trace = nullptr;
  int64_t *acc = nullptr, *lvlw = nullptr, *base = nullptr, *bsum = nullptr;
  int32_t *lvlc = nullptr, *pairs = nullptr, *alpha0 = nullptr;
  Ctl *ctl = nullptr;
  GridBar *bar = nullptr;
};

struct fr_context {
  int device = 0;
  hipStream_t stream = nullptr;
  int num_cus = 0;
  int64_t wall_khz = 0;
  fr_tuning tune{256, 4, 8, 6};
  int validate = 1;
  int occ_corridor = 1, occ_build = 1, occ_flow = 1, occ_finish = 1;
  int occ_tpb = 0;  // block size the flow occupancy was computed for
  DevBufs d;
  Ctl *h_ctl = nullptr;  // pinned
  int32_t stamp = 2;
  // stats of the last call
  double ms[8] = {0};
  int64_t counters[8] = {0};
  hipEvent_t ev[6] = {};
};

static const int MAX_BLOCKS = 8192;
// The occupancy query reports up to 7 resident 256-thread workgroups per CU
// for some kernels here, yet a cooperative grid of that size did not become
// co-resident on gfx950 (the bounded grid barrier timed out).  Persistent
// grids therefore stay at <= 4 workgroups per CU, a size every kernel ran at.
#define FR_MAX_BLOCKS_PER_CU 4

static void dfree(void *p) {
  if (p) (void)hipFree(p);
}

static void free_vertex_arc(DevBufs &d) {
  dfree(d.mark); dfree(d.vmap); dfree(d.f0); dfree(d.f1); dfree(d.lglob); dfree(d.loff);
  dfree(d.lpair); dfree(d.ldeg); dfree(d.excess); dfree(d.label); dfree(d.ins); dfree(d.fa);
  dfree(d.fb); dfree(d.sinks); dfree(d.partw); dfree(d.lflag); dfree(d.side); dfree(d.gx);
  dfree(d.gv); dfree(d.lhead); dfree(d.lrev); dfree(d.rcap); dfree(d.ga); dfree(d.gw);
  dfree(d.parts);
  d.parts = nullptr;
  d.mark = d.vmap = d.f0 = d.f1 = d.lglob = d.loff = d.lpair = d.ldeg = d.excess = d.label =
      d.ins = d.fa = d.fb = d.sinks = d.partw = d.gx = d.gv = nullptr;
  d.lflag = nullptr;
  d.side = nullptr;
  d.lhead = d.lrev = d.rcap = d.ga = d.gw = nullptr;
  d.ncap = d.acap = 0;
}

template <typename T>
static hipError_t dalloc(T **p, int64_t count) {
  return hipMalloc((void **)p, sizeof(T) * (size_t)(count > 0 ? count : 1));
}

static int32_t ensure_capacity(fr_context *c, int64_t n, int64_t narcs, int64_t k) {
  DevBufs &d = c->d;
  if (n > d.ncap || narcs > d.acap) {
    int64_t nc = std::max(n, d.ncap), ac = std::max(narcs, d.acap);
    free_vertex_arc(d);
    hipError_t e = hipSuccess;
#define A_(p, cnt) if (e == hipSuccess) e = dalloc(&d.p, cnt)
    A_(mark, nc); A_(vmap, nc); A_(f0, nc); A_(f1, nc); A_(lglob, nc); A_(loff, nc + 1);
    A_(lpair, nc); A_(ldeg, nc); A_(excess, nc); A_(label, nc); A_(ins, nc); A_(fa, nc);
    A_(fb, nc); A_(sinks, nc); A_(partw, nc); A_(lflag, nc); A_(side, nc); A_(gx, nc + 1);
    A_(gv, nc); A_(lhead, ac); A_(lrev, ac); A_(rcap, ac); A_(ga, ac); A_(gw, ac);
    A_(parts, nc);
#undef A_
    if (e != hipSuccess) {
      free_vertex_arc(d);
      return FR_E_OOM;
    }
    if (hipMemset(d.mark, 0, sizeof(int32_t) * (size_t)nc) != hipSuccess) return FR_E_DEVICE;
    d.ncap = nc;
    d.acap = ac;
    c->stamp = 2;
  }
  if (k > d.kcap) {
    dfree(d.blk2pair); dfree(d.blk2side); dfree(d.bw); dfree(d.qadj);
    d.blk2pair = d.blk2side = nullptr;
    d.bw = nullptr;
    d.qadj = nullptr;
    if (dalloc(&d.blk2pair, k) != hipSuccess || dalloc(&d.blk2side, k) != hipSuccess ||
        dalloc(&d.bw, k) != hipSuccess || dalloc(&d.qadj, k * k) != hipSuccess)
      return FR_E_OOM;
    d.kcap = k;
  }
  if (c->stamp > (1 << 29)) {  // marks are compared against a growing stamp
    if (hipMemset(d.mark, 0, sizeof(int32_t) * (size_t)d.ncap) != hipSuccess) return FR_E_DEVICE;
    c->stamp = 2;
  }
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
    case FR_E_SOLVER_LIMIT: return "push/relabel sweep limit reached";
    default: return "unknown error";
  }
}

static bool verbose() {
  static int v = -1;
  if (v < 0) {
    const char *e = getenv("FR_VERBOSE");
    v = (e && *e && *e != '0') ? 1 : 0;
  }
  return v == 1;
}

static int occupancy(const void *fn, int tpb, int num_cus) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, tpb, 0) != hipSuccess || nb < 1)
    nb = 1;
  return nb;
}

static const void *flow_kernel(int tpb) {
  switch (tpb) {
    case 64: return (const void *)k_flow<64>;
    case 128: return (const void *)k_flow<128>;
    case 512: return (const void *)k_flow<512>;
    case 1024: return (const void *)k_flow<1024>;
    default: return (const void *)k_flow<256>;
  }
}

static void refresh_occupancy(fr_context *c) {
  c->occ_corridor = occupancy((const void *)k_corridor, 256, c->num_cus);
  c->occ_build = occupancy((const void *)k_build, 256, c->num_cus);
  c->occ_finish = occupancy((const void *)k_finish, 256, c->num_cus);
  c->occ_flow = occupancy(flow_kernel(c->tune.block_threads), c->tune.block_threads, c->num_cus);
  c->occ_tpb = c->tune.block_threads;
  if (verbose())
    fprintf(stderr, "flowrefine: occupancy corridor %d build %d flow(%d) %d finish %d, %d CUs\n",
            c->occ_corridor, c->occ_build, c->tune.block_threads, c->occ_flow, c->occ_finish,
            c->num_cus);
}

extern "C" int32_t fr_create(int32_t device, void *hip_stream, fr_context **out) {
  if (!out) return FR_E_INVALID_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return FR_E_DEVICE;
  if (hipSetDevice(device) != hipSuccess) return FR_E_DEVICE;
  fr_context *c = new (std::nothrow) fr_context();
  if (!c) return FR_E_OOM;
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  hipDeviceProp_t prop;
  int coop = 0, rate = 0;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess ||
      hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, device) != hipSuccess ||
      hipDeviceGetAttribute(&rate, hipDeviceAttributeWallClockRate, device) != hipSuccess || !coop) {
    delete c;
    return FR_E_DEVICE;
  }
  c->num_cus = prop.multiProcessorCount;
  c->wall_khz = rate > 0 ? rate : 100000;
  DevBufs &d = c->d;
  hipError_t e = hipSuccess;
#define A_(p, cnt) if (e == hipSuccess) e = dalloc(&d.p, cnt)
  A_(ps, FR_MAX_PAIRS); A_(trace, (int64_t)FR_MAX_PAIRS * FR_MAX_ITERS);
  A_(acc, (int64_t)FR_MAX_PAIRS * FR_NACC); A_(lvlw, 6 * FR_MAX_PAIRS);
  A_(lvlc, 6 * FR_MAX_PAIRS); A_(pairs, 2 * FR_MAX_PAIRS); A_(alpha0, FR_MAX_PAIRS);
  A_(base, FR_MAX_ALPHA + 1); A_(bsum, MAX_BLOCKS + 1); A_(ctl, 1); A_(bar, 1);
  A_(scal, 8);
#undef A_
  if (e == hipSuccess) e = hipMemset(d.bar, 0, sizeof(GridBar));
  if (e == hipSuccess) e = hipHostMalloc((void **)&c->h_ctl, sizeof(Ctl), hipHostMallocDefault);
  for (int i = 0; i < 6 && e == hipSuccess; i++) e = hipEventCreate(&c->ev[i]);
  if (e != hipSuccess) {
    fr_destroy(c);
    return FR_E_OOM;
  }
  refresh_occupancy(c);
  *out = c;
  return FR_OK;
}

extern "C" int32_t fr_destroy(fr_context *c) {
  if (!c) return FR_E_INVALID_ARG;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  free_vertex_arc(c->d);
  DevBufs &d = c->d;
  dfree(d.blk2pair); dfree(d.blk2side); dfree(d.bw); dfree(d.qadj); dfree(d.scal); dfree(d.ps); dfree(d.trace); dfree(d.acc);
  dfree(d.lvlw); dfree(d.lvlc); dfree(d.pairs); dfree(d.alpha0); dfree(d.base); dfree(d.bsum);
  dfree(d.ctl); dfree(d.bar);
  if (c->h_ctl) (void)hipHostFree(c->h_ctl);
  for (int i = 0; i < 6; i++)
    if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
  delete c;
  return FR_OK;
}

extern "C" int32_t fr_set_tuning(fr_context *c, const fr_tuning *t) {
  if (!c || !t) return FR_E_INVALID_ARG;
  int bt = t->block_threads;
  if (!(bt == 64 || bt == 128 || bt == 256 || bt == 512 || bt == 1024)) return FR_E_INVALID_ARG;
  if (t->blocks_per_cu < 1 || t->blocks_per_cu > FR_MAX_BLOCKS_PER_CU) return FR_E_INVALID_ARG;
  if (!(t->tpv == 1 || t->tpv == 2 || t->tpv == 4 || t->tpv == 8 || t->tpv == 16))
    return FR_E_INVALID_ARG;
  if (t->relabel_period < 1 || t->relabel_period > 1000000) return FR_E_INVALID_ARG;
  c->tune = *t;
  (void)hipSetDevice(c->device);
  refresh_occupancy(c);
  return FR_OK;
}

extern "C" int32_t fr_get_tuning(fr_context *c, fr_tuning *t) {
  if (!c || !t) return FR_E_INVALID_ARG;
  *t = c->tune;
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
      p->max_iters < 1 || p->max_iters > FR_MAX_ITERS || p->eps_ppm < 0 || p->eps_ppm > 100000000)
    return FR_E_INVALID_ARG;
  return FR_OK;
}

static int cooperative(fr_context *c, const void *fn, int blocks, int tpb, void **args) {
  hipError_t e = hipLaunchCooperativeKernel(fn, dim3(blocks), dim3(tpb), args, 0, c->stream);
  if (e != hipSuccess) {
    last_hip_error = e;
    c->counters[6] = 100 + (int)e;
    if (verbose())
      fprintf(stderr, "flowrefine: cooperative launch of %d x %d failed: %s\n", blocks, tpb,
              hipGetErrorString(e));
    return FR_E_DEVICE;
  }
  return FR_OK;
}

// Shared driver of the pair and batch entry points.
static int32_t run_batch(fr_context *c, const fr_graph *g, int32_t *part, int32_t k,
                         const int32_t *pairs, int32_t npairs, const fr_params *p,
                         const int32_t *alpha_start, fr_result *res, int8_t *side_out,
                         fr_solve *trace) {
  if (!c || !g || !part || !pairs || !res || npairs < 1 || npairs > FR_MAX_PAIRS || k < 2 ||
      g->n < 1 || !g->xadj || !g->adjncy || !g->adjwgt || !g->vwgt)
    return FR_E_INVALID_ARG;
  int32_t rc = check_params(p);
  if (rc) return rc;
  {
    std::vector<uint8_t> used((size_t)k, 0);
    for (int i = 0; i < npairs; i++) {
      int32_t a = pairs[2 * i], b = pairs[2 * i + 1];
      if (a < 0 || b < 0 || a >= k || b >= k || a == b) return FR_E_INVALID_PAIR;
      if (used[a] || used[b]) return FR_E_PAIRS_NOT_DISJOINT;
      used[a] = used[b] = 1;
    }
  }
  HIPCHK(hipSetDevice(c->device));
  c->counters[6] = 0;
  hipStream_t st = c->stream;
  const int64_t n = g->n;
  int32_t narcs32 = 0;
  if (g->on_device) {
    HIPCHK(hipMemcpyAsync(&narcs32, g->xadj + n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  } else {
    narcs32 = g->xadj[n];
  }
  if (narcs32 < 0) return FR_E_INVALID_GRAPH;
  const int64_t narcs = narcs32;
  rc = ensure_capacity(c, n, narcs, k);
  if (rc) return rc;
  DevBufs &d = c->d;
  const int32_t *xadj = g->xadj, *adjncy = g->adjncy, *adjwgt = g->adjwgt, *vwgt = g->vwgt;
  if (!g->on_device) {
    HIPCHK(hipMemcpyAsync(d.gx, g->xadj, sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d.ga, g->adjncy, sizeof(int32_t) * narcs, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d.gw, g->adjwgt, sizeof(int32_t) * narcs, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d.gv, g->vwgt, sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d.partw, part, sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
    xadj = d.gx;
    adjncy = d.ga;
    adjwgt = d.gw;
    vwgt = d.gv;
  } else {
    HIPCHK(hipMemcpyAsync(d.partw, part, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st));
  }
  // block -> pair maps
  std::vector<int32_t> b2p((size_t)k, -1), b2s((size_t)k, 0);
  for (int i = 0; i < npairs; i++) {
    b2p[pairs[2 * i]] = i;
    b2p[pairs[2 * i + 1]] = i;
    b2s[pairs[2 * i]] = 0;
    b2s[pairs[2 * i + 1]] = 1;
  }
  HIPCHK(hipMemcpyAsync(d.blk2pair, b2p.data(), sizeof(int32_t) * k, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(d.blk2side, b2s.data(), sizeof(int32_t) * k, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(d.pairs, pairs, sizeof(int32_t) * 2 * npairs, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemsetAsync(d.bw, 0, sizeof(int64_t) * k, st));
  memset(c->h_ctl, 0, sizeof(Ctl));
  c->h_ctl->stamp = c->stamp;
  HIPCHK(hipMemcpyAsync(d.ctl, c->h_ctl, sizeof(Ctl), hipMemcpyHostToDevice, st));

  KArgs A;
  memset(&A, 0, sizeof(A));
  A.n = (int32_t)n;
  A.k = k;
  A.xadj = xadj;
  A.adjncy = adjncy;
  A.adjwgt = adjwgt;
  A.vwgt = vwgt;
  A.part = d.partw;
  A.P = npairs;
  A.blk2pair = d.blk2pair;
  A.blk2side = d.blk2side;
  A.ps = d.ps;
  A.trace = d.trace;
  A.base = d.base;
  A.area_mode = p->area_mode;
  A.depth = p->depth;
  A.alpha_max = p->alpha_max;
  A.adaptive = p->adaptive;
  A.max_iters = p->max_iters;
  A.eps_ppm = p->eps_ppm;
  A.mark = d.mark; A.vmap = d.vmap; A.f0 = d.f0; A.f1 = d.f1;
  A.lglob = d.lglob; A.loff = d.loff; A.lpair = d.lpair; A.ldeg = d.ldeg; A.excess = d.excess;
  A.label = d.label; A.ins = d.ins; A.fa = d.fa; A.fb = d.fb; A.sinks = d.sinks; A.lflag = d.lflag;
  A.lhead = d.lhead; A.lrev = d.lrev; A.rcap = d.rcap;
  A.acc = d.acc; A.lvlw = d.lvlw; A.lvlc = d.lvlc; A.bsum = d.bsum; A.ctl = d.ctl; A.bar = d.bar;
  A.side_out = d.side;
  A.tpv = c->tune.tpv;
  A.relabel_period = c->tune.relabel_period;
  A.max_sweeps = 4 * (n + 16) + 1000000;
  A.spin_limit = (uint64_t)c->wall_khz * 1000ull * 20ull;  // 20 s

  const int sblocks = std::min(4 * c->num_cus, MAX_BLOCKS);
  (void)hipEventRecord(c->ev[0], st);
  if (c->validate) {
    hipLaunchKernelGGL(k_validate, dim3(sblocks), dim3(256), 0, st, A, narcs);
    HIPCHK(hipGetLastError());
  }
  hipLaunchKernelGGL(k_setup, dim3(sblocks), dim3(256), 0, st, A, d.bw);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(c->h_ctl, d.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (c->h_ctl->bad_graph) return FR_E_INVALID_GRAPH;
  if (c->h_ctl->bad_part) return FR_E_INVALID_PART;
  const int64_t cV = c->h_ctl->cV, maxc = c->h_ctl->maxc;
  // L_max = (1+eps) c(V)/k + max c(v) (Sec. 2.1) and the area bases
  // floor((1 + alpha eps) c(V) / k), exact in 128-bit arithmetic
  const unsigned __int128 den = (unsigned __int128)1000000 * (unsigned)k;
  A.lmax = floor_div_u128((unsigned __int128)(1000000 + (int64_t)p->eps_ppm) * (uint64_t)cV, den) +
           maxc;
  std::vector<int64_t> base((size_t)p->alpha_max + 1, 0);
  for (int al = 0; al <= p->alpha_max; al++)
    base[al] = floor_div_u128(
        (unsigned __int128)(1000000 + (int64_t)al * p->eps_ppm) * (uint64_t)cV, den);
  HIPCHK(hipMemcpyAsync(d.base, base.data(), sizeof(int64_t) * base.size(), hipMemcpyHostToDevice,
                        st));
  std::vector<int32_t> a0((size_t)npairs);
  for (int i = 0; i < npairs; i++) {
    int al = alpha_start ? alpha_start[i] : p->alpha;
    a0[i] = std::min(std::max(al, 1), p->alpha_max);
  }
  HIPCHK(hipMemcpyAsync(d.alpha0, a0.data(), sizeof(int32_t) * npairs, hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_pair_init, dim3(1), dim3(256), 0, st, A, d.pairs, d.bw, d.alpha0);
  HIPCHK(hipGetLastError());

  const int nb_cor = std::min(c->num_cus * std::min(c->occ_corridor, c->tune.blocks_per_cu), MAX_BLOCKS);
  const int nb_bld = std::min(c->num_cus * std::min(c->occ_build, c->tune.blocks_per_cu), MAX_BLOCKS);
  const int nb_flw = std::min(c->num_cus * std::min(c->occ_flow, c->tune.blocks_per_cu), MAX_BLOCKS);
  const int nb_fin = std::min(c->num_cus * std::min(c->occ_finish, c->tune.blocks_per_cu), MAX_BLOCKS);
  const void *kflow = flow_kernel(c->tune.block_threads);
  int32_t round = 0;
  void *args1[] = {&A};
  void *args2[] = {&A, &round};
  int32_t status = FR_OK;
  for (round = 0; round < p->max_iters; round++) {
    if ((rc = cooperative(c, (const void *)k_corridor, nb_cor, 256, args1))) return rc;
    if ((rc = cooperative(c, (const void *)k_build, nb_bld, 256, args1))) return rc;
    if ((rc = cooperative(c, kflow, nb_flw, c->tune.block_threads, args1))) return rc;
    if ((rc = cooperative(c, (const void *)k_finish, nb_fin, 256, args2))) return rc;
    HIPCHK(hipMemcpyAsync(c->h_ctl, d.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    GridBar hb;
    HIPCHK(hipMemcpyAsync(&hb, d.bar, sizeof(GridBar), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (hb.abort) {
      (void)hipMemsetAsync(d.bar, 0, sizeof(GridBar), st);
      (void)hipStreamSynchronize(st);
      status = FR_E_DEVICE;
      c->counters[6] = 50;
      if (verbose()) fprintf(stderr, "flowrefine: grid barrier timed out\n");
      break;
    }
    if (c->h_ctl->err) {
      status = c->h_ctl->err;
      c->counters[6] = c->h_ctl->diag;
      if (verbose())
        fprintf(stderr, "flowrefine: device error %d (check %d) in round %d\n", c->h_ctl->err,
                c->h_ctl->diag, round);
      break;
    }
    if (c->h_ctl->active_pairs == 0) break;
  }
  c->stamp = c->h_ctl->stamp;
  if (status != FR_OK) {
    c->stamp += 2;
    return status;
  }
  if (side_out) {
    hipLaunchKernelGGL(k_side_out, dim3(sblocks), dim3(256), 0, st, A);
    hipLaunchKernelGGL(k_side_out2, dim3(sblocks), dim3(256), 0, st, A);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(side_out, d.side, n, hipMemcpyDeviceToHost, st));
  }
  std::vector<PairState> ps((size_t)npairs);
  HIPCHK(hipMemcpyAsync(ps.data(), d.ps, sizeof(PairState) * npairs, hipMemcpyDeviceToHost, st));
  std::vector<fr_solve> tr((size_t)npairs * p->max_iters);
  HIPCHK(hipMemcpyAsync(tr.data(), d.trace, sizeof(fr_solve) * tr.size(), hipMemcpyDeviceToHost, st));
  (void)hipEventRecord(c->ev[1], st);
  if (g->on_device)
    HIPCHK(hipMemcpyAsync(part, d.partw, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st));
  else
    HIPCHK(hipMemcpyAsync(part, d.partw, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, c->ev[0], c->ev[1]);
  c->ms[4] = ms;
  c->counters[0] = c->h_ctl->sweeps;
  c->counters[1] = c->h_ctl->relabels;
  c->counters[2] = c->h_ctl->bfs_levels;
  c->counters[3] = c->h_ctl->gr_levels;
  c->counters[4] = c->h_ctl->cl_levels;
  c->counters[5] = round + (round < p->max_iters ? 1 : 0);
  for (int i = 0; i < npairs; i++) {
    const PairState &s = ps[i];
    fr_result &r = res[i];
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
    if (s.applied > 0) r.status = FR_ACCEPTED;
    else if (s.last_dec == FR_DEC_NOT_ADJACENT) r.status = FR_NOT_ADJACENT;
    else if (s.last_dec == FR_DEC_INFEASIBLE) r.status = FR_REJECTED_IMBALANCE;
    else r.status = FR_NO_IMPROVEMENT;
    if (trace)
      for (int j = 0; j < s.iters; j++)
        trace[(size_t)i * p->max_iters + j] = tr[(size_t)i * p->max_iters + j];
  }
  return FR_OK;
}

extern "C" int32_t flow_refine_pair(fr_context *c, const fr_graph *g, int32_t *part, int32_t k,
                                    int32_t a, int32_t b, const fr_params *p, fr_result *res,
                                    int8_t *side_out, fr_solve *trace) {
  int32_t pr[2] = {a, b};
  if (p && p->use_mlp) return FR_E_INVALID_ARG;
  return run_batch(c, g, part, k, pr, 1, p, nullptr, res, side_out, trace);
}

extern "C" int32_t flow_refine_batch(fr_context *c, const fr_graph *g, int32_t *part, int32_t k,
                                     const int32_t *pairs, int32_t npairs, const fr_params *p,
                                     fr_result *res, fr_solve *trace) {
  if (p && p->use_mlp) return FR_E_INVALID_ARG;  // learned factor: not loaded
  return run_batch(c, g, part, k, pairs, npairs, p, nullptr, res, nullptr, trace);
}

// ---------------------------------------------------------------------------
// quotient graph, colouring and the refinement sweep

static int32_t graph_narcs(fr_context *c, const fr_graph *g, int64_t *narcs) {
  int32_t na = 0;
  if (g->on_device) {
    HIPCHK(hipMemcpyAsync(&na, g->xadj + g->n, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
  } else {
    na = g->xadj[g->n];
  }
  if (na < 0) return FR_E_INVALID_GRAPH;
  *narcs = na;
  return FR_OK;
}

// Quotient edges (a < b, ascending) of a partition held on the device and
// their greedy colours.
static int32_t quotient_dev(fr_context *c, int32_t n, const int32_t *xadj, const int32_t *adjncy,
                            const int32_t *part, int32_t k, std::vector<int32_t> &edges,
                            std::vector<int32_t> &colour) {
  DevBufs &d = c->d;
  hipStream_t st = c->stream;
  KArgs A;
  memset(&A, 0, sizeof(A));
  A.n = n;
  A.k = k;
  A.xadj = xadj;
  A.adjncy = adjncy;
  A.part = (int32_t *)part;
  HIPCHK(hipMemsetAsync(d.qadj, 0, (size_t)k * k, st));
  hipLaunchKernelGGL(k_quotient, dim3(std::min(4 * c->num_cus, MAX_BLOCKS)), dim3(256), 0, st, A,
                     d.qadj);
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
  // greedy edge colouring in (a, b) order: smallest colour free at both ends
  std::vector<std::vector<uint8_t>> used;
  for (size_t i = 0; i < edges.size() / 2; i++) {
    int32_t x = edges[2 * i], y = edges[2 * i + 1], col = 0;
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
  if (!c || !g || !part || !edges || !colour || !nedges || k < 1 || g->n < 1)
    return FR_E_INVALID_ARG;
  HIPCHK(hipSetDevice(c->device));
  int64_t narcs = 0;
  int32_t rc = graph_narcs(c, g, &narcs);
  if (rc) return rc;
  if ((rc = ensure_capacity(c, g->n, narcs, k))) return rc;
  DevBufs &d = c->d;
  hipStream_t st = c->stream;
  const int32_t *xadj = g->xadj, *adjncy = g->adjncy, *dpart = part;
  if (!g->on_device) {
    HIPCHK(hipMemcpyAsync(d.gx, g->xadj, sizeof(int32_t) * (g->n + 1), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d.ga, g->adjncy, sizeof(int32_t) * narcs, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d.parts, part, sizeof(int32_t) * g->n, hipMemcpyHostToDevice, st));
    xadj = d.gx;
    adjncy = d.ga;
    dpart = d.parts;
  }
  std::vector<int32_t> e, col;
  if ((rc = quotient_dev(c, g->n, xadj, adjncy, dpart, k, e, col))) return rc;
  *nedges = (int32_t)col.size();
  if ((int64_t)col.size() > max_edges) return FR_E_INVALID_ARG;
  memcpy(edges, e.data(), sizeof(int32_t) * e.size());
  memcpy(colour, col.data(), sizeof(int32_t) * col.size());
  return FR_OK;
}

extern "C" int32_t flow_refine_sweep(fr_context *c, const fr_graph *g, int32_t *part, int32_t k,
                                     const fr_params *p, int32_t max_sweeps,
                                     int64_t *total_cut_out, int64_t *stats) {
  if (!c || !g || !part || !p || max_sweeps < 1 || k < 2 || g->n < 1) return FR_E_INVALID_ARG;
  int32_t rc = check_params(p);
  if (rc) return rc;
  if (p->use_mlp) return FR_E_INVALID_ARG;
  HIPCHK(hipSetDevice(c->device));
  int64_t narcs = 0;
  if ((rc = graph_narcs(c, g, &narcs))) return rc;
  if ((rc = ensure_capacity(c, g->n, narcs, k))) return rc;
  DevBufs &d = c->d;
  hipStream_t st = c->stream;
  fr_graph dg = *g;
  if (!g->on_device) {
    HIPCHK(hipMemcpyAsync(d.gx, g->xadj, sizeof(int32_t) * (g->n + 1), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d.ga, g->adjncy, sizeof(int32_t) * narcs, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d.gw, g->adjwgt, sizeof(int32_t) * narcs, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d.gv, g->vwgt, sizeof(int32_t) * g->n, hipMemcpyHostToDevice, st));
    dg.xadj = d.gx;
    dg.adjncy = d.ga;
    dg.adjwgt = d.gw;
    dg.vwgt = d.gv;
    dg.on_device = 1;
  }
  HIPCHK(hipMemcpyAsync(d.parts, part, sizeof(int32_t) * g->n,
                        g->on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
  int64_t st_[4] = {0, 0, 0, 0};
  std::vector<int32_t> e, col, pairs;
  std::vector<fr_result> res;
  for (int32_t s = 0; s < max_sweeps; s++) {
    if ((rc = quotient_dev(c, g->n, dg.xadj, dg.adjncy, d.parts, k, e, col))) return rc;
    int32_t ncol = 0;
    for (int32_t x : col) ncol = std::max(ncol, x + 1);
    int64_t changed = 0;
    for (int32_t cc = 0; cc < ncol; cc++) {
      pairs.clear();
      for (size_t i = 0; i < col.size(); i++)
        if (col[i] == cc) {
          pairs.push_back(e[2 * i]);
          pairs.push_back(e[2 * i + 1]);
        }
      int32_t np = (int32_t)(pairs.size() / 2);
      res.assign((size_t)np, fr_result{});
      for (int32_t off = 0; off < np; off += FR_MAX_PAIRS) {
        int32_t cnt = std::min(FR_MAX_PAIRS, np - off);
        rc = run_batch(c, &dg, d.parts, k, pairs.data() + 2 * off, cnt, p, nullptr,
                       res.data() + off, nullptr, nullptr);
        if (rc) return rc;
      }
      for (const fr_result &r : res) {
        st_[1] += r.iters;
        st_[3] += r.region_edges;
        if (r.applied) changed++;
      }
    }
    st_[0]++;
    st_[2] += changed;
    if (changed == 0) break;
  }
  // total cut
  KArgs A;
  memset(&A, 0, sizeof(A));
  A.n = g->n;
  A.k = k;
  A.xadj = dg.xadj;
  A.adjncy = dg.adjncy;
  A.adjwgt = dg.adjwgt;
  A.part = d.parts;
  HIPCHK(hipMemsetAsync(d.scal, 0, sizeof(int64_t), st));
  hipLaunchKernelGGL(k_total_cut, dim3(std::min(4 * c->num_cus, MAX_BLOCKS)), dim3(256), 0, st, A,
                     d.scal);
  HIPCHK(hipGetLastError());
  int64_t tc = 0;
  HIPCHK(hipMemcpyAsync(&tc, d.scal, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(part, d.parts, sizeof(int32_t) * g->n,
                        g->on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (total_cut_out) *total_cut_out = tc;
  if (stats) memcpy(stats, st_, sizeof(st_));
  return FR_OK;
}
