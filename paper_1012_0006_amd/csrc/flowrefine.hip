// libflowrefine: host driver and C ABI (declared in include/flowrefine.h).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <numeric>
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

#define FR_MAX_PAIRS 4096
#define FR_MAX_K 8192
#define FR_MAX_BLOCKS_PER_CU 8

struct DevBufs {
  int64_t ncap = 0, acap = 0, kcap = 0;
  // per vertex
  int32_t *mark = nullptr, *vmap = nullptr, *uvert = nullptr, *lg = nullptr, *lo = nullptr,
          *ex = nullptr, *lab = nullptr, *ins = nullptr, *LA = nullptr, *LB = nullptr,
          *SNK = nullptr, *partw = nullptr, *parts = nullptr, *gx = nullptr, *gv = nullptr;
  uint8_t *lflag = nullptr;
  int8_t *side = nullptr;
  // per arc
  int32_t *lh = nullptr, *lr = nullptr, *rc = nullptr, *ga = nullptr, *gw = nullptr;
  // per block
  int32_t *blk2pair = nullptr;
  int64_t *bstat = nullptr;  // [3k]: weight, vertex count, arc count per block
  uint8_t *qadj = nullptr;   // k*k
  // per pair (fixed maximum)
  PairState *ps = nullptr;
  fr_solve *trace = nullptr;
  int32_t *pairs = nullptr, *order = nullptr, *ucnt = nullptr;
  int64_t *voff = nullptr, *aoff = nullptr, *base = nullptr, *scal = nullptr;
  Ctl *ctl = nullptr;
};

struct fr_context {
  int device = 0;
  hipStream_t stream = nullptr;
  int num_cus = 0;
  fr_tuning tune{1024, 2, 4, 200};
  int validate = 1;
  DevBufs d;
  Ctl *h_ctl = nullptr;  // pinned
  int32_t stamp = 2;
  double wall_khz = 100000.0;  // device constant-rate clock
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
                     &d.LB, &d.SNK, &d.partw, &d.parts, &d.gx, &d.gv, &d.lh, &d.lr, &d.rc,
                     &d.ga, &d.gw};
  for (auto pp : v32) {
    dfree(*pp);
    *pp = nullptr;
  }
  dfree(d.lflag);
  d.lflag = nullptr;
  dfree(d.side);
  d.side = nullptr;
  d.ncap = d.acap = 0;
}

static int32_t ensure_capacity(fr_context *c, int64_t n, int64_t narcs, int64_t k) {
  DevBufs &d = c->d;
  if (n > d.ncap || narcs > d.acap) {
    const int64_t nc = std::max(n, d.ncap), ac = std::max(narcs, d.acap);
    free_vertex_arc(d);
    hipError_t e = hipSuccess;
#define A_(p, cnt) \
  if (e == hipSuccess) e = dalloc(&d.p, cnt)
    A_(mark, nc); A_(vmap, nc); A_(uvert, nc); A_(lg, nc); A_(lo, nc + FR_MAX_PAIRS + 1);
    A_(ex, nc); A_(lab, nc); A_(ins, nc); A_(LA, nc); A_(LB, nc); A_(SNK, nc); A_(partw, nc);
    A_(parts, nc); A_(gx, nc + 1); A_(gv, nc); A_(lflag, nc); A_(side, nc);
    A_(lh, ac); A_(lr, ac); A_(rc, ac); A_(ga, ac); A_(gw, ac);
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
    dfree(d.blk2pair); dfree(d.bstat); dfree(d.qadj);
    d.blk2pair = nullptr;
    d.bstat = nullptr;
    d.qadj = nullptr;
    if (dalloc(&d.blk2pair, k) != hipSuccess || dalloc(&d.bstat, 3 * k) != hipSuccess ||
        dalloc(&d.qadj, k * k) != hipSuccess)
      return FR_E_OOM;
    d.kcap = k;
  }
  if (c->stamp > (1 << 29)) {  // corridor marks are compared against a growing stamp
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
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
    delete c;
    return FR_E_DEVICE;
  }
  c->num_cus = prop.multiProcessorCount;
  int rate = 0;
  if (hipDeviceGetAttribute(&rate, hipDeviceAttributeWallClockRate, device) == hipSuccess && rate > 0)
    c->wall_khz = rate;
  DevBufs &d = c->d;
  hipError_t e = hipSuccess;
#define A_(p, cnt) \
  if (e == hipSuccess) e = dalloc(&d.p, cnt)
  A_(ps, FR_MAX_PAIRS); A_(trace, (int64_t)FR_MAX_PAIRS * FR_MAX_ITERS); A_(pairs, 2 * FR_MAX_PAIRS);
  A_(order, FR_MAX_PAIRS); A_(ucnt, FR_MAX_PAIRS); A_(voff, FR_MAX_PAIRS + 1);
  A_(aoff, FR_MAX_PAIRS + 1); A_(base, FR_MAX_ALPHA + 1); A_(scal, 8); A_(ctl, 1);
#undef A_
  if (e == hipSuccess) e = hipHostMalloc((void **)&c->h_ctl, sizeof(Ctl), hipHostMallocDefault);
  for (int i = 0; i < 4 && e == hipSuccess; i++) e = hipEventCreate(&c->ev[i]);
  if (e != hipSuccess) {
    fr_destroy(c);
    return FR_E_OOM;
  }
  *out = c;
  return FR_OK;
}

extern "C" int32_t fr_destroy(fr_context *c) {
  if (!c) return FR_E_INVALID_ARG;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  free_vertex_arc(c->d);
  DevBufs &d = c->d;
  dfree(d.blk2pair); dfree(d.bstat); dfree(d.qadj); dfree(d.ps); dfree(d.trace); dfree(d.pairs);
  dfree(d.order); dfree(d.ucnt); dfree(d.voff); dfree(d.aoff); dfree(d.base); dfree(d.scal);
  dfree(d.ctl);
  if (c->h_ctl) (void)hipHostFree(c->h_ctl);
  for (int i = 0; i < 4; i++)
    if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
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
  c->tune = *t;
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

typedef void (*solve_fn)(KArgs);

static solve_fn solve_kernel(int tpb) {
  switch (tpb) {
    case 256: return k_solve<256>;
    case 512: return k_solve<512>;
    default: return k_solve<1024>;
  }
}

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

// Shared driver of the pair, batch and sweep entry points.  The graph is on
// the device (staged by the caller for host graphs); dpart is a device array
// that receives the result only on success.
static int32_t run_batch_dev(fr_context *c, const fr_graph *g, int64_t narcs, int32_t *dpart,
                             int32_t k, const int32_t *pairs, int32_t npairs, const fr_params *p,
                             const int32_t *alpha_start, fr_result *res, int8_t *side_out,
                             fr_solve *trace) {
  hipStream_t st = c->stream;
  DevBufs &d = c->d;
  const int64_t n = g->n;
  HIPCHK(hipMemcpyAsync(d.partw, dpart, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st));
  std::vector<int32_t> b2p((size_t)k, -1);
  for (int i = 0; i < npairs; i++) b2p[pairs[2 * i]] = b2p[pairs[2 * i + 1]] = i;
  HIPCHK(hipMemcpyAsync(d.blk2pair, b2p.data(), sizeof(int32_t) * k, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(d.pairs, pairs, sizeof(int32_t) * 2 * npairs, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemsetAsync(d.bstat, 0, sizeof(int64_t) * 3 * k, st));
  memset(c->h_ctl, 0, sizeof(Ctl));
  HIPCHK(hipMemcpyAsync(d.ctl, c->h_ctl, sizeof(Ctl), hipMemcpyHostToDevice, st));

  KArgs A;
  memset(&A, 0, sizeof(A));
  A.n = (int32_t)n;
  A.k = k;
  A.xadj = g->xadj;
  A.adjncy = g->adjncy;
  A.adjwgt = g->adjwgt;
  A.vwgt = g->vwgt;
  A.part = d.partw;
  A.P = npairs;
  A.pairs = d.pairs;
  A.order = d.order;
  A.blk2pair = d.blk2pair;
  A.ps = d.ps;
  A.trace = d.trace;
  A.base = d.base;
  A.area_mode = p->area_mode;
  A.depth = p->depth;
  A.alpha_max = p->alpha_max;
  A.adaptive = p->adaptive;
  A.max_iters = p->max_iters;
  A.eps_ppm = p->eps_ppm;
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
  A.lh = d.lh;
  A.lr = d.lr;
  A.rc = d.rc;
  A.ctl = d.ctl;
  A.tpv = c->tune.tpv;
  A.relabel_period = c->tune.relabel_period;
  A.max_sweeps = 4 * (n + 16) + 1000000;
  A.side_out = d.side;

  const int sblocks = std::min(4 * c->num_cus, 8192);
  (void)hipEventRecord(c->ev[0], st);
  if (c->validate) {
    hipLaunchKernelGGL(k_validate, dim3(sblocks), dim3(256), 0, st, A, narcs);
    HIPCHK(hipGetLastError());
  }
  int64_t *bw = d.bstat, *bcnt = d.bstat + k, *barc = d.bstat + 2 * k;
  hipLaunchKernelGGL(k_setup, dim3(sblocks), dim3(256), 0, st, A, bw, bcnt, barc);
  HIPCHK(hipGetLastError());
  std::vector<int64_t> hb((size_t)3 * k);
  HIPCHK(hipMemcpyAsync(hb.data(), d.bstat, sizeof(int64_t) * 3 * k, hipMemcpyDeviceToHost, st));
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
  // arena slices and the largest-first order of the pairs
  std::vector<int64_t> voff((size_t)npairs + 1, 0), aoff((size_t)npairs + 1, 0);
  std::vector<PairState> ps((size_t)npairs);
  for (int i = 0; i < npairs; i++) {
    const int32_t a = pairs[2 * i], b = pairs[2 * i + 1];
    voff[i + 1] = voff[i] + hb[k + a] + hb[k + b];
    aoff[i + 1] = aoff[i] + hb[2 * k + a] + hb[2 * k + b];
    PairState &s = ps[i];
    memset(&s, 0, sizeof(s));
    s.a = a;
    s.b = b;
    int al = alpha_start ? alpha_start[i] : p->alpha;
    al = std::min(std::max(al, 1), p->alpha_max);
    s.alpha = s.start_alpha = s.final_alpha = al;
    s.cA = hb[a];
    s.cB = hb[b];
    s.cut = s.cut0 = -1;
  }
  std::vector<int32_t> order((size_t)npairs);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
    return aoff[x + 1] - aoff[x] > aoff[y + 1] - aoff[y];
  });
  HIPCHK(hipMemcpyAsync(d.voff, voff.data(), sizeof(int64_t) * (npairs + 1), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(d.aoff, aoff.data(), sizeof(int64_t) * (npairs + 1), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(d.order, order.data(), sizeof(int32_t) * npairs, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(d.ps, ps.data(), sizeof(PairState) * npairs, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemsetAsync(d.ucnt, 0, sizeof(int32_t) * npairs, st));
  hipLaunchKernelGGL(k_union, dim3(sblocks), dim3(256), 0, st, A);
  HIPCHK(hipGetLastError());
  A.stamp0 = c->stamp;
  c->stamp += 2 * p->max_iters + 2;
  const int tpb = c->tune.block_threads;
  const int64_t slots = (int64_t)c->num_cus * c->tune.blocks_per_cu;
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(npairs, slots));
  (void)hipEventRecord(c->ev[1], st);
  hipLaunchKernelGGL(solve_kernel(tpb), dim3(blocks), dim3(tpb), 0, st, A);
  HIPCHK(hipGetLastError());
  (void)hipEventRecord(c->ev[2], st);
  HIPCHK(hipMemcpyAsync(c->h_ctl, d.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (c->h_ctl->err) {
    c->counters[6] = c->h_ctl->diag;
    if (verbose())
      fprintf(stderr, "flowrefine: device error %d (check %d)\n", c->h_ctl->err, c->h_ctl->diag);
    return c->h_ctl->err;
  }
  if (side_out) {
    hipLaunchKernelGGL(k_side_fill, dim3(sblocks), dim3(256), 0, st, A);
    hipLaunchKernelGGL(k_side_scatter, dim3(sblocks), dim3(256), 0, st, A);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(side_out, d.side, n, hipMemcpyDeviceToHost, st));
  }
  HIPCHK(hipMemcpyAsync(ps.data(), d.ps, sizeof(PairState) * npairs, hipMemcpyDeviceToHost, st));
  std::vector<fr_solve> tr;
  if (trace) {
    tr.resize((size_t)npairs * p->max_iters);
    HIPCHK(hipMemcpyAsync(tr.data(), d.trace, sizeof(fr_solve) * tr.size(), hipMemcpyDeviceToHost,
                          st));
  }
  HIPCHK(hipMemcpyAsync(dpart, d.partw, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st));
  (void)hipEventRecord(c->ev[3], st);
  HIPCHK(hipStreamSynchronize(st));
  float t01 = 0.f, t12 = 0.f, t03 = 0.f;
  (void)hipEventElapsedTime(&t01, c->ev[0], c->ev[1]);
  (void)hipEventElapsedTime(&t12, c->ev[1], c->ev[2]);
  (void)hipEventElapsedTime(&t03, c->ev[0], c->ev[3]);
  c->ms[0] = t01;  // validation, setup, arena
  c->ms[1] = t12;  // the batched solve kernel
  c->ms[4] = t03;  // whole call on the device
  int64_t sw = 0, rl = 0, bl = 0, gl = 0, cl = 0, wk[W_COUNT] = {0};
  double ph_c = 0, ph_b = 0, ph_r = 0, ph_p = 0, ph_f = 0;
  for (int i = 0; i < npairs; i++) {
    const PairState &s = ps[i];
    sw += s.sweeps;
    rl += s.relabels;
    bl += s.bfs_levels;
    gl += s.gr_levels;
    cl += s.cl_levels;
    for (int j = 0; j < W_COUNT; j++) wk[j] += s.work[j];
    ph_c += s.t_corridor;
    ph_b += s.t_build;
    ph_r += s.t_relabel;
    ph_p += s.t_push;
    ph_f += s.t_closure + s.t_finish;
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
  c->counters[0] = sw;
  c->counters[1] = rl;
  c->counters[2] = bl;
  c->counters[3] = gl;
  c->counters[4] = cl;
  c->counters[5] = blocks;
  c->counters[6] = 0;
  for (int j = 0; j < W_COUNT; j++) c->counters[16 + j] = wk[j];
  // per-phase device time summed over the pairs' workgroups
  c->ms[2] = ph_c / c->wall_khz;
  c->ms[3] = ph_b / c->wall_khz;
  c->ms[5] = ph_r / c->wall_khz;
  c->ms[6] = ph_p / c->wall_khz;
  c->ms[7] = ph_f / c->wall_khz;
  return FR_OK;
}

// Stage a host graph (and partition) on the device when needed.
struct Staged {
  fr_graph g;
  int32_t *dpart;
  int64_t narcs;
};

static int32_t stage(fr_context *c, const fr_graph *g, int32_t *part, int32_t k, Staged *s) {
  int64_t narcs = 0;
  int32_t rc = graph_narcs(c, g, &narcs);
  if (rc) return rc;
  if ((rc = ensure_capacity(c, g->n, narcs, k))) return rc;
  DevBufs &d = c->d;
  hipStream_t st = c->stream;
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

static int32_t unstage(fr_context *c, const fr_graph *g, int32_t *part, const Staged &s) {
  if (!g->on_device) {
    HIPCHK(hipMemcpyAsync(part, s.dpart, sizeof(int32_t) * g->n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
  }
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
  std::vector<uint8_t> used((size_t)k, 0);
  for (int i = 0; i < npairs; i++) {
    const int32_t a = pairs[2 * i], b = pairs[2 * i + 1];
    if (a < 0 || b < 0 || a >= k || b >= k || a == b) return FR_E_INVALID_PAIR;
    if (used[a] || used[b]) return FR_E_PAIRS_NOT_DISJOINT;
    used[a] = used[b] = 1;
  }
  return FR_OK;
}

static int32_t refine(fr_context *c, const fr_graph *g, int32_t *part, int32_t k,
                      const int32_t *pairs, int32_t npairs, const fr_params *p,
                      const int32_t *alpha_start, fr_result *res, int8_t *side_out,
                      fr_solve *trace) {
  int32_t rc = check_batch_args(c, g, part, k, pairs, npairs, p);
  if (rc) return rc;
  if (!res) return FR_E_INVALID_ARG;
  HIPCHK(hipSetDevice(c->device));
  Staged s;
  if ((rc = stage(c, g, part, k, &s))) return rc;
  rc = run_batch_dev(c, &s.g, s.narcs, s.dpart, k, pairs, npairs, p, alpha_start, res, side_out,
                     trace);
  if (rc) return rc;
  return unstage(c, g, part, s);
}

extern "C" int32_t flow_refine_pair(fr_context *c, const fr_graph *g, int32_t *part, int32_t k,
                                    int32_t a, int32_t b, const fr_params *p, fr_result *res,
                                    int8_t *side_out, fr_solve *trace) {
  const int32_t pr[2] = {a, b};
  if (p && p->use_mlp) return FR_E_INVALID_ARG;
  return refine(c, g, part, k, pr, 1, p, nullptr, res, side_out, trace);
}

extern "C" int32_t flow_refine_batch(fr_context *c, const fr_graph *g, int32_t *part, int32_t k,
                                     const int32_t *pairs, int32_t npairs, const fr_params *p,
                                     fr_result *res, fr_solve *trace) {
  if (p && p->use_mlp) return FR_E_INVALID_ARG;  // no area-factor network loaded
  return refine(c, g, part, k, pairs, npairs, p, nullptr, res, nullptr, trace);
}

// ---------------------------------------------------------------------------
// quotient graph, colouring and the refinement sweep

// Quotient edges (a < b, ascending) of a device partition and their greedy
// colours: each edge, in (a, b) order, takes the smallest colour free at
// both of its blocks, so every colour class is a matching.
static int32_t quotient_dev(fr_context *c, const fr_graph *g, const int32_t *dpart, int32_t k,
                            std::vector<int32_t> &edges, std::vector<int32_t> &colour) {
  DevBufs &d = c->d;
  hipStream_t st = c->stream;
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
  HIPCHK(hipSetDevice(c->device));
  Staged s;
  int32_t rc = stage(c, g, const_cast<int32_t *>(part), k, &s);
  if (rc) return rc;
  std::vector<int32_t> e, col;
  if ((rc = quotient_dev(c, &s.g, s.dpart, k, e, col))) return rc;
  *nedges = (int32_t)col.size();
  if ((int64_t)col.size() > max_edges) return FR_E_INVALID_ARG;
  memcpy(edges, e.data(), sizeof(int32_t) * e.size());
  memcpy(colour, col.data(), sizeof(int32_t) * col.size());
  return FR_OK;
}

extern "C" int32_t flow_refine_sweep(fr_context *c, const fr_graph *g, int32_t *part, int32_t k,
                                     const fr_params *p, int32_t max_sweeps,
                                     int64_t *total_cut_out, int64_t *stats) {
  if (!c || !g || !part || !p || max_sweeps < 1 || k < 2 || k > FR_MAX_K || g->n < 1)
    return FR_E_INVALID_ARG;
  int32_t rc = check_params(p);
  if (rc) return rc;
  if (p->use_mlp) return FR_E_INVALID_ARG;
  HIPCHK(hipSetDevice(c->device));
  Staged s;
  if ((rc = stage(c, g, part, k, &s))) return rc;
  DevBufs &d = c->d;
  hipStream_t st = c->stream;
  // the caller's partition changes only on success: work on a copy
  int32_t *work = d.parts;
  if (g->on_device)
    HIPCHK(hipMemcpyAsync(work, part, sizeof(int32_t) * g->n, hipMemcpyDeviceToDevice, st));
  int64_t acc[4] = {0, 0, 0, 0};
  std::vector<int32_t> e, col, pairs;
  std::vector<fr_result> res;
  for (int32_t sw = 0; sw < max_sweeps; sw++) {
    if ((rc = quotient_dev(c, &s.g, work, k, e, col))) return rc;
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
      const int32_t np = (int32_t)(pairs.size() / 2);
      res.assign((size_t)np, fr_result{});
      for (int32_t off = 0; off < np; off += FR_MAX_PAIRS) {
        const int32_t cnt = std::min(FR_MAX_PAIRS, np - off);
        rc = run_batch_dev(c, &s.g, s.narcs, work, k, pairs.data() + 2 * off, cnt, p, nullptr,
                           res.data() + off, nullptr, nullptr);
        if (rc) return rc;
      }
      for (const fr_result &r : res) {
        acc[1] += r.iters;
        acc[3] += r.region_edges;
        if (r.applied) changed++;
      }
    }
    acc[0]++;
    acc[2] += changed;
    if (changed == 0) break;
  }
  KArgs A;
  memset(&A, 0, sizeof(A));
  A.n = g->n;
  A.k = k;
  A.xadj = s.g.xadj;
  A.adjncy = s.g.adjncy;
  A.adjwgt = s.g.adjwgt;
  A.part = work;
  HIPCHK(hipMemsetAsync(d.scal, 0, sizeof(int64_t), st));
  hipLaunchKernelGGL(k_total_cut, dim3(std::min(4 * c->num_cus, 8192)), dim3(256), 0, st, A, d.scal);
  HIPCHK(hipGetLastError());
  int64_t tc = 0;
  HIPCHK(hipMemcpyAsync(&tc, d.scal, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(part, work, sizeof(int32_t) * g->n,
                        g->on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (total_cut_out) *total_cut_out = tc;
  if (stats) memcpy(stats, acc, sizeof(acc));
  return FR_OK;
}
