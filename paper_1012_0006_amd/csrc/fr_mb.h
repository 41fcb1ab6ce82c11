// Most balanced minimum cut (Sanders & Schulz, Section 4.1.1) on the GPU:
// one workgroup per entry, after the flow kernel has left a maximum preflow,
// exact distance labels and the smallest source set S_min.
//
// With a maximum preflow, the minimum cuts are the sets closed under residual
// arcs that contain S_min and avoid every vertex that can still reach the
// sink (label < NL).  The free vertices M in between were listed by the flow
// kernel.  Their residual strongly connected components form a DAG whose
// closed sets are exactly the remaining choices:
//   1. union-find over residual arcs usable in both directions (such
//      vertices share a component): the "bidirectional classes", grid-wide
//      over the free vertices of all entries (k_mb_scan, k_mb_union); the
//      same pass lists the one-way residual arcs inside M (saturated edges);
//   2. the quotient graph Q of the classes over those one-way arcs, and
//      Tarjan's SCC algorithm on Q in one lane (LDS when Q is small);
//   3. the component DAG (weights, key ids, in-degrees, arcs);
//   4. sweeps, one per wave: Kahn's algorithm taking the ready component
//      with the smallest SplitMix64 key (a wave-wide minimum) moves them to the sink side
//      one by one, starting from the largest minimum source side; the first
//      most balanced cut is kept;
//   5. the chosen components join the source side; the solve's record gets
//      the new block weights and decision.
// The components and their reachability order are the same for every
// maximum flow or preflow, and the sweep order depends on nothing else, so
// the result equals that of any exact implementation of the same rule.
#pragma once
#include "fr_kernels.h"

#define MB_TPB 1024
#define MB_LCOMP 2048     // components whose DAG is held in LDS; more: device memory
#define MB_LQ 1024        // quotient nodes handled in LDS
#define MB_LQA 4096       // quotient arcs handled in LDS
#define MB_LDAG 4096      // component arcs held in LDS
#define MB_RS_BYTES 24576 // sweep state of the concurrent sweeps (in-degrees, states)
#define MBK 8             // arc records in flight per lane

struct MBShared {
  union {
    struct {                         // Tarjan's scratch (LDS path)
      int32_t low[MB_LQ], stk[MB_LQ], cnode[MB_LQ], cpos[MB_LQ];
    } t;
    struct {                         // the component DAG, built after Tarjan
      int64_t cw[MB_LCOMP];          // component weights
      int32_t ckey[MB_LCOMP];        // component key id: smallest global vertex id
      int32_t cend[MB_LCOMP];        // component arcs: counts, then end offsets
      int32_t cin[MB_LCOMP];         // in-degrees among the components
      int16_t adj[MB_LDAG];          // component arcs (when they fit)
      uint8_t sink[MB_LCOMP];        // chosen cut: component on the sink side
    } c;
  } u1;
  union {
    struct {                         // the quotient graph (LDS path), until the DAG is built
      int32_t qidx[MB_LQ];           // Tarjan index / component of each quotient node
      int32_t qoff[MB_LQ];           // quotient arcs: counts, then start offsets
      int32_t qarc[MB_LQA];
    } q;
    uint32_t rs[MB_RS_BYTES / 4];    // sweep state (in-degrees and states)
  } u2;
  int64_t red[64];
  int64_t lane_bal[MB_TPB / WAVE];
  int32_t lane_pos[MB_TPB / WAVE];
  int64_t best_bal;
  int32_t best_rep, best_pos;
  int32_t nq, eq, nc, ne, n1w, skip;
};
static_assert(sizeof(MBShared) <= 80 * 1024, "two workgroups per CU");

// SplitMix64 (Steele, Lea & Flood 2014): output number n of the generator
// started at seed, i.e. its 64-bit finaliser applied to seed + n * gamma.
__device__ __forceinline__ uint64_t mb_splitmix(uint64_t seed, uint64_t n) {
  uint64_t z = seed + n * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// key of the component with key id g in sweep r
__device__ __forceinline__ uint64_t mb_key(uint64_t seed, int32_t r, int32_t g) {
  return mb_splitmix(seed, ((((uint64_t)(uint32_t)r) << 32) | (uint32_t)g) + 1ull);
}

// minimum of v over the lanes with the same key, one atomic per distinct key
// of the wave (keys < 0 take no part).  Converged wave only.
__device__ __forceinline__ void wave_min_by_key(int32_t *base, int key, int32_t v) {
  unsigned long long todo = __ballot(key >= 0);
  while (todo) {
    const int leader = __ffsll(todo) - 1;
    const int k0 = __shfl(key, leader);
    const bool mine = key == k0;
    int32_t x = mine ? v : 0x7fffffff;
    for (int o = 32; o > 0; o >>= 1) x = min(x, __shfl_xor(x, o));
    if (lane64() == leader) atomicMin(base + k0, x);
    todo &= ~__ballot(mine);
  }
}

__device__ __forceinline__ int32_t aload(const int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// union-find root with path halving; parents only move to smaller ids of the
// same class, so racing halvings store valid ancestors
__device__ __forceinline__ int32_t uf_find(int32_t *par, int32_t x) {
  for (;;) {
    const int32_t y = aload(par + x);
    if (y == x) return x;
    const int32_t z = aload(par + y);
    if (z != y) __hip_atomic_store(par + x, z, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    x = z;
  }
}

// hook the larger root under the smaller: the root of a class ends up as its
// smallest vertex
__device__ __forceinline__ void uf_union(int32_t *par, int32_t u, int32_t v) {
  for (;;) {
    u = uf_find(par, u);
    v = uf_find(par, v);
    if (u == v) return;
    const int32_t hi = max(u, v), lo = min(u, v);
    if (atomicCAS(par + hi, hi, lo) == hi) return;
  }
}

// Exclusive scan of a[0..N) in place (LDS or device memory); returns the
// total.  All threads call it.
__device__ int32_t mb_exscan(int32_t *a, int32_t N, int64_t *red) {
  int64_t carry = 0;
  for (int32_t b0 = 0; b0 < N; b0 += blockDim.x) {
    const int32_t i = b0 + (int32_t)threadIdx.x;
    const int64_t v = i < N ? a[i] : 0;
    int64_t tot;
    const int64_t ex = block_exscan64(v, &tot, red);
    if (i < N) a[i] = (int32_t)(carry + ex);
    carry += tot;
  }
  __syncthreads();
  return (int32_t)carry;
}

// One sweep, run by one wave: Kahn's algorithm over the C components that
// takes, among the ready ones (all predecessors placed), the one with the
// smallest key -- the lanes hold C/64 components each and a wave-wide minimum
// picks it; the placed component moves to the sink side and its arcs release
// their targets.  wa/wb: block weights with every free component on the
// source side.  Returns, in every lane, the first position with the smallest
// max(wa, wb) (0 = none moved) and its balance; with mark set, flags the
// components moved up to position stop.
template <typename ADJ>
struct MBSweep {
  int32_t C;
  const int32_t *cin, *cend;
  const ADJ *adj;  // component arcs: int16 in LDS or int32 in device memory
  const int64_t *cw;
  const int32_t *ckey;
  uint64_t seed;
  __device__ int32_t run(int32_t rep, int32_t *ind, uint8_t *state, int64_t wa, int64_t wb,
                         int32_t stop, uint8_t *mark, int64_t *best_out, Ctl *ctl) const {
    const int lane = lane64();
    for (int32_t c = lane; c < C; c += WAVE) {  // state: 0 waiting, 1 ready, 2 placed
      const int32_t d = cin[c];
      ind[c] = d;
      state[c] = d == 0 ? 1 : 0;
    }
    int64_t best = wa > wb ? wa : wb;
    int32_t bj = 0;
    for (int32_t j = 1; j <= stop; j++) {
      uint64_t bk = 0;
      int32_t bc = -1;
      for (int32_t c = lane; c < C; c += WAVE)
        if (state[c] == 1) {
          const uint64_t k = mb_key(seed, rep, ckey[c]);
          if (bc < 0 || k < bk) {
            bk = k;
            bc = c;
          }
        }
      // the wave's minimum (keys of distinct components differ): lane by lane
      // in scalar registers when few lanes hold a candidate, else a butterfly
      unsigned long long cand = __ballot(bc >= 0);
      if (__popcll(cand) <= 8) {
        uint64_t wk = 0;
        int32_t wc = -1;
        while (cand) {
          const int l = __ffsll(cand) - 1;
          cand &= cand - 1;
          const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)bk, l);
          const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(bk >> 32), l);
          const uint64_t k = ((uint64_t)hi << 32) | lo;
          if (wc < 0 || k < wk) {
            wk = k;
            wc = __builtin_amdgcn_readlane(bc, l);
          }
        }
        bk = wk;
        bc = wc;
      } else {
        for (int o = WAVE / 2; o > 0; o >>= 1) {
          const uint32_t lo = __shfl_xor((uint32_t)bk, o), hi = __shfl_xor((uint32_t)(bk >> 32), o);
          const uint64_t ok = ((uint64_t)hi << 32) | lo;
          const int32_t oc = __shfl_xor(bc, o);
          if (oc >= 0 && (bc < 0 || ok < bk)) {
            bk = ok;
            bc = oc;
          }
        }
      }
      if (bc < 0) {  // nothing ready: a cycle among the components, cannot happen
        if (lane == 0) {
          ctl->err = FR_E_DEVICE;
          ctl->diag = DIAG_MB;
        }
        break;
      }
      if (lane == 0) {
        state[bc] = 2;
        if (mark) mark[bc] = 1;
      }
      wa -= cw[bc];
      wb += cw[bc];
      const int64_t bal = wa > wb ? wa : wb;
      if (bal < best) {
        best = bal;
        bj = j;
      }
      const int32_t e1 = cend[bc];
      for (int32_t e = (bc ? cend[bc - 1] : 0) + lane; e < e1; e += WAVE) {
        const int32_t d = adj[e];
        if (atomicSub(ind + d, 1) == 1) state[d] = 1;
      }
    }
    *best_out = best;
    return bj;
  }
};

// Quotient-graph SCC (Tarjan 1972) in one lane: idx[q] = -1 unvisited,
// >= 0 visit index while on the component stack, -2 - c once in component c.
// Returns the number of components.
__device__ __forceinline__ int32_t mb_tarjan(int32_t nq, int32_t eq, const int32_t *qoff,
                                             const int32_t *qarc, int32_t *idx, int32_t *low,
                                             int32_t *stk, int32_t *cnode, int32_t *cpos) {
  int32_t next = 0, ns = 0, nc = 0;
  for (int32_t root = 0; root < nq; root++) {
    if (idx[root] != -1) continue;
    // the node being searched lives in registers (v, its next arc e, its arc
    // end, its lowest reachable index lv); the call stack keeps the parents'
    // (node, next arc) in cnode/cpos and their lowest index in low
    int32_t depth = 0;
    int32_t v = root, e = qoff[root], end = root + 1 < nq ? qoff[root + 1] : eq;
    int32_t lv = next;
    idx[root] = next++;
    stk[ns++] = root;
    for (;;) {
      if (e < end) {
        const int32_t w = qarc[e++];
        const int32_t iw = idx[w];
        if (iw == -1) {  // tree arc: descend
          cnode[depth] = v;
          cpos[depth] = e;
          low[v] = lv;
          depth++;
          v = w;
          e = qoff[w];
          end = w + 1 < nq ? qoff[w + 1] : eq;
          lv = next;
          idx[w] = next++;
          stk[ns++] = w;
        } else if (iw >= 0 && iw < lv) {  // on the component stack
          lv = iw;
        }
        continue;
      }
      if (lv == idx[v]) {  // v closes a component
        int32_t x;
        do {
          x = stk[--ns];
          idx[x] = -2 - nc;
        } while (x != v);
        nc++;
      }
      if (depth == 0) break;
      depth--;
      const int32_t u = cnode[depth];
      const int32_t lu = low[u];
      lv = lv < lu ? lv : lu;
      v = u;
      e = cpos[depth];
      end = u + 1 < nq ? qoff[u + 1] : eq;
    }
  }
  return nc;
}

// Entries that take part in the most balanced cut this launch and their
// free-vertex counts, as prefix sums over the entries (one block).
__device__ __forceinline__ int32_t mb_free_count(const KArgs &A, int32_t p) {
  const PairState &ps = A.ps[p];
  if (ps.done || A.srec[p].decision == FR_DEC_NOT_ADJACENT) return 0;
  return min(A.pcnt[p], ps.nr);
}

__global__ void __launch_bounds__(1024) k_mb_scan(KArgs A, int32_t it) {
  __shared__ int64_t red[17];
  (void)it;
  int64_t carry = 0;
  for (int32_t b0 = 0; b0 < A.P; b0 += blockDim.x) {
    const int32_t p = b0 + (int32_t)threadIdx.x;
    const int64_t v = (p < A.P && A.ctl->err == 0) ? mb_free_count(A, p) : 0;
    int64_t tot;
    const int64_t ex = block_exscan64(v, &tot, red);
    if (p < A.P) A.mpre[p] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) A.mpre[A.P] = carry;
}

// Step 1 over the free vertices of every entry, one lane per vertex with its
// arc records loaded MBK at a time: union of the ends of every residual arc
// usable both ways (agent-scope atomics, so the workgroups of one entry may
// sit on any XCD), and the entry's one-way arcs inside M appended to its
// list (count in pcnt[P + p]).
__global__ void __launch_bounds__(256) k_mb_union(KArgs A, int32_t it) {
  (void)it;
  const int64_t total = A.mpre[A.P];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t p = pair_of(A.mpre, A.P, i);
    const int64_t vb = A.voff[p], ab = A.aoff[p];
    int32_t *par = A.LA + vb;
    const int32_t *lo = A.lo + vb + p;
    const Arc *arc = A.arc + ab;
    int32_t *w1 = A.mbq + ab;
    const int32_t u = A.LB[vb + (i - A.mpre[p])];
    const int32_t e1 = lo[u + 1];
    for (int32_t c0 = lo[u]; c0 < e1; c0 += MBK) {
      Arc x[MBK];
#pragma unroll
      for (int k = 0; k < MBK; k++) x[k] = c0 + k < e1 ? arc[c0 + k] : Arc{0, 0, 0ull};
      int32_t pv[MBK];
#pragma unroll
      for (int k = 0; k < MBK; k++) pv[k] = res_own(x[k].rc) > 0 ? par[x[k].lh] : -1;
#pragma unroll
      for (int k = 0; k < MBK; k++) {
        if (pv[k] < 0) continue;
        if (res_rev(x[k].rc) > 0) {
          if (x[k].lh > u) uf_union(par, u, x[k].lh);
        } else {
          w1[atomicAdd(A.pcnt + A.P + p, 1)] = c0 + k;
        }
      }
    }
  }
}

// The mb_reps sweeps, one per wave, `per` at a time: sweep l of a batch
// keeps its in-degrees at ind + l * C and its state bytes at st + l * C (LDS,
// or device memory for large component graphs); then a replay of the winning
// sweep by the first wave flags its sink components in `sink`.
template <typename ADJ>
__device__ __forceinline__ void mb_sweeps(const KArgs &A, MBShared &sh, const MBSweep<ADJ> &S,
                                          int64_t wa0, int64_t wb0, int32_t *ind, uint8_t *st,
                                          int32_t per, uint8_t *sink) {
  const int32_t C = S.C;
  if (threadIdx.x == 0) {
    sh.best_rep = -1;
    sh.best_pos = 0;
    sh.best_bal = 0;
  }
  for (int32_t r0 = 0; r0 < A.mb_reps; r0 += per) {
    const int32_t nl = min(per, A.mb_reps - r0);
    const int l = threadIdx.x / WAVE;
    if (l < nl) {
      int64_t bal;
      const int32_t j = S.run(r0 + l, ind + (int64_t)l * C, st + (int64_t)l * C, wa0, wb0, C,
                              nullptr, &bal, A.ctl);
      if (lane64() == 0) {
        sh.lane_bal[l] = bal;
        sh.lane_pos[l] = j;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int k = 0; k < nl; k++)
        if (sh.best_rep < 0 || sh.lane_bal[k] < sh.best_bal) {
          sh.best_bal = sh.lane_bal[k];
          sh.best_rep = r0 + k;
          sh.best_pos = sh.lane_pos[k];
        }
    }
    __syncthreads();
  }
  // the chosen cut: replay the winning sweep up to its position
  if (threadIdx.x < WAVE && sh.best_pos > 0) {
    int64_t bal;
    S.run(sh.best_rep, ind, st, wa0, wb0, sh.best_pos, sink, &bal, A.ctl);
  }
  __syncthreads();
}

__global__ void __launch_bounds__(MB_TPB) k_mb(KArgs A, int32_t it) {
  __shared__ MBShared sh;
  (void)it;
  const int32_t p = blockIdx.x;
  // the free-vertex count the flow kernel left in pcnt[p]; cleared for the
  // next iteration's boundary kernel
  const int32_t nm0 = A.pcnt[p];
  const int32_t n1w0 = A.pcnt[A.P + p];
  if (threadIdx.x == 0) {
    const fr_solve &rec = A.srec[p];
    sh.skip = (A.ps[p].done || A.ctl->err != 0 || rec.decision == FR_DEC_NOT_ADJACENT) ? 1 : 0;
    sh.nq = 0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    A.pcnt[p] = 0;
    A.pcnt[A.P + p] = 0;
  }
  if (sh.skip) return;
  const int64_t t0 = wall_clock64();
  const PairView V = make_view(A, p);
  const int32_t nr = uni(A.ps[p].nr);
  const int32_t nm = uni(min(nm0, nr));
  // per-entry statistics, by thread 0 at every exit
  auto done = [&](int64_t comps, int64_t big) {
    if (threadIdx.x == 0) {
      PairState &ps = A.ps[p];
      ps.mb_free += nm;
      ps.mb_comp += comps;
      ps.mb_big += big;
      ps.t_mb += wall_clock64() - t0;
    }
  };
  if (nm == 0) {
    done(0, 0);
    return;
  }
  int32_t *par = V.LA;        // [nr]: -1 outside M; class parent, later the component
  const int32_t *ml = V.LB;   // the free vertices M
  int32_t *w1 = A.mbq + A.aoff[p];  // one-way arcs inside M, then (device path) quotient arcs

  // ---- 1. (k_mb_union did the union-find and listed the one-way arcs)
  // compression (every free vertex points at its class root, the class's
  // smallest vertex) and the roots numbered as quotient nodes
  int32_t *qid = V.lab;  // [root] -> quotient node
  BLOCK_WAVE_LOOP(j, nm) {
    bool root = false;
    int32_t u = 0;
    if (j < nm) {
      u = ml[j];
      int32_t r = u;
      for (int32_t y = par[r]; y != r; y = par[r]) r = y;
      par[u] = r;
      root = r == u;
    }
    const int pos = wave_append(&sh.nq, root);
    if (root) qid[u] = pos;
  }
  __syncthreads();
  // ---- 2. quotient graph over the one-way arcs between classes
  const int32_t nq = uni(sh.nq), n1w = uni(n1w0);
  const bool lq = A.mb_lds && nq <= MB_LQ;
  int32_t *qoff = lq ? sh.u2.q.qoff : V.ex;
  for (int32_t q = threadIdx.x; q < nq; q += blockDim.x) qoff[q] = 0;
  __syncthreads();
  auto one_way = [&](int32_t j, auto &&f) {
    const Arc x = V.arc[w1[j]];
    const int32_t ru = par[V.arc[x.lr].lh], rv = par[x.lh];
    if (ru != rv) f(qid[ru], qid[rv]);
  };
  for (int32_t j = threadIdx.x; j < n1w; j += blockDim.x)
    one_way(j, [&](int32_t a, int32_t) { atomicAdd(qoff + a, 1); });
  __syncthreads();
  const int32_t eq = mb_exscan(qoff, nq, sh.red);
  if (threadIdx.x == 0) sh.eq = eq;
  // all of Q and Tarjan's scratch in LDS, or all in device memory
  const bool lt = lq && eq <= MB_LQA;
  if (lq && !lt) {
    for (int32_t q = threadIdx.x; q < nq; q += blockDim.x) V.ex[q] = qoff[q];
    __syncthreads();
    qoff = V.ex;
  }
  int32_t *qarc = lt ? sh.u2.q.qarc : w1 + n1w;  // eq <= n1w <= arc slots / 2
  int32_t *cur = lt ? sh.u1.t.cpos : V.SNK;
  for (int32_t q = threadIdx.x; q < nq; q += blockDim.x) cur[q] = qoff[q];
  __syncthreads();
  for (int32_t j = threadIdx.x; j < n1w; j += blockDim.x)
    one_way(j, [&](int32_t a, int32_t b) { qarc[atomicAdd(cur + a, 1)] = b; });
  __syncthreads();  // the arc records are dead from here on
  // ---- Tarjan on the quotient graph (its scratch: LDS, or the arc arena)
  int32_t *W = reinterpret_cast<int32_t *>(V.arc);
  int32_t *idx = lt ? sh.u2.q.qidx : W;
  for (int32_t q = threadIdx.x; q < nq; q += blockDim.x) idx[q] = -1;
  __syncthreads();
  if (threadIdx.x == 0) {
    if (lt) {
      sh.nc = mb_tarjan(nq, eq, sh.u2.q.qoff, sh.u2.q.qarc, sh.u2.q.qidx, sh.u1.t.low, sh.u1.t.stk,
                        sh.u1.t.cnode, sh.u1.t.cpos);
    } else if (nq > V.na) {  // cannot happen: nq <= corridor vertices <= arc slots
      A.ctl->err = FR_E_DEVICE;
      A.ctl->diag = DIAG_MB;
      sh.nc = -1;
    } else {
      sh.nc = mb_tarjan(nq, eq, V.ex, w1 + n1w, W, W + nq, W + 2 * (int64_t)nq,
                        W + 3 * (int64_t)nq, V.SNK);
    }
  }
  __syncthreads();
  const int32_t C = uni(sh.nc);
  if (C < 0) {
    done(0, 0);
    return;
  }
  // ---- 3. the component DAG: in LDS up to MB_LCOMP components, else in
  // device memory (then Tarjan ran there too, so nq > MB_LQ): weights, key
  // ids and arc ends in the entry's slice of mbc (4 words per vertex slot,
  // C <= nq <= corridor vertices), in-degrees in the label array once the
  // quotient-node ids it holds are dead, sink flags in the sink-list array
  const bool big = C > MB_LCOMP;
  int64_t *cw = sh.u1.c.cw;
  int32_t *ckey = sh.u1.c.ckey, *cend = sh.u1.c.cend, *cin = sh.u1.c.cin;
  uint8_t *sink = sh.u1.c.sink;
  if (big) {
    int32_t *X = A.mbc + 4 * A.voff[p];
    cw = reinterpret_cast<int64_t *>(X);
    ckey = X + 2 * (int64_t)C;
    cend = X + 3 * (int64_t)C;
    cin = V.lab;
    sink = reinterpret_cast<uint8_t *>(V.SNK);
  }
  for (int32_t c = threadIdx.x; c < C; c += blockDim.x) {
    cw[c] = 0;
    ckey[c] = 0x7fffffff;
    cend[c] = 0;
    if (!big) cin[c] = 0;
    sink[c] = 0;
  }
  __syncthreads();
  // every free vertex: its component (into par), the components' weights and
  // key ids; four vertices per lane with their loads issued together
  int64_t wfree = 0;
  for (int64_t b0 = (int64_t)(threadIdx.x & ~63u) * 4; b0 < nm; b0 += 4 * (int64_t)blockDim.x) {
    int32_t u[4], r[4], g[4], c[4];
    int64_t w[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const int64_t j = b0 + 64 * k + lane64();
      u[k] = j < nm ? ml[j] : -1;
    }
#pragma unroll
    for (int k = 0; k < 4; k++) {
      r[k] = u[k] >= 0 ? par[u[k]] : 0;
      g[k] = u[k] >= 0 ? V.lg[u[k]] : 0;
    }
#pragma unroll
    for (int k = 0; k < 4; k++) {
      c[k] = u[k] >= 0 ? -2 - idx[qid[r[k]]] : -1;
      w[k] = u[k] >= 0 ? A.vwgt[g[k]] : 0;
    }
#pragma unroll
    for (int k = 0; k < 4; k++) {
      if (u[k] >= 0) par[u[k]] = c[k];
      wfree += w[k];
      wave_add_by_key(reinterpret_cast<unsigned long long *>(cw), 1, 0, c[k], w[k]);
      wave_min_by_key(ckey, c[k], g[k]);
    }
  }
  if (big) {  // the quotient-node ids are dead: the label array takes the in-degrees
    __syncthreads();
    for (int32_t c = threadIdx.x; c < C; c += blockDim.x) cin[c] = 0;
    __syncthreads();
  }
  // component arcs, one lane per quotient arc (a hub class can own most of
  // them): its source node by binary search over the offsets
  auto qsrc = [&](int32_t e) {
    int32_t lo = 0, hi = nq;
    while (hi - lo > 1) {
      const int32_t mid = (lo + hi) >> 1;
      if (qoff[mid] <= e) lo = mid;
      else hi = mid;
    }
    return lo;
  };
  for (int32_t e = threadIdx.x; e < eq; e += blockDim.x) {
    const int32_t c = -2 - idx[qsrc(e)], d = -2 - idx[qarc[e]];
    if (d != c) {
      atomicAdd(&cend[c], 1);
      atomicAdd(&cin[d], 1);
    }
  }
  {
    int64_t s1[1] = {wfree};
    block_sums<1>(s1, sh.red);
    wfree = s1[0];
  }
  const int32_t ne = mb_exscan(cend, C, sh.red);
  // int16 component ids in LDS only for the small DAG
  const bool ladj = !big && A.mb_lds && ne <= MB_LDAG;
  int32_t *gadj = W + (lt ? 0 : nq);
  // fill: cend[c] counts up from c's start to its end
  for (int32_t e = threadIdx.x; e < eq; e += blockDim.x) {
    const int32_t c = -2 - idx[qsrc(e)], d = -2 - idx[qarc[e]];
    if (d != c) {
      const int32_t pos = atomicAdd(&cend[c], 1);
      if (ladj) sh.u1.c.adj[pos] = (int16_t)d;
      else gadj[pos] = d;
    }
  }
  __syncthreads();
  // ---- 4. sweeps, one per wave, in batches whose state fits: LDS for the
  // small DAG; for the large one the in-degrees go to the excess array
  // (quotient offsets, dead; nr >= C words per sweep) and the state bytes to
  // the Tarjan index array (dead; 4 nq >= 4 C bytes), which ends below the
  // component arcs at W + nq
  const fr_solve rec0 = A.srec[p];
  const int64_t wa0 = rec0.wa + wfree, wb0 = rec0.wb - wfree;  // all free components with s
  const uint64_t seed = (uint64_t)(uint32_t)A.mb_seed;
  int32_t *ind;
  uint8_t *stb;
  int32_t per;
  if (big) {
    per = max(1, min(MB_TPB / WAVE, min(nr / C, (int32_t)((4 * (int64_t)nq) / C))));
    ind = V.ex;
    stb = reinterpret_cast<uint8_t *>(W);
  } else {
    per = max(1, min(MB_TPB / WAVE, (int32_t)(MB_RS_BYTES / (5 * C))));
    ind = reinterpret_cast<int32_t *>(sh.u2.rs);
    stb = reinterpret_cast<uint8_t *>(ind + (int64_t)per * C);
  }
  if (ladj)
    mb_sweeps(A, sh, MBSweep<int16_t>{C, cin, cend, sh.u1.c.adj, cw, ckey, seed}, wa0, wb0, ind,
              stb, per, sink);
  else
    mb_sweeps(A, sh, MBSweep<int32_t>{C, cin, cend, gadj, cw, ckey, seed}, wa0, wb0, ind, stb,
              per, sink);
  // ---- 5. components left on the source side join S_min
  int64_t acc[2] = {0, 0};  // weight, vertices
  BLOCK_WAVE_LOOP(j, nm) {
    if (j < nm) {
      const int32_t u = ml[j];
      if (!sink[par[u]]) {
        V.ins[u] = 1;
        acc[0] += A.vwgt[V.lg[u]];
        acc[1] += 1;
      }
    }
  }
  block_sums<2>(acc, sh.red);
  if (threadIdx.x == 0) {
    fr_solve rec = A.srec[p];
    rec.wa += acc[0];
    rec.wb -= acc[0];
    rec.source_side += acc[1];
    const bool feas = rec.wa <= A.lmax && rec.wb <= A.lmax;
    rec.decision = !feas ? FR_DEC_INFEASIBLE
                         : (rec.cut_candidate < rec.cut_before ? FR_DEC_APPLY : FR_DEC_EQUAL);
    A.srec[p] = rec;
  }
  done(C, big ? 1 : 0);
}
