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
//      vertices share a component): the "bidirectional classes";
//   2. the quotient graph Q of the classes over the one-way residual arcs,
//      and Tarjan's SCC algorithm on Q in one lane (LDS when Q is small);
//   3. the component DAG (weights, key ids, in-degrees, arcs);
//   4. sweeps, one lane each: Kahn's algorithm taking the ready component
//      with the smallest SplitMix64 key moves components to the sink side
//      one by one, starting from the largest minimum source side; the first
//      most balanced cut is kept;
//   5. the chosen components join the source side; the solve's record gets
//      the new block weights and decision.
// The components and their reachability order are the same for every
// maximum flow or preflow, and the sweep order depends on nothing else, so
// the result equals that of any exact implementation of the same rule.
#pragma once
#include "fr_kernels.h"

#define MB_TPB 256
#define MB_LQ 1024        // quotient nodes handled in LDS
#define MB_LQA 1024       // quotient arcs handled in LDS
#define MB_LDAG 4096      // component arcs held in LDS
#define MB_RS_BYTES 20480 // per-lane sweep state (in-degrees and heaps)

struct MBShared {
  int64_t cw[FR_MB_MAX_COMP];      // component weights
  int32_t ckey[FR_MB_MAX_COMP];    // component key id: smallest global vertex id
  int32_t cend[FR_MB_MAX_COMP];    // component arcs: counts, then end offsets
  int32_t cin[FR_MB_MAX_COMP];     // in-degrees among the components
  int32_t qidx[MB_LQ];             // Tarjan index / component of each quotient node
  int16_t adj[MB_LDAG];            // component arcs (when they fit)
  uint8_t sink[FR_MB_MAX_COMP];    // chosen cut: component on the sink side
  union {
    struct {
      int32_t qoff[MB_LQ];         // quotient arcs: counts, then start offsets
      int32_t qarc[MB_LQA];
      int32_t low[MB_LQ], stk[MB_LQ], cnode[MB_LQ], cpos[MB_LQ];
    } t;
    uint32_t rs[MB_RS_BYTES / 4];
  } u;
  int64_t red[64];
  int64_t lane_bal[WAVE];
  int32_t lane_pos[WAVE];
  int64_t best_bal;
  int32_t best_rep, best_pos;
  int32_t nq, eq, nc, ne, skip;
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

// Binary min-heap of component ids ordered by their sweep keys.
struct MBHeap {
  int16_t *h;
  int32_t n;
  const int32_t *ckey;
  uint64_t seed;
  int32_t rep;
  __device__ __forceinline__ uint64_t key(int32_t c) const { return mb_key(seed, rep, ckey[c]); }
  __device__ void push(int32_t c) {
    int32_t i = n++;
    const uint64_t kc = key(c);
    while (i > 0) {
      const int32_t pa = (i - 1) >> 1;
      const int32_t cp = h[pa];
      if (key(cp) <= kc) break;
      h[i] = (int16_t)cp;
      i = pa;
    }
    h[i] = (int16_t)c;
  }
  __device__ int32_t pop() {
    const int32_t top = h[0];
    const int32_t last = h[--n];
    const uint64_t kl = key(last);
    int32_t i = 0;
    for (;;) {
      int32_t ch = 2 * i + 1;
      if (ch >= n) break;
      uint64_t kc = key(h[ch]);
      if (ch + 1 < n) {
        const uint64_t k2 = key(h[ch + 1]);
        if (k2 < kc) {
          ch++;
          kc = k2;
        }
      }
      if (kl <= kc) break;
      h[i] = h[ch];
      i = ch;
    }
    if (n > 0) h[i] = (int16_t)last;
    return top;
  }
};

// One sweep in one lane: Kahn's algorithm over the C components with the
// smallest key first; component j of the order moves to the sink side.
// wa/wb: block weights with every free component on the source side.
// Returns the first position with the smallest max(wa, wb) (0 = none moved)
// and its balance; with mark set, stops there and flags the moved components.
struct MBSweep {
  int32_t C;
  const int32_t *cin, *cend, *gadj;
  const int16_t *ladj;
  const int64_t *cw;
  const int32_t *ckey;
  uint64_t seed;
  __device__ __forceinline__ int32_t arc(int32_t e) const { return ladj ? ladj[e] : gadj[e]; }
  __device__ int32_t run(int32_t rep, int32_t *ind, int16_t *heap, int64_t wa, int64_t wb,
                         int32_t stop, uint8_t *mark, int64_t *best_out, Ctl *ctl) const {
    MBHeap H{heap, 0, ckey, seed, rep};
    for (int32_t c = 0; c < C; c++) {
      ind[c] = cin[c];
      if (ind[c] == 0) H.push(c);
    }
    int64_t best = wa > wb ? wa : wb;
    int32_t bj = 0;
    for (int32_t j = 1; j <= stop; j++) {
      if (H.n == 0) {  // a cycle among the components: cannot happen
        ctl->err = FR_E_DEVICE;
        ctl->diag = DIAG_MB;
        break;
      }
      const int32_t c = H.pop();
      if (mark) mark[c] = 1;
      wa -= cw[c];
      wb += cw[c];
      const int64_t bal = wa > wb ? wa : wb;
      if (bal < best) {
        best = bal;
        bj = j;
      }
      for (int32_t e = c ? cend[c - 1] : 0; e < cend[c]; e++) {
        const int32_t d = arc(e);
        if (--ind[d] == 0) H.push(d);
      }
    }
    *best_out = best;
    return bj;
  }
};

// Quotient-graph SCC (Tarjan 1972) in one lane: idx[q] = -1 unvisited,
// >= 0 visit index while on the component stack, -2 - c once in component c.
// Returns the number of components.
__device__ int32_t mb_tarjan(int32_t nq, int32_t eq, const int32_t *qoff, const int32_t *qarc,
                             int32_t *idx, int32_t *low, int32_t *stk, int32_t *cnode,
                             int32_t *cpos) {
  int32_t next = 0, ns = 0, nc = 0;
  for (int32_t root = 0; root < nq; root++) {
    if (idx[root] != -1) continue;
    int32_t depth = 0;
    cnode[0] = root;
    cpos[0] = qoff[root];
    idx[root] = low[root] = next++;
    stk[ns++] = root;
    while (depth >= 0) {
      const int32_t v = cnode[depth];
      const int32_t e = cpos[depth];
      const int32_t end = v + 1 < nq ? qoff[v + 1] : eq;
      if (e < end) {
        cpos[depth] = e + 1;
        const int32_t w = qarc[e];
        const int32_t iw = idx[w];
        if (iw == -1) {
          idx[w] = low[w] = next++;
          stk[ns++] = w;
          depth++;
          cnode[depth] = w;
          cpos[depth] = qoff[w];
        } else if (iw >= 0 && iw < low[v]) {
          low[v] = iw;
        }
        continue;
      }
      if (low[v] == idx[v]) {
        int32_t x;
        do {
          x = stk[--ns];
          idx[x] = -2 - nc;
        } while (x != v);
        nc++;
      }
      depth--;
      if (depth >= 0) {
        const int32_t u = cnode[depth];
        if (low[v] < low[u]) low[u] = low[v];
      }
    }
  }
  return nc;
}

__global__ void __launch_bounds__(MB_TPB) k_mb(KArgs A, int32_t it) {
  __shared__ MBShared sh;
  (void)it;
  const int32_t p = blockIdx.x;
  // the free-vertex count the flow kernel left in pcnt[p]; cleared for the
  // next iteration's boundary kernel
  const int32_t nm0 = A.pcnt[p];
  if (threadIdx.x == 0) {
    const fr_solve &rec = A.srec[p];
    sh.skip = (A.ps[p].done || A.ctl->err != 0 || rec.decision == FR_DEC_NOT_ADJACENT) ? 1 : 0;
    sh.nq = 0;
  }
  __syncthreads();
  if (threadIdx.x == 0) A.pcnt[p] = 0;
  if (sh.skip) return;
  const int64_t t0 = wall_clock64();
  const PairView V = make_view(A, p);
  const int32_t nr = uni(A.ps[p].nr);
  const int32_t nm = uni(min(nm0, nr));
  // per-entry statistics, by thread 0 at every exit
  auto done = [&](int64_t comps, int64_t limited) {
    if (threadIdx.x == 0) {
      PairState &ps = A.ps[p];
      ps.mb_free += nm;
      ps.mb_comp += comps;
      ps.mb_limited += limited;
      ps.t_mb += wall_clock64() - t0;
    }
  };
  if (nm == 0) {
    done(0, 0);
    return;
  }
  int32_t *par = V.LA;        // [nr]: -1 outside M; class parent, later the component
  const int32_t *ml = V.LB;   // the free vertices M

  // ---- 1. bidirectional classes
  for_groups<8>(nm, [&](int item, bool valid, int gl) {
    if (!valid) return;
    const int32_t u = ml[item];
    const int32_t e1 = V.lo[u + 1];
    for (int32_t e = V.lo[u] + gl; e < e1; e += 8) {
      const Arc x = V.arc[e];
      const int32_t v = x.lh;
      if (v > u && res_own(x.rc) > 0 && res_rev(x.rc) > 0 && par[v] >= 0) uf_union(par, u, v);
    }
  });
  __syncthreads();
  BLOCK_WAVE_LOOP(j, nm) {
    if (j < nm) {
      const int32_t u = ml[j];
      int32_t r = u;
      for (int32_t y = aload(par + r); y != r; y = aload(par + r)) r = y;
      par[u] = r;
    }
  }
  __syncthreads();
  // ---- 2. quotient graph: class roots numbered, one-way arcs between classes
  int32_t *qid = V.lab;  // [root] -> quotient node
  BLOCK_WAVE_LOOP(j, nm) {
    const bool root = j < nm && par[ml[j]] == ml[j];
    const int pos = wave_append(&sh.nq, root);
    if (root) qid[ml[j]] = pos;
  }
  __syncthreads();
  const int32_t nq = uni(sh.nq);
  const bool lq = A.mb_lds && nq <= MB_LQ;
  int32_t *qoff = lq ? sh.u.t.qoff : V.ex;
  for (int32_t q = threadIdx.x; q < nq; q += blockDim.x) qoff[q] = 0;
  __syncthreads();
  auto one_way = [&](int32_t u, bool valid, int gl, auto &&f) {
    if (!valid) return;
    const int32_t ru = par[u];
    const int32_t e1 = V.lo[u + 1];
    for (int32_t e = V.lo[u] + gl; e < e1; e += 8) {
      const Arc x = V.arc[e];
      const int32_t v = x.lh;
      if (res_own(x.rc) > 0 && res_rev(x.rc) == 0) {
        const int32_t rv = par[v];
        if (rv >= 0 && rv != ru) f(qid[ru], qid[rv]);
      }
    }
  };
  for_groups<8>(nm, [&](int item, bool valid, int gl) {
    one_way(valid ? ml[item] : 0, valid, gl, [&](int32_t a, int32_t) { atomicAdd(qoff + a, 1); });
  });
  __syncthreads();
  const int32_t eq = mb_exscan(qoff, nq, sh.red);
  if (threadIdx.x == 0) sh.eq = eq;
  const bool lqa = lq && eq <= MB_LQA;
  int32_t *qarc = lqa ? sh.u.t.qarc : A.mbq + A.aoff[p];
  int32_t *cur = lq ? sh.u.t.cpos : V.SNK;
  for (int32_t q = threadIdx.x; q < nq; q += blockDim.x) cur[q] = qoff[q];
  __syncthreads();
  for_groups<8>(nm, [&](int item, bool valid, int gl) {
    one_way(valid ? ml[item] : 0, valid, gl, [&](int32_t a, int32_t b) {
      qarc[atomicAdd(cur + a, 1)] = b;
    });
  });
  __syncthreads();  // the arc records are dead from here on
  // ---- Tarjan on the quotient graph (its scratch: LDS, or the arc arena,
  //      whose records are no longer read)
  int32_t *W = reinterpret_cast<int32_t *>(V.arc);
  int32_t *idx = lq ? sh.qidx : W;
  for (int32_t q = threadIdx.x; q < nq; q += blockDim.x) idx[q] = -1;
  __syncthreads();
  if (threadIdx.x == 0) {
    if (!lq && nq > V.na) {  // cannot happen: nq <= corridor vertices <= arc slots
      A.ctl->err = FR_E_DEVICE;
      A.ctl->diag = DIAG_MB;
      sh.nc = FR_MB_MAX_COMP + 1;
    } else {
      int32_t *low = lq ? sh.u.t.low : W + nq;
      int32_t *stk = lq ? sh.u.t.stk : W + 2 * (int64_t)nq;
      int32_t *cnode = lq ? sh.u.t.cnode : W + 3 * (int64_t)nq;
      int32_t *cpos = lq ? sh.u.t.cpos : V.SNK;
      sh.nc = mb_tarjan(nq, eq, qoff, qarc, idx, low, stk, cnode, cpos);
    }
  }
  __syncthreads();
  const int32_t C = uni(sh.nc);
  if (C > FR_MB_MAX_COMP) {  // too many components: the smallest source set stays
    done(C, 1);
    return;
  }
  // ---- 3. the component DAG
  for (int32_t c = threadIdx.x; c < C; c += blockDim.x) {
    sh.cw[c] = 0;
    sh.ckey[c] = 0x7fffffff;
    sh.cend[c] = 0;
    sh.cin[c] = 0;
    sh.sink[c] = 0;
  }
  __syncthreads();
  int64_t wfree = 0;
  BLOCK_WAVE_LOOP(j, nm) {
    if (j < nm) {
      const int32_t u = ml[j];
      const int32_t c = -2 - idx[qid[par[u]]];
      const int32_t g = V.lg[u];
      const int64_t w = A.vwgt[g];
      par[u] = c;
      wfree += w;
      atomicAdd((unsigned long long *)&sh.cw[c], (unsigned long long)w);
      atomicMin(&sh.ckey[c], g);
    }
  }
  for (int32_t q = threadIdx.x; q < nq; q += blockDim.x) {
    const int32_t c = -2 - idx[q];
    const int32_t end = q + 1 < nq ? qoff[q + 1] : eq;
    for (int32_t e = qoff[q]; e < end; e++) {
      const int32_t d = -2 - idx[qarc[e]];
      if (d != c) {
        atomicAdd(&sh.cend[c], 1);
        atomicAdd(&sh.cin[d], 1);
      }
    }
  }
  {
    int64_t s1[1] = {wfree};
    block_sums<1>(s1, sh.red);
    wfree = s1[0];
  }
  const int32_t ne = mb_exscan(sh.cend, C, sh.red);
  const bool ladj = A.mb_lds && ne <= MB_LDAG;
  int32_t *gadj = W + (lq ? 0 : nq);
  // fill: cend[c] counts up from c's start to its end
  for (int32_t q = threadIdx.x; q < nq; q += blockDim.x) {
    const int32_t c = -2 - idx[q];
    const int32_t end = q + 1 < nq ? qoff[q + 1] : eq;
    for (int32_t e = qoff[q]; e < end; e++) {
      const int32_t d = -2 - idx[qarc[e]];
      if (d != c) {
        const int32_t pos = atomicAdd(&sh.cend[c], 1);
        if (ladj) sh.adj[pos] = (int16_t)d;
        else gadj[pos] = d;
      }
    }
  }
  __syncthreads();
  // ---- 4. sweeps, one lane each, in batches that fit the LDS state
  const fr_solve rec0 = A.srec[p];
  const int64_t wa0 = rec0.wa + wfree, wb0 = rec0.wb - wfree;  // all free components with s
  const uint64_t seed = (uint64_t)(uint32_t)A.mb_seed;
  const MBSweep S{C, sh.cin, sh.cend, gadj, ladj ? sh.adj : nullptr, sh.cw, sh.ckey, seed};
  const int32_t per = max(1, min(WAVE, (int32_t)(MB_RS_BYTES / (6 * C))));
  if (threadIdx.x == 0) {
    sh.best_rep = -1;
    sh.best_pos = 0;
    sh.best_bal = 0;
  }
  for (int32_t r0 = 0; r0 < A.mb_reps; r0 += per) {
    const int32_t nl = min(per, A.mb_reps - r0);
    if (threadIdx.x < (unsigned)nl) {
      const int l = threadIdx.x;
      int32_t *ind = reinterpret_cast<int32_t *>(sh.u.rs) + (int64_t)l * C;
      int16_t *heap = reinterpret_cast<int16_t *>(reinterpret_cast<int32_t *>(sh.u.rs) +
                                                  (int64_t)nl * C) + (int64_t)l * C;
      int64_t bal;
      const int32_t j = S.run(r0 + l, ind, heap, wa0, wb0, C, nullptr, &bal, A.ctl);
      sh.lane_bal[l] = bal;
      sh.lane_pos[l] = j;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int l = 0; l < nl; l++)
        if (sh.best_rep < 0 || sh.lane_bal[l] < sh.best_bal) {
          sh.best_bal = sh.lane_bal[l];
          sh.best_rep = r0 + l;
          sh.best_pos = sh.lane_pos[l];
        }
    }
    __syncthreads();
  }
  // the chosen cut: replay the winning sweep up to its position
  if (threadIdx.x == 0 && sh.best_pos > 0) {
    int64_t bal;
    S.run(sh.best_rep, reinterpret_cast<int32_t *>(sh.u.rs),
          reinterpret_cast<int16_t *>(reinterpret_cast<int32_t *>(sh.u.rs) + C), wa0, wb0,
          sh.best_pos, sh.sink, &bal, A.ctl);
  }
  __syncthreads();
  // ---- 5. components left on the source side join S_min
  int64_t acc[2] = {0, 0};  // weight, vertices
  BLOCK_WAVE_LOOP(j, nm) {
    if (j < nm) {
      const int32_t u = ml[j];
      if (!sh.sink[par[u]]) {
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
  done(C, 0);
}
