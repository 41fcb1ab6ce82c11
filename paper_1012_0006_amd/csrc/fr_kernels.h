// Device code of libflowrefine: max-flow min-cut pair refinement
// (Sanders & Schulz, Section 4.1) for gfx950.
//
// A round refines the pairs of one quotient-graph matching.  Each pair owns
// W consecutive entries ("slots") that solve the current partition at the
// factors alpha, alpha/2, ... of its halving chain at once; an adaptive
// iteration of every entry is a chain of kernels:
//   k_iter_begin   compact the entries still iterating
//   k_bnd          pair boundary and cut (grid-wide over the pairs' unions)
//   k_corr         bounded BFS corridor (one workgroup per entry)
//   k_iter_mid     prefix sums of the corridor sizes
//   k_net_*        corridor network: arc counts, CSR offsets, arcs, reverse
//                  arcs and the initial preflow (grid-wide)
//   k_flow         global relabels, push/relabel passes, residual closure
//                  and the candidate's record (one workgroup per entry)
//   k_select       the adaptive rule over the finished slots, write-back of
//                  the applied candidate, factors of the next iteration
// Bulk scans use the whole chip; the latency-bound searches stay inside one
// workgroup, its LDS and its L1.  Kernel boundaries order every step, so no
// cross-XCD cache maintenance is needed.
//
// Pairs own disjoint blocks, hence disjoint vertices: their corridors and
// flows never touch, and every per-entry buffer is a slice of a shared arena
// sized by the pair's vertex and arc counts.  The slots of one pair share
// vertices and keep separate corridor marks.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "fr_internal.h"

#define WAVE 64

__device__ __forceinline__ int lane64() { return (int)__lane_id(); }

// A value every lane holds the same copy of (read from LDS after a barrier),
// moved to a scalar register so loop control and addresses built from it
// stay scalar.
__device__ __forceinline__ int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Append for lanes with want=true among the ACTIVE lanes of the wave: one
// atomic per wave on *counter (LDS or global).  Returns the slot or -1.
__device__ __forceinline__ int wave_append(int32_t *counter, bool want) {
  unsigned long long m = __ballot(want);
  if (m == 0ull) return -1;
  int leader = __ffsll((unsigned long long)m) - 1;
  int lane = lane64();
  int base = 0;
  if (lane == leader) base = atomicAdd(counter, (int)__popcll(m));
  base = __shfl(base, leader);
  int off = (int)__popcll(m & ((1ull << lane) - 1ull));
  return want ? base + off : -1;
}

// list[pos] = v when the slot exists; a slot beyond the capacity is a logic
// error and is recorded instead of written.
__device__ __forceinline__ void put_bounded(int32_t *list, int pos, int64_t cap, int32_t v,
                                            Ctl *ctl) {
  if (pos >= 0 && pos < cap) {
    list[pos] = v;
  } else if (pos >= 0) {
    ctl->err = FR_E_DEVICE;
    ctl->diag = DIAG_LIST;
  }
}

// Exclusive scan of one int64 per thread over the block; *total = the sum.
// lds holds blockDim.x/64 + 1 entries.  All threads call it.
__device__ int64_t block_exscan64(int64_t v, int64_t *total, int64_t *lds) {
  int lane = lane64(), w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int64_t x = v;
  for (int o = 1; o < WAVE; o <<= 1) {
    int64_t t = __shfl_up(x, o);
    if (lane >= o) x += t;
  }
  if (lane == WAVE - 1) lds[w] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t run = 0;
    for (int i = 0; i < nw; i++) {
      int64_t t = lds[i];
      lds[i] = run;
      run += t;
    }
    lds[nw] = run;
  }
  __syncthreads();
  int64_t res = lds[w] + x - v;
  *total = lds[nw];
  __syncthreads();
  return res;
}

// Sums of N int64 values over the block, returned in every thread
// (lds: 16*N entries).  All threads call it.
template <int N>
__device__ void block_sums(int64_t (&v)[N], int64_t *lds) {
  const int lane = lane64(), w = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int j = 0; j < N; j++) {
    int64_t x = v[j];
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    if (lane == 0) lds[w * N + j] = x;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < N; j++) {
    int64_t s = 0;
    for (int i = 0; i < nw; i++) s += lds[i * N + j];
    v[j] = s;
  }
  __syncthreads();
}

// wave-uniform block-stride iteration: every lane of a wave runs the same
// number of iterations (i may be out of range on the last one)
#define BLOCK_WAVE_LOOP(i, N)                                                              \
  for (int64_t _b = (int64_t)(threadIdx.x & ~63u); _b < (int64_t)(N); _b += blockDim.x) \
    for (int64_t i = _b + lane64(), _once = 1; _once; _once = 0)

// ------------------------------------------------------------------------
// setup kernels

// Adds v into base[key * stride + slot] for the active lanes with key >= 0,
// one atomic per distinct key of the wave (partitions of spatially ordered
// vertices give one or two keys per wave).  Converged wave only.
__device__ __forceinline__ void wave_add_by_key(unsigned long long *base, int stride, int slot,
                                                int key, int64_t v) {
  unsigned long long todo = __ballot(key >= 0);
  while (todo) {
    const int leader = __ffsll(todo) - 1;
    const int k0 = __shfl(key, leader);
    const bool mine = key == k0;
    int64_t x = mine ? v : 0;
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    if (lane64() == leader && x != 0)
      atomicAdd(&base[(int64_t)k0 * stride + slot], (unsigned long long)x);
    todo &= ~__ballot(mine);
  }
}

// Slot for every lane with key >= 0 in the list of its key: one atomic per
// distinct key of the wave.  Converged wave only.
__device__ __forceinline__ int wave_append_by_key(int32_t *counters, int key) {
  unsigned long long todo = __ballot(key >= 0);
  int slot = -1;
  const int lane = lane64();
  while (todo) {
    const int leader = __ffsll(todo) - 1;
    const int k0 = __shfl(key, leader);
    const unsigned long long m = __ballot(key == k0);
    int base = 0;
    if (lane == leader) base = atomicAdd(&counters[k0], (int)__popcll(m));
    base = __shfl(base, leader);
    if (key == k0) slot = base + (int)__popcll(m & ((1ull << lane) - 1ull));
    todo &= ~m;
  }
  return slot;
}

// Per-lane running sums of N per-pair quantities, added to their per-pair
// totals (dst[j][key * stride[j] + slot[j]]) only when the lane's pair
// changes and at the end, so a kernel over many items of few pairs issues few
// atomics.  Every lane of the wave calls add() and flush().
template <int N>
struct KeyedSums {
  int key = -1;
  int64_t v[N];
  __device__ KeyedSums() {
    for (int j = 0; j < N; j++) v[j] = 0;
  }
  template <typename Out>
  __device__ __forceinline__ void add(int k, const int64_t (&x)[N], Out &&out) {
    const bool change = key >= 0 && k >= 0 && k != key;
    if (__ballot(change)) {
      for (int j = 0; j < N; j++) out(j, change ? key : -1, v[j]);
      if (change)
        for (int j = 0; j < N; j++) v[j] = 0;
    }
    if (k >= 0) {
      key = k;
      for (int j = 0; j < N; j++) v[j] += x[j];
    }
  }
  template <typename Out>
  __device__ __forceinline__ void flush(Out &&out) {
    for (int j = 0; j < N; j++) out(j, key, v[j]);
  }
};

// Calls f for chunks of 64 consecutive vertices [u0, u0 + 64): each wave
// walks a contiguous run of chunks, so sums keyed by block or pair change key
// only at block borders and reach device memory a few times per wave.
// Workgroups are dispatched round-robin over the 8 XCDs, so workgroup g
// takes its runs from the (g mod 8)-th eighth of the vertex range, and
// neighbouring vertices (whose blocks the arcs look up) stay in one XCD's
// L2.  Wave-uniform; every wave of the grid calls it.
// f(u0, pv, x0) also gets the lane's vertex's block part[u] and arc start
// xadj[u] (-1 and INT32_MAX past the graph), loaded one chunk ahead so that
// their latency overlaps the previous chunk's work.
template <typename F>
__device__ __forceinline__ void wave_chunk_runs(const KArgs &A, F &&f) {
  const int64_t n = A.n;
  const int64_t nchunk = (n + 63) / 64;
  const int xcd = (int)(blockIdx.x % 8u);
  const int64_t nbx = ((int64_t)gridDim.x - xcd + 7) / 8;  // workgroups on this XCD
  const int64_t per = (nchunk + 7) / 8;
  const int wpb = (int)(blockDim.x >> 6);
  const int64_t r_lo = min(nchunk, xcd * per), r_hi = min(nchunk, (xcd + 1) * per);
  const int64_t nw = nbx * wpb;  // waves on this XCD
  const int64_t run = (r_hi - r_lo + nw - 1) / nw;
  const int64_t wi = (int64_t)(blockIdx.x / 8u) * wpb + (threadIdx.x >> 6);
  const int64_t c_lo = min(r_hi, r_lo + wi * run), c_hi = min(r_hi, c_lo + run);
  auto load = [&](int64_t c, int32_t &pv, int32_t &x0) {
    const int64_t u = c * 64 + lane64();
    const bool in = c < c_hi && u < n;
    pv = in ? A.part[u] : -1;
    x0 = in ? A.xadj[u] : 0x7fffffff;
  };
  int32_t pv, x0;
  load(c_lo, pv, x0);
  for (int64_t c = c_lo; c < c_hi; c++) {
    int32_t pn, xn;
    load(c + 1, pn, xn);
    f(c * 64, pv, x0);
    pv = pn;
    x0 = xn;
  }
}

// Boundary flag and cut weight of the 64 vertices of one chunk, one lane
// each: the lane's vertex has arcs [x0, the next lane's x0), the chunk's
// arcs are [E0, E1); with y2 >= 0 the vertex is a boundary vertex when a
// neighbour lies in block y2 >> 1, and its cut weight sums the weights of
// those arcs when y2 & 1 is 0 (lanes past the graph pass x0 = INT32_MAX and
// y2 = -1).  The arcs are read coalesced, KB per lane in flight; each finds
// its tail by a binary search over the lanes' range starts.  sb / scw: the
// wave's 64 LDS slots.
__device__ __forceinline__ void chunk_boundary(const KArgs &A, int32_t x0, int32_t y2, int32_t E0,
                                               int32_t E1, uint32_t *sb,
                                               unsigned long long *scw, bool &bnd,
                                               int64_t &cw) {
  const int lane = lane64();
  sb[lane] = 0u;
  scw[lane] = 0ull;
  constexpr int KB = 2;
  for (int32_t e0 = E0; e0 < E1; e0 += 64 * KB) {
    int32_t o[KB], ty[KB], v[KB];
#pragma unroll
    for (int q = 0; q < KB; q++) {
      const int32_t e = e0 + 64 * q + lane;
      int l = 0;
      for (int step = 32; step > 0; step >>= 1) {
        const int32_t t = __shfl(x0, l + step);
        if (t <= e) l += step;
      }
      o[q] = l;
      ty[q] = __shfl(y2, l);
      if (e >= E1) ty[q] = -1;
      v[q] = ty[q] >= 0 ? A.adjncy[e] : 0;
    }
#pragma unroll
    for (int q = 0; q < KB; q++) {
      const int32_t e = e0 + 64 * q + lane;
      if (ty[q] >= 0 && A.part[v[q]] == (ty[q] >> 1)) {
        atomicOr(&sb[o[q]], 1u);
        if (!(ty[q] & 1)) atomicAdd(&scw[o[q]], (unsigned long long)A.adjwgt[e]);
      }
    }
  }
  bnd = sb[lane] != 0u;
  cw = (int64_t)scw[lane];
}

// c(V), max c(v) and the range check of the partition (once per call).
__global__ void __launch_bounds__(256) k_graph_stats(KArgs A) {
  __shared__ int64_t s_red[16];
  int64_t sum = 0;
  int32_t mx = 0;
  int bad = 0;
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < A.n;
       u += (int64_t)gridDim.x * blockDim.x) {
    const int32_t w = A.vwgt[u];
    const int32_t x = A.part[u];
    sum += w;
    mx = w > mx ? w : mx;
    if (w < 0) bad |= 2;
    if (x < 0 || x >= A.k) bad |= 1;
  }
  int64_t v[1] = {sum};
  block_sums<1>(v, s_red);
  if (threadIdx.x == 0) atomicAdd((unsigned long long *)&A.ctl->cV, (unsigned long long)v[0]);
  for (int o = 32; o > 0; o >>= 1) {
    const int32_t t = __shfl_xor(mx, o);
    mx = t > mx ? t : mx;
  }
  if (lane64() == 0 && mx > 0) atomicMax((long long *)&A.ctl->maxc, (long long)mx);
  if (bad & 1) atomicOr(&A.ctl->bad_part, 1);
  if (bad & 2) atomicOr(&A.ctl->bad_graph, 1);
}

// Start of a round (one block): block -> pair map, cleared block statistics,
// union fill counters, pair queues, per-pair sums and list counters.
__global__ void __launch_bounds__(1024) k_round_init(KArgs A) {
  for (int i = threadIdx.x; i < A.k; i += blockDim.x) {
    A.blk2pair[i] = -1;
    A.binfo[2 * i] = -1;
    A.binfo[2 * i + 1] = 0;
  }
  for (int i = threadIdx.x; i < 3 * A.k; i += blockDim.x) A.bstat[i] = 0;
  for (int i = threadIdx.x; i < A.P; i += blockDim.x) A.ucnt[i] = 0;
  if (A.fstat)
    for (int i = threadIdx.x; i < 4 * A.P; i += blockDim.x) A.fstat[i] = 0;
  for (int i = threadIdx.x; i < 4 * A.max_iters; i += blockDim.x) A.queue[i] = 0;
  for (int i = threadIdx.x; i < A.P * PA_N; i += blockDim.x) A.pacc[i] = 0;
  for (int i = threadIdx.x; i < 2 * A.P; i += blockDim.x) A.pcnt[i] = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < A.P; i += blockDim.x) {
    if (i % A.W) continue;  // a pair's blocks map to its first entry
    A.blk2pair[A.pairs[2 * i]] = i;
    A.blk2pair[A.pairs[2 * i + 1]] = i;
  }
}

// Weight, vertex count and arc count of every block in a pair of the round.
__global__ void __launch_bounds__(256) k_block_stats(KArgs A) {
  unsigned long long *bw = (unsigned long long *)A.bstat;
  unsigned long long *bc = bw + A.k, *ba = bw + 2 * A.k;
  KeyedSums<3> sums;
  auto out = [&](int j, int key, int64_t v) {
    wave_add_by_key(j == 0 ? bw : (j == 1 ? bc : ba), 1, 0, key, v);
  };
  wave_chunk_runs(A, [&](int64_t u0, int32_t blk, int32_t x0) {
    const int64_t u = u0 + lane64();
    int key = -1;
    int32_t w = 0, deg = 0;
    if (blk >= 0 && A.blk2pair[blk] >= 0) {
      key = blk;
      w = A.vwgt[u];
      deg = A.xadj[u + 1] - x0;
    }
    const int64_t x[3] = {w, 1, deg};
    sums.add(key, x, out);
  });
  sums.flush(out);
}

// Arena slices (prefix sums of the pairs' vertex and arc counts), the
// largest-first order in which workgroups take the pairs, and the initial
// pair states.  One block.
__global__ void __launch_bounds__(1024) k_arena(KArgs A) {
  __shared__ int64_t s_scan[17];
  const int64_t *bw = A.bstat, *bc = A.bstat + A.k, *ba = A.bstat + 2 * A.k;
  const int P = A.P;
  const int per = (P + blockDim.x - 1) / blockDim.x;
  const int lo = threadIdx.x * per, hi = min(lo + per, P);
  int64_t sv = 0, sa = 0;
  for (int i = lo; i < hi; i++) {
    sv += bc[A.pairs[2 * i]] + bc[A.pairs[2 * i + 1]];
    sa += ba[A.pairs[2 * i]] + ba[A.pairs[2 * i + 1]];
  }
  int64_t tv, ta;
  int64_t rv = block_exscan64(sv, &tv, s_scan);
  int64_t ra = block_exscan64(sa, &ta, s_scan);
  for (int i = lo; i < hi; i++) {
    A.voff[i] = rv;
    A.aoff[i] = ra;
    rv += bc[A.pairs[2 * i]] + bc[A.pairs[2 * i + 1]];
    ra += ba[A.pairs[2 * i]] + ba[A.pairs[2 * i + 1]];
  }
  if (threadIdx.x == 0) {
    A.voff[P] = tv;
    A.aoff[P] = ta;
  }
  for (int i = threadIdx.x; i < P; i += blockDim.x) {
    const int32_t a = A.pairs[2 * i], b = A.pairs[2 * i + 1];
    const int64_t na = ba[a] + ba[b];
    int rank = 0;
    for (int q = 0; q < P; q++) {
      const int64_t nq = ba[A.pairs[2 * q]] + ba[A.pairs[2 * q + 1]];
      rank += (nq > na || (nq == na && q < i)) ? 1 : 0;
    }
    A.order[rank] = i;
    PairState s;
    memset(&s, 0, sizeof(s));
    s.a = a;
    s.b = b;
    int al = A.alpha0 ? A.alpha0[i - i % A.W] : 1;  // start factor: the pair's first entry
    al = al < 1 ? 1 : (al > A.alpha_max ? A.alpha_max : al);
    s.start_alpha = s.final_alpha = al;
    s.alpha = al >> (i % A.W);  // slot s solves at the s-th halving
    s.done = s.alpha < 1 ? 1 : 0;
    s.cA = bw[a];
    s.cB = bw[b];
    s.cut = s.cut0 = -1;
    A.ps[i] = s;
  }
}

// ---- input checks (every call unless switched off): offsets monotone, ids
//      in range, no self loop, no repeated neighbour, weights in [1, 2^30),
//      symmetric with equal weights.  A vertex with at most FR_VAL_HUB arcs is
//      checked by scanning its own list and its neighbours' lists.  A vertex
//      with more arcs ("hub") gets an open-addressing hash table of its
//      neighbours (key, weight): inserting finds its repeated neighbours, and
//      the reverse-arc check of every arc into it probes the table.  Work is
//      O(m FR_VAL_HUB) plus O(1) expected per hub arc, instead of O(sum deg^2).
#define FR_VAL_HUB 16

// table slots of a hub: a power of two at least twice its degree
__device__ __forceinline__ int64_t hub_slots(int64_t deg) {
  int64_t t = 64;
  while (t < 2 * deg) t <<= 1;
  return t;
}

__device__ __forceinline__ uint32_t hub_hash(int32_t key) {
  return (uint32_t)key * 2654435761u;  // Knuth's multiplicative hash
}

// degree of u when its offsets are well formed, else -1 (reported by k_validate)
__device__ __forceinline__ int64_t checked_degree(const KArgs &A, int64_t u, int64_t narcs) {
  const int32_t b = A.xadj[u], e = A.xadj[u + 1];
  if (b < 0 || e < b || e > narcs) return -1;
  return (int64_t)e - b;
}

// pass 1: table slots of all hubs (ctr[0] += slots)
__global__ void __launch_bounds__(256) k_val_hub_size(KArgs A, int64_t narcs,
                                                      unsigned long long *ctr) {
  unsigned long long acc = 0;
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < A.n;
       u += (int64_t)gridDim.x * blockDim.x) {
    const int64_t deg = checked_degree(A, u, narcs);
    if (deg > FR_VAL_HUB) acc += (unsigned long long)hub_slots(deg);
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if (lane64() == 0 && acc) atomicAdd(ctr, acc);
}

// pass 2: each hub's table offset (hdir, -1 for the other vertices), slots
// handed out by ctr[1]
__global__ void __launch_bounds__(256) k_val_hub_alloc(KArgs A, int64_t narcs, int64_t *hdir,
                                                       unsigned long long *ctr) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < A.n;
       u += (int64_t)gridDim.x * blockDim.x) {
    const int64_t deg = checked_degree(A, u, narcs);
    hdir[u] = deg > FR_VAL_HUB ? (int64_t)atomicAdd(ctr + 1, (unsigned long long)hub_slots(deg))
                               : -1;
  }
}

// pass 3: one wave per hub inserts its arcs (keys start at -1 = empty)
__global__ void __launch_bounds__(256) k_val_hub_insert(KArgs A, const int64_t *hdir,
                                                        int32_t *tkey, int32_t *tw) {
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t u = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); u < A.n;
       u += nw) {
    const int64_t off = hdir[u];
    if (off < 0) continue;
    const int32_t b = A.xadj[u], e = A.xadj[u + 1];
    const int64_t mask = hub_slots((int64_t)e - b) - 1;
    for (int32_t j = b + lane64(); j < e; j += 64) {
      const int32_t v = A.adjncy[j];
      if (v < 0) continue;  // out of range: reported by k_validate
      const int64_t h = (int64_t)(hub_hash(v) & (uint32_t)mask);
      for (int64_t q = 0; q <= mask; q++) {
        const int64_t slot = off + ((h + q) & mask);
        const int32_t old = atomicCAS(&tkey[slot], -1, v);
        if (old == -1) {
          tw[slot] = A.adjwgt[j];
          break;
        }
        if (old == v) {  // repeated neighbour
          atomicOr(&A.ctl->bad_graph, 1);
          break;
        }
      }
    }
  }
}

// The per-arc checks; hdir null: no hub tables (every list scanned).
__global__ void __launch_bounds__(256) k_validate(KArgs A, int64_t narcs, const int64_t *hdir,
                                                  const int32_t *tkey, const int32_t *tw) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < A.n;
       u += (int64_t)gridDim.x * blockDim.x) {
    const int32_t b = A.xadj[u], e = A.xadj[u + 1];
    if (b < 0 || e < b || e > narcs || (u == 0 && b != 0)) {
      atomicOr(&A.ctl->bad_graph, 1);
      continue;
    }
    const bool hub_u = hdir && hdir[u] >= 0;  // its repeats were checked on insertion
    for (int32_t j = b; j < e; j++) {
      const int32_t v = A.adjncy[j], w = A.adjwgt[j];
      bool ok = v >= 0 && v < A.n && v != (int32_t)u && w >= 1 && w < (1 << 30);
      for (int32_t q = b; ok && !hub_u && q < j; q++)
        if (A.adjncy[q] == v) ok = false;
      if (ok && hdir && hdir[v] >= 0) {
        // the reverse arc in v's table
        const int64_t off = hdir[v];
        const int64_t mask = hub_slots((int64_t)A.xadj[v + 1] - A.xadj[v]) - 1;
        const int64_t h = (int64_t)(hub_hash((int32_t)u) & (uint32_t)mask);
        bool found = false;
        for (int64_t q = 0; q <= mask; q++) {
          const int64_t slot = off + ((h + q) & mask);
          const int32_t key = tkey[slot];
          if (key == (int32_t)u) {
            found = tw[slot] == w;
            break;
          }
          if (key == -1) break;
        }
        ok = found;
      } else if (ok) {
        bool found = false;
        const int32_t vb = A.xadj[v], ve = A.xadj[v + 1];
        for (int32_t q = vb; q < ve && q < narcs && q >= 0; q++)
          if (A.adjncy[q] == (int32_t)u) {
            found = A.adjwgt[q] == w;
            break;
          }
        ok = found;
      }
      if (!ok) {
        atomicOr(&A.ctl->bad_graph, 1);
        break;
      }
    }
  }
}

// vertices of the two blocks of every pair, gathered into the pair's arena
__global__ void __launch_bounds__(256) k_union(KArgs A) {
  wave_chunk_runs(A, [&](int64_t u0, int32_t x, int32_t) {
    const int64_t u = u0 + lane64();
    const int32_t p = x >= 0 ? A.blk2pair[x] : -1;
    const int pos = wave_append_by_key(A.ucnt, p);
    if (p >= 0 && A.voff[p] + pos < A.voff[p + 1]) A.uvert[A.voff[p] + pos] = (int32_t)u;
  });
}

// ------------------------------------------------------------------------
// per-pair solver

// Shared-memory state of one workgroup.
// LDS working set of the flow phases: two vertex bitmaps (visited marks of
// the relabel and closure searches, queued marks of the sweeps) cover
// corridors of up to 32 * FR_BM_WORDS vertices; larger corridors use the
// global label / mark arrays instead.  The first FR_LDS_LIST entries of each
// frontier list live in LDS, the rest in the pair's global list.
#define FR_BM_WORDS 4096
#define FR_LDS_LIST 2048

template <int TPB>
struct SolveShared {
  union {
    unsigned long long hist[2048];  // radix select of the last BFS level
    struct {
      uint32_t bm[2][FR_BM_WORDS];
      int32_t ls[2][FR_LDS_LIST];
    } f;
  } u;
  int64_t red[16 * 8];            // block reductions
  int64_t scan[TPB / 64 + 1];
  int64_t W[2], U[2];             // BFS: taken weight and bound per side
  int64_t rarcs, rcap, rcin;      // corridor arcs, capacity sum, old a-b weight inside
  fr_solve rec;                   // record of the current solve
  unsigned long long work[W_COUNT];
  int32_t cnt[3];                 // rotating list counters
  int32_t nfree;                  // free vertices listed for the most balanced cut
  int32_t use_max;                // the candidate is the largest minimum source side
  int32_t nr;                     // corridor size
  int32_t nsnk;                   // sink-border vertices
  int32_t pair;                   // queue slot
  int32_t slice_end;              // the flow stops here until the next launch
  int32_t state[2];               // BFS: 1 = still expanding
  int32_t mode[2];                // BFS: level take mode (0 none, 1 all, 2 prefix)
  int32_t digit;
  int32_t stop;
  int64_t before;
};

// The last level of one side (block x) is cut in ascending id: find the first
// vertex y0 whose inclusive weight prefix exceeds R and mark every vertex of
// that side with id >= y0 as outside (S + 1).  Radix descent over the id bits
// in three passes (11 + 10 + 10 bits) with an LDS histogram of weights.
template <int TPB>
__device__ void cut_level(const KArgs &A, int32_t *mark, int32_t x, const int32_t *list,
                          int32_t cnt, int64_t R, int32_t S, SolveShared<TPB> &sh) {
  uint32_t prefix = 0, mask = 0;
  int64_t rem = R;
  for (int pass = 0; pass < 3; pass++) {
    const int shift = pass == 0 ? 20 : (pass == 1 ? 10 : 0);
    const int nbk = pass == 0 ? 2048 : 1024;
    for (int i = threadIdx.x; i < nbk; i += TPB) sh.u.hist[i] = 0ull;
    __syncthreads();
    for (int i = threadIdx.x; i < cnt; i += TPB) {
      const int32_t u = list[i];
      if (A.part[u] == x && ((uint32_t)u & mask) == prefix)
        atomicAdd(&sh.u.hist[((uint32_t)u >> shift) & (nbk - 1)],
                  (unsigned long long)(int64_t)A.vwgt[u]);
    }
    __syncthreads();
    const int per = (nbk + TPB - 1) / TPB;
    int64_t mine = 0;
    for (int j = 0; j < per; j++) {
      const int d = threadIdx.x * per + j;
      if (d < nbk) mine += (int64_t)sh.u.hist[d];
    }
    int64_t tot;
    int64_t before = block_exscan64(mine, &tot, sh.scan);
    if (threadIdx.x == 0) sh.digit = -1;
    __syncthreads();
    for (int j = 0; j < per; j++) {
      const int d = threadIdx.x * per + j;
      if (d >= nbk) break;
      const int64_t h = (int64_t)sh.u.hist[d];
      if (before <= rem && before + h > rem) {
        sh.digit = d;
        sh.before = before;
      }
      before += h;
    }
    __syncthreads();
    const int d = sh.digit;
    const int64_t bef = sh.before;
    __syncthreads();
    if (d < 0) return;  // the whole level fits
    rem -= bef;
    prefix |= (uint32_t)d << shift;
    mask |= (uint32_t)(nbk - 1) << shift;
  }
  const int32_t y0 = (int32_t)prefix;
  for (int i = threadIdx.x; i < cnt; i += TPB) {
    const int32_t u = list[i];
    if (A.part[u] == x && u >= y0) mark[u] = S + 1;
  }
  __syncthreads();
}

// Pointers into the arena slice of one pair.
struct PairView {
  int32_t a, b;
  int64_t nv, na;  // vertex / arc slots
  const int32_t *uv;
  int32_t *lg, *lo, *ex, *lab, *ins, *LA, *LB, *SNK;
  uint8_t *fl;
  Arc *arc;
};

// Residual pairs: each arc holds its own residual capacity in the low 32 bits
// and that of its reverse arc in the high 32 bits, so the backward searches
// read r(v -> w) at the arc w -> v.  A push of x along an arc adds
// (x << 32) - x to its pair and x - (x << 32) to the reverse arc's pair: no
// borrow or carry crosses the halves, as residuals stay in [0, 2^31).
__device__ __forceinline__ int32_t res_own(unsigned long long p) { return (int32_t)(uint32_t)p; }
__device__ __forceinline__ int32_t res_rev(unsigned long long p) { return (int32_t)(uint32_t)(p >> 32); }
__device__ __forceinline__ unsigned long long res_pair(int32_t own, int32_t rev) {
  return ((unsigned long long)(uint32_t)rev << 32) | (uint32_t)own;
}

// A frontier list: entries below ns in LDS (s), the rest in global memory (g).
struct ListRef {
  int32_t *g;
  int32_t *s;
  int32_t ns;
};

__device__ __forceinline__ int32_t lget(const ListRef &L, int32_t i) {
  return i < L.ns ? L.s[i] : L.g[i];
}

__device__ __forceinline__ void lput(const ListRef &L, int pos, int64_t cap, int32_t v, Ctl *ctl) {
  if (pos < L.ns) L.s[pos] = v;
  else put_bounded(L.g, pos, cap, v, ctl);
}

// Marks bit v of an LDS bitmap; true for the lane that set it first.
__device__ __forceinline__ bool bm_claim(uint32_t *bm, int32_t v) {
  const uint32_t bit = 1u << (v & 31);
  return (atomicOr(&bm[v >> 5], bit) & bit) == 0u;
}

// Work counters: every lane of the wave calls it with its count (0 for none);
// one LDS atomic per wave instead of one per item.
__device__ __forceinline__ void count_work_wave(unsigned long long *work, int slot, int32_t v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if (lane64() == 0 && v) atomicAdd(&work[slot], (unsigned long long)v);
}

// One push/relabel pass with T lanes per vertex over `cur` (lock-free:
// residuals and excess change by atomics; labels are read without
// synchronisation -- they only grow, and termination is decided by an exact
// global relabel).  Vertices that received flow and vertices still active go
// to `next`, each once: with an LDS bitmap (qbm, cleared) the first lane to
// mark a vertex queues it and every atomic is fire-and-forget; without one,
// the returning excess update (old value 0) decides.
template <int TPB, int T>
__device__ void pr_sweep(const KArgs &A, const PairView &V, const ListRef &cur, int32_t cnt,
                         const ListRef &next, int32_t *next_cnt, int32_t NL,
                         unsigned long long *wcnt, uint32_t *qbm) {
  const int lane = lane64();
  const int gl = lane & (T - 1);
  const int gid = threadIdx.x / T;
  constexpr int G = TPB / T;
  const int wave_first = (int)(threadIdx.x & ~63u) / T;
  for (int base = wave_first; base < cnt; base += G) {
    const int item = base + (gid - wave_first);
    const bool valid = item < cnt;
    const int32_t u = valid ? lget(cur, item) : 0;
    // the group leader reads label and excess once: excess may grow
    // concurrently, and every lane must push against the same value; the
    // arc range is read by all lanes at the same time
    // (contracted terminals: and the residual of u -> t, which only the
    // vertex's own discharge changes)
    int32_t d = NL, e = 0, rt = 0;
    if (valid && gl == 0) {
      d = V.lab[u];
      e = V.ex[u];
      if (A.terminals) rt = V.SNK[u];
    }
    int32_t ab = valid ? V.lo[u] : 0;
    int32_t ae = valid ? V.lo[u + 1] : 0;
    if (T > 1) {
      d = __shfl(d, 0, T);
      e = __shfl(e, 0, T);
      rt = __shfl(rt, 0, T);
    }
    const bool work = valid && d < NL && e > 0;
    if (!work) ab = ae = 0;
    int64_t erem = e, pushed = 0;
    // the arc to t first: always admissible (t is at label 0); once it is
    // saturated it takes no part in the relabel
    if (work && rt > 0) {
      const int32_t amt = e < rt ? e : rt;
      if (gl == 0) V.SNK[u] = rt - amt;
      erem -= amt;
      pushed += amt;
    }
    int32_t minres = 0x7fffffff;
    count_work_wave(wcnt, W_SWEEP_ITEMS, (work && gl == 0) ? 1 : 0);
    count_work_wave(wcnt, W_SWEEP_ARCS, (work && gl == 0) ? ae - ab : 0);
    // K chunks of T arcs per step: their loads are in flight together
    constexpr int K = T >= 8 ? 1 : 8 / T;
    int32_t h[K], r[K], ra[K], dh[K];
    // pushes along the arcs of the chunk at c0 that are admissible for label
    // dcur (residual left, head label below dcur), in arc order, until the
    // excess is used up; r[] keeps the residual left
    auto push_chunk = [&](int32_t c0, int32_t dcur) {
#pragma unroll
      for (int k = 0; k < K; k++) {
        const int32_t a = c0 + k * T + gl;
        const int64_t adm = (r[k] > 0 && dh[k] < dcur) ? (int64_t)r[k] : 0;
        int64_t inc = adm;
        if (T > 1) {
          for (int o = 1; o < T; o <<= 1) {
            const int64_t t = __shfl_up(inc, o, T);
            if (gl >= o) inc += t;
          }
        }
        const int64_t pre = inc - adm;
        const int64_t tot = T > 1 ? __shfl(inc, T - 1, T) : inc;
        int64_t amt = 0;
        if (adm > 0 && erem > pre) amt = adm < erem - pre ? adm : erem - pre;
        bool act = false;
        if (amt > 0) {
          const unsigned long long x = (unsigned long long)amt;
          atomicAdd(&V.arc[a].rc, (x << 32) - x);
          atomicAdd(&V.arc[ra[k]].rc, x - (x << 32));
          if (qbm) {
            atomicAdd(&V.ex[h[k]], (int32_t)amt);
            act = dh[k] > 0 && bm_claim(qbm, h[k]);
          } else {
            const int32_t old = atomicAdd(&V.ex[h[k]], (int32_t)amt);
            act = old == 0 && dh[k] > 0;
          }
        }
        const int pos = wave_append(next_cnt, act);
        if (act) lput(next, pos, V.nv, h[k], A.ctl);
        r[k] -= (int32_t)amt;
        const int64_t used = tot < erem ? tot : erem;
        erem -= used;
        pushed += used;
      }
    };
    for (int32_t c0 = ab; c0 < ae; c0 += T * K) {
#pragma unroll
      for (int k = 0; k < K; k++) {
        const int32_t a = c0 + k * T + gl;
        const bool in = a < ae;
        Arc x = {0, 0, 0ull};
        if (in) x = V.arc[a];
        h[k] = x.lh;
        r[k] = res_own(x.rc);
        ra[k] = x.lr;
      }
#pragma unroll
      for (int k = 0; k < K; k++) dh[k] = r[k] > 0 ? V.lab[h[k]] : 0x7fffffff;
      push_chunk(c0, d);
#pragma unroll
      for (int k = 0; k < K; k++)
        if (r[k] > 0 && dh[k] < minres) minres = dh[k];
    }
    if (T > 1) {
      for (int o = T >> 1; o > 0; o >>= 1) {
        const int32_t t = __shfl_xor(minres, o, T);
        minres = t < minres ? t : minres;
      }
    }
    // relabel to one above the lowest residual neighbour
    int32_t nd = d;
    if (work && erem > 0) {
      int64_t cand = minres == 0x7fffffff ? (int64_t)NL : (int64_t)minres + 1;
      if (cand > NL) cand = NL;
      if (cand > d) nd = (int32_t)cand;
    }
    if (work && gl == 0 && nd > d) V.lab[u] = nd;
    // discharge on: after a relabel the arcs to the lowest neighbours are
    // admissible; a vertex whose arcs fit one chunk still holds them
    const bool second = work && erem > 0 && nd > d && nd < NL && ae - ab <= T * K;
    if (__any(second)) push_chunk(ab, second ? nd : INT32_MIN);
    bool again = false;
    if (work && gl == 0) {
      if (qbm) {
        // flow pushed into u during this pass queued u already
        if (pushed > 0) atomicSub(&V.ex[u], (int32_t)pushed);
        again = e - pushed > 0 && nd < NL && bm_claim(qbm, u);
      } else {
        int64_t left = e;
        if (pushed > 0) left = (int64_t)atomicSub(&V.ex[u], (int32_t)pushed) - pushed;
        again = left > 0 && nd < NL;
      }
    }
    const int pos = wave_append(next_cnt, again);
    if (again) lput(next, pos, V.nv, u, A.ctl);
  }
}

template <int TPB>
__device__ void pr_sweep_any(const KArgs &A, const PairView &V, const ListRef &cur, int32_t cnt,
                             const ListRef &next, int32_t *next_cnt, int32_t NL,
                             unsigned long long *wcnt, uint32_t *qbm) {
  // Lanes per vertex: the tuning's value (1 and 16 run as 2 and 8), lowered
  // while the list would take more than one pass of the workgroup -- every
  // extra pass costs the whole chain of dependent loads and atomics again,
  // while 2 or 4 lanes still keep 8 arcs of a vertex in flight.  Results do
  // not depend on it.
  int t = A.tpv <= 2 ? 2 : (A.tpv == 4 ? 4 : 8);
  while (t > 2 && (int64_t)cnt * t > TPB) t >>= 1;
  if (t == 2) pr_sweep<TPB, 2>(A, V, cur, cnt, next, next_cnt, NL, wcnt, qbm);
  else if (t == 4) pr_sweep<TPB, 4>(A, V, cur, cnt, next, next_cnt, NL, wcnt, qbm);
  else pr_sweep<TPB, 8>(A, V, cur, cnt, next, next_cnt, NL, wcnt, qbm);
}

template <int TPB>
__device__ __forceinline__ void count_work(SolveShared<TPB> &sh, int slot, int32_t v) {
  count_work_wave(sh.work, slot, v);
}

// Rotating list counters: a phase appends into cnt[(c+1)%3] while thread 0
// clears cnt[(c+2)%3]; after the barrier c advances.  One barrier per phase.
struct Rot {
  int c = 0;
};

// Lanes per list item in the searches of the flow phases (relabel, closure):
// the arcs of one vertex are read by GTF lanes at once, each with KF arcs in
// flight, so a level costs a few dependent memory latencies, not one per arc.
#define GTF 4
#define KF 2

// Calls f(item, valid, gl) for list items 0..N-1, one group of G lanes per
// item; the trip count is uniform over each wave.
template <int G, typename F>
__device__ __forceinline__ void for_groups(int32_t N, F &&f) {
  const int gl = lane64() & (G - 1);
  const int wf = (int)(threadIdx.x & ~63u) / G;
  const int gid = (int)threadIdx.x / G;
  const int step = (int)blockDim.x / G;
  for (int base = wf; base < N; base += step) {
    const int item = base + (gid - wf);
    f(item, item < N, gl);
  }
}

// Lanes per item of a corridor BFS level: GTF while the level fits one pass
// of the workgroup, else 2, else 1 -- every extra pass would pay the level's
// chain of dependent loads again; each item keeps 8 arcs in flight at any
// width.  f(Lanes<G>) runs the level; results do not depend on G.  (The flow
// phases' searches keep GTF lanes: their levels are short, and one
// instantiation keeps that kernel within its registers.)
template <int G>
struct Lanes {
  static constexpr int g = G, k = 8 / G;
};

template <typename F>
__device__ __forceinline__ void by_width(int32_t cnt, F &&f) {
  if ((int64_t)cnt * GTF <= (int64_t)blockDim.x) f(Lanes<GTF>{});
  else if ((int64_t)cnt * 2 <= (int64_t)blockDim.x) f(Lanes<2>{});
  else f(Lanes<1>{});
}

// Sets the bitmap words of vertices 0..nr-1 to the ballot of pred(i) (one
// store per 32 vertices; words past nr come out 0).  All threads call it.
template <typename P>
__device__ __forceinline__ void bm_fill(uint32_t *bm, int32_t nr, P &&pred) {
  BLOCK_WAVE_LOOP(i, nr) {
    const bool on = i < nr && pred((int32_t)i);
    const unsigned long long m = __ballot(on);
    const int lane = lane64();
    if (lane == 0) bm[i >> 5] = (uint32_t)m;
    if (lane == 32) bm[i >> 5] = (uint32_t)(m >> 32);
  }
}

// Frontier lists of the flow phases: slot k (0/1) pairs the global list
// (LA/LB) with its LDS part when the bitmaps are in use.
template <int TPB>
__device__ __forceinline__ ListRef flist(const PairView &V, SolveShared<TPB> &sh, int k,
                                         bool lds) {
  ListRef L;
  L.g = k ? V.LB : V.LA;
  L.s = sh.u.f.ls[k];
  L.ns = lds ? FR_LDS_LIST : 0;
  return L;
}

// Exact distance labels: BFS from the sink backwards over residual arcs (v
// gets d+1 when the arc v -> w into a labelled w has residual capacity);
// unreached vertices keep NL and are inactive.  Pinned terminals: the BFS
// starts at the sink border (label 0).  Contracted terminals: it starts at the
// vertices whose arc to t has residual capacity left (label 1).  With lds set
// the visited marks are an LDS bitmap (bm[0]) and bm[1] is cleared for the
// sweeps; otherwise labels are claimed by compare-and-swap.  Leaves the
// active list (excess > 0, label < NL, not border) in list slot 0 and
// returns its size.
template <int TPB>
__device__ int32_t global_relabel(const KArgs &A, const PairView &V, int32_t nr, int32_t NL,
                                  SolveShared<TPB> &sh, Rot &R, int64_t &levels, bool lds) {
  uint32_t *vis = sh.u.f.bm[0];
  const bool term = A.terminals != 0;
  // start labels (sink border 0, source border NL + 1, the rest NL) and, with
  // the LDS bitmaps, visited = border and a cleared second bitmap: one pass,
  // four vertices per lane with their flags loaded together (contracted
  // terminals set no border flag: every label NL, nothing visited)
  for (int64_t b0 = (int64_t)(threadIdx.x & ~63u) * 4; b0 < nr; b0 += 4 * (int64_t)blockDim.x) {
    uint32_t f[4];
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const int64_t i = b0 + 64 * j + lane64();
      f[j] = i < nr ? V.fl[i] : 0u;
    }
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const int64_t i = b0 + 64 * j + lane64();
      if (i < nr) V.lab[i] = LF_SNK(f[j]) ? 0 : (LF_SRC(f[j]) ? NL + 1 : NL);
      if (lds) {
        const unsigned long long m = __ballot(i < nr && (f[j] & LF_BORDER));
        const int64_t w0 = (b0 + 64 * j) >> 5;  // 64-aligned: two bitmap words
        if (lane64() == 0) {
          vis[w0] = (uint32_t)m;
          sh.u.f.bm[1][w0] = 0u;
        }
        if (lane64() == 32) {
          vis[w0 + 1] = (uint32_t)(m >> 32);
          sh.u.f.bm[1][w0 + 1] = 0u;
        }
      }
    }
  }
  if (term) {
    // contracted terminals: the vertices with a residual arc to t start at
    // label 1, visited, listed in slot 1 as the first level.  This pass
    // splits the vertices over the waves differently from the one above, so
    // it waits for that one's label and bitmap stores first.
    __syncthreads();
    const ListRef start = flist(V, sh, 1, lds);
    int32_t *scnt = &sh.cnt[(R.c + 1) % 3];
    BLOCK_WAVE_LOOP(i, nr) {
      const bool first = i < nr && V.SNK[i] > 0;
      if (first) V.lab[i] = 1;
      if (lds) {
        const unsigned long long m = __ballot(first);
        if (lane64() == 0) vis[i >> 5] = (uint32_t)m;
        if (lane64() == 32) vis[i >> 5] = (uint32_t)(m >> 32);
      }
      const int pos = wave_append(scnt, first);
      if (first) lput(start, pos, V.nv, (int32_t)i, A.ctl);
    }
  }
  // the levels alternate between list slots 0 and 1: `nextl` takes the next
  // level, `spare` is the other slot; swapped each level (a slot chosen by a
  // run-time index would make the compiler keep both bases in scratch)
  ListRef cur, nextl = flist(V, sh, 0, lds), spare = flist(V, sh, 1, lds);
  int32_t cnt, lev;
  if (term) {
    if (threadIdx.x == 0) sh.cnt[(R.c + 2) % 3] = 0;
    __syncthreads();
    R.c = (R.c + 1) % 3;
    cur = spare;  // slot 1
    cnt = uni(min(sh.cnt[R.c], (int32_t)V.nv));
    lev = 1;
  } else {
    if (threadIdx.x == 0) sh.cnt[(R.c + 1) % 3] = 0;
    __syncthreads();
    cur.g = V.SNK;
    cur.s = nullptr;
    cur.ns = 0;
    cnt = uni(min(sh.nsnk, (int32_t)V.nv));
    lev = 0;
  }
  while (cnt > 0) {
    const ListRef next = nextl;
    int32_t *ncnt = &sh.cnt[(R.c + 1) % 3];
    const int32_t nl = lev + 1;
    for_groups<GTF>(cnt, [&](int item, bool valid, int gl) {
      const int32_t w = valid ? lget(cur, item) : 0;
      const int32_t e0 = valid ? V.lo[w] : 0, e1 = valid ? V.lo[w + 1] : 0;
      count_work(sh, W_GR_ITEMS, (valid && gl == 0) ? 1 : 0);
      count_work(sh, W_GR_ARCS, (valid && gl == 0) ? e1 - e0 : 0);
      for (int32_t c0 = e0; c0 < e1; c0 += GTF * KF) {
        int32_t v[KF], r[KF];
#pragma unroll
        for (int k = 0; k < KF; k++) {
          const int32_t a = c0 + k * GTF + gl;
          Arc x = {0, 0, 0ull};
          if (a < e1) x = V.arc[a];
          v[k] = x.lh;
          r[k] = res_rev(x.rc);
        }
#pragma unroll
        for (int k = 0; k < KF; k++) {
          bool claim = false;
          if (r[k] > 0) {
            if (lds) {
              const bool seen = (vis[v[k] >> 5] >> (v[k] & 31)) & 1u;
              if (!seen) {
                claim = bm_claim(vis, v[k]);
                if (claim) V.lab[v[k]] = nl;
              }
            } else if (V.lab[v[k]] == NL) {
              claim = atomicCAS(&V.lab[v[k]], NL, nl) == NL;
            }
          }
          const int pos = wave_append(ncnt, claim);
          if (claim) lput(next, pos, V.nv, v[k], A.ctl);
        }
      }
    });
    if (threadIdx.x == 0) sh.cnt[(R.c + 2) % 3] = 0;
    __syncthreads();
    R.c = (R.c + 1) % 3;
    cnt = uni(min(sh.cnt[R.c], (int32_t)V.nv));
    cur = next;
    nextl = spare;
    spare = next;
    lev++;
  }
  levels += lev;
  {
    const ListRef act_list = flist(V, sh, 0, lds);
    int32_t *ncnt = &sh.cnt[(R.c + 1) % 3];
    // active vertices, four per lane with their loads issued together
    for (int64_t b0 = (int64_t)(threadIdx.x & ~63u) * 4; b0 < nr; b0 += 4 * (int64_t)blockDim.x) {
      uint32_t f[4];
      int32_t e[4], l[4];
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const int64_t i = b0 + 64 * j + lane64();
        const bool in = i < nr;
        f[j] = in ? V.fl[i] : LF_BORDER;
        e[j] = in ? V.ex[i] : 0;
        l[j] = in ? V.lab[i] : NL;
      }
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const bool act = !(f[j] & LF_BORDER) && e[j] > 0 && l[j] < NL;
        const int pos = wave_append(ncnt, act);
        if (act) lput(act_list, pos, V.nv, (int32_t)(b0 + 64 * j + lane64()), A.ctl);
      }
    }
    if (threadIdx.x == 0) sh.cnt[(R.c + 2) % 3] = 0;
    __syncthreads();
    R.c = (R.c + 1) % 3;
  }
  return uni(min(sh.cnt[R.c], (int32_t)V.nv));
}

// ------------------------------------------------------------------------
// One adaptive flow iteration of every pair of a round is a chain of
// kernels: pair boundary (grid-wide), bounded BFS corridor (one workgroup
// per pair), network build (grid-wide, with a per-pair offset scan), then
// flow, closure, decision and factor update (one workgroup per pair).  The
// host enqueues the chain max_iters times; launch `it` performs solve `it` of
// every pair still iterating (all pairs start together and each solves once
// per launch), pairs that stopped are skipped.  Bulk scans over all vertices
// of the two blocks or of the corridor use the whole chip; the latency-bound
// searches stay inside one workgroup and its LDS.

// pair owning arena vertex slot i: voff[p] <= i < voff[p + 1]
__device__ __forceinline__ int32_t pair_of(const int64_t *voff, int32_t P, int64_t i) {
  int32_t lo = 0, hi = P;
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if (voff[mid] <= i) lo = mid;
    else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ PairView make_view(const KArgs &A, int32_t p) {
  PairView V;
  V.a = A.pairs[2 * p];
  V.b = A.pairs[2 * p + 1];
  const int64_t vb = A.voff[p];
  const int64_t ab = A.aoff[p];
  V.nv = A.voff[p + 1] - vb;
  V.na = A.aoff[p + 1] - ab;
  V.uv = A.uvert + vb;
  V.lg = A.lg + vb;
  V.lo = A.lo + vb + p;
  V.ex = A.ex + vb;
  V.lab = A.lab + vb;
  V.ins = A.ins + vb;
  V.LA = A.LA + vb;
  V.LB = A.LB + vb;
  V.SNK = A.SNK + vb;
  V.fl = A.lflag + vb;
  V.arc = A.arc + ab;
  return V;
}

// corridor marks and local ids of entry p (its slot's arrays)
// Corridor mark stamp of entry p's current iteration (two per iteration:
// S in the corridor, S + 1 cut off from it)
__device__ __forceinline__ int32_t stamp_of(const KArgs &A, int32_t p) {
  return A.stamp0 + 2 * A.ps[p].iter;
}
__device__ __forceinline__ int32_t *mark_of(const KArgs &A, int32_t p) {
  return A.mark + (int64_t)(p % A.W) * A.mstride;
}
__device__ __forceinline__ int32_t *vmap_of(const KArgs &A, int32_t p) {
  return A.vmap + (int64_t)(p % A.W) * A.mstride;
}

// Items of the compacted range of the live slots (pre = vpre or cpre), one
// lane each: f(p, item) with p the slot and item the offset inside it (p = -1
// past the end).  The wave's first item finds its slot by binary search, the
// other lanes step on from there (a wave's 64 items span few slots).  The
// trip count is uniform over each wave.
template <typename F>
__device__ __forceinline__ void grid_items(const KArgs &A, const int64_t *pre, F &&f) {
  const int32_t na = *A.nact;
  const int64_t N = pre[na];
  for (int64_t b0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) & ~(int64_t)63; b0 < N;
       b0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = b0 + lane64();
    int32_t p = -1;
    int64_t item = 0;
    if (i < N) {
      int32_t j = pair_of(pre, na, b0);
      while (pre[j + 1] <= i) j++;  // ends below na: i < pre[na]
      p = A.act[j];
      item = i - pre[j];
    }
    f(p, item);
  }
}

// Start of launch `it` (one block): the pairs still iterating, compacted in
// pair order, and the prefix sums of their union sizes.
__global__ void __launch_bounds__(1024) k_iter_begin(KArgs A, int32_t it) {
  __shared__ int64_t s_scan[17];
  const int P = A.P;
  // this launch's counters (a ring over max_iters launches): the corridor
  // and flow queues, the flow's running and started entries
  if (threadIdx.x < 4) A.queue[4 * (it % A.max_iters) + threadIdx.x] = 0;
  const int per = (P + blockDim.x - 1) / blockDim.x;
  const int lo = threadIdx.x * per, hi = min(lo + per, P);
  // the entries whose next corridor is due (the others are idle, or in a
  // solve that continues from an earlier launch)
  auto due = [&](int i) { return !A.ps[i].done && A.ps[i].phase == 0; };
  int64_t cnt = 0, sz = 0;
  for (int i = lo; i < hi; i++)
    if (due(i)) {
      cnt++;
      sz += A.voff[i + 1] - A.voff[i];
    }
  int64_t tc, ts;
  int64_t rc = block_exscan64(cnt, &tc, s_scan);
  int64_t rs = block_exscan64(sz, &ts, s_scan);
  for (int i = lo; i < hi; i++)
    if (due(i)) {
      A.act[rc] = i;
      A.vpre[rc] = rs;
      rc++;
      rs += A.voff[i + 1] - A.voff[i];
    }
  if (threadIdx.x == 0) {
    *A.nact = (int32_t)tc;
    A.vpre[tc] = ts;
  }
  // per block of the round: its pair's first entry while a slot's corridor
  // is due, the other block and the side (the boundary pass's lookup)
  for (int i = threadIdx.x; i < P; i += blockDim.x) {
    if (i % A.W) continue;
    bool live = false;
    for (int32_t s = 0; s < A.W; s++) live = live || due(i + s);
    const int32_t a = A.pairs[2 * i], b = A.pairs[2 * i + 1];
    A.binfo[2 * a] = live ? i : -1;
    A.binfo[2 * a + 1] = b << 1;
    A.binfo[2 * b] = live ? i : -1;
    A.binfo[2 * b + 1] = (a << 1) | 1;
  }
}

// After the corridor kernel (one block): prefix sums of the active pairs'
// corridor sizes.
__global__ void __launch_bounds__(1024) k_iter_mid(KArgs A, int32_t it) {
  __shared__ int64_t s_scan[17];
  (void)it;
  const int na = *A.nact;
  const int per = (na + blockDim.x - 1) / blockDim.x;
  const int lo = threadIdx.x * per, hi = min(lo + per, na);
  int64_t sz = 0;
  for (int j = lo; j < hi; j++) sz += A.ps[A.act[j]].nr;
  int64_t ts;
  int64_t rs = block_exscan64(sz, &ts, s_scan);
  for (int j = lo; j < hi; j++) {
    A.cpre[j] = rs;
    rs += A.ps[A.act[j]].nr;
  }
  if (threadIdx.x == 0) A.cpre[na] = ts;
}

#define PS_WORDS ((int)(sizeof(PairState) / 8))
#define PS_WORK (((int)offsetof(PairState, work)) / 8)
static_assert(sizeof(PairState) % 8 == 0, "PairState is summed as 8-byte words");

// Items 0..N-1 of entry p over the workgroup, one lane each: f(p, item), with
// p = -1 past the end; the trip count is uniform over each wave.
template <typename F>
__device__ __forceinline__ void pair_items(int32_t p, int64_t N, F &&f) {
  BLOCK_WAVE_LOOP(i, N) f(i < N ? p : -1, i < N ? i : (int64_t)0);
}

// The boundary pass over the union lists (vertices of a and b) of the entries
// that `items` hands out: f(p, slot) for union slot `slot` of entry p.
template <typename Items>
__device__ __forceinline__ void bnd_union(const KArgs &A, Items &&items) {
  unsigned long long *acc = (unsigned long long *)A.pacc;
  unsigned long long *psw = (unsigned long long *)A.ps;
  // pair cut, boundary weight a / b, boundary count a / b, vertices, arcs
  KeyedSums<7> sums;
  auto out = [&](int j, int key, int64_t v) {
    if (j < 5) wave_add_by_key(acc, PA_N, PA_CUT + j, key, v);
    else wave_add_by_key(psw, PS_WORDS, PS_WORK + (j == 5 ? W_BND_VERTS : W_BND_ARCS), key, v);
  };
  items([&](int32_t p, int64_t slot) {
    // one pass per pair: the first entry's (the other slots copy it)
    const bool on = p >= 0 && p % A.W == 0;
    const int32_t a = on ? A.pairs[2 * p] : 0, b = on ? A.pairs[2 * p + 1] : 0;
    // the union list is held by the pair's first entry
    const int32_t u = on ? A.uvert[A.voff[A.blk2pair[a]] + slot] : 0;
    const int side = on && A.part[u] == b;
    const int32_t y = side ? a : b;
    const int32_t e0 = on ? A.xadj[u] : 0, e1 = on ? A.xadj[u + 1] : 0;
    bool bnd = false;
    int64_t cw = 0;
    for (int32_t e = e0; e < e1; e++) {
      if (A.part[A.adjncy[e]] == y) {
        bnd = true;
        if (!side) cw += A.adjwgt[e];
      }
    }
    const bool bl = on && bnd;
    const int64_t w = bl ? A.vwgt[u] : 0;
    if (bl) mark_of(A, p)[u] = stamp_of(A, p);
    const int64_t x[7] = {cw, bl && !side ? w : 0, bl && side ? w : 0, bl && !side ? 1 : 0,
                          bl && side ? 1 : 0, 1, e1 - e0};
    sums.add(on ? p : -1, x, out);
    const int pos = wave_append_by_key(A.pcnt, bl ? p : -1);
    if (bl) put_bounded(A.SNK + A.voff[p], pos, A.voff[p + 1] - A.voff[p], u, A.ctl);
  });
  sums.flush(out);
}

// ---- pair boundary (Sec. 4.1): vertices of a with a neighbour in b and vice
//      versa become BFS level 0 (marked with the stamp S); also the pair cut
//      and the boundary weight and size per side.
//      Every slot of a pair solves the same partition, so the boundary is
//      computed once, for the pair's first entry: its sums, its marks and its
//      list (in the entry's SNK slice, which nothing reads before the network
//      build); each slot's corridor copies the list and marks it in its own
//      marks.  While the pairs still iterating cover a large part of the
//      graph, the kernel walks all vertices in chunks of 64 (coalesced arcs,
//      the pair from the block); late in a round, with few pairs left, it
//      walks only their union lists.
__global__ void __launch_bounds__(256) k_bnd(KArgs A, int32_t it) {
  (void)it;
  unsigned long long *acc = (unsigned long long *)A.pacc;
  unsigned long long *psw = (unsigned long long *)A.ps;
  const int64_t total = A.vpre[*A.nact];  // union items of the live slots
  if (4 * total >= (int64_t)A.n) {
    // pair cut, boundary weight a / b, boundary count a / b, vertices, arcs
    KeyedSums<7> sums;
    // keyed by the pair's first entry (live: binfo), which the other slots
    // copy from at the corridor's start
    auto out = [&](int j, int key, int64_t v) {
      if (j < 5) wave_add_by_key(acc, PA_N, PA_CUT + j, key, v);
      else wave_add_by_key(psw, PS_WORDS, PS_WORK + (j == 5 ? W_BND_VERTS : W_BND_ARCS), key, v);
    };
    // per lane of the block: boundary flag and cut weight of its vertex
    __shared__ uint32_t s_bnd[256];
    __shared__ unsigned long long s_cw[256];
    const int lane = lane64();
    const int wl = (int)(threadIdx.x & ~63u);
    wave_chunk_runs(A, [&](int64_t u0, int32_t pv, int32_t x0) {
      const int64_t u = u0 + lane;
      const int64_t last = min((int64_t)A.n, u0 + 64);
      const bool in = u < last;
      // the vertex's block -> its pair's first live entry, the other block
      // and the side (binfo, set at the start of every iteration)
      int32_t p0 = -1, y2 = -1;
      if (in) {
        p0 = A.binfo[2 * pv];
        y2 = A.binfo[2 * pv + 1];
      }
      if (p0 < 0) y2 = -1;
      const int32_t E1 = A.xadj[last];
      // the next lane's arc start, shuffled by the whole wave (a lane that
      // reads an inactive lane gets 0)
      const int32_t xn = __shfl(x0, (lane + 1) & 63);
      const int32_t x1 = u + 1 < last ? xn : E1;
      bool bnd;
      int64_t cw;
      chunk_boundary(A, x0, y2, __shfl(x0, 0), E1, s_bnd + wl, s_cw + wl, bnd, cw);
      const bool bl = p0 >= 0 && bnd;
      const int side = y2 & 1;
      const int64_t w = bl ? A.vwgt[u] : 0;
      const int64_t x[7] = {cw, bl && !side ? w : 0, bl && side ? w : 0, bl && !side ? 1 : 0,
                            bl && side ? 1 : 0, 1, in ? x1 - x0 : 0};
      sums.add(p0, x, out);
      const int32_t p = bl ? p0 : -1;
      if (p >= 0) mark_of(A, p)[u] = stamp_of(A, p);
      const int pos = wave_append_by_key(A.pcnt, p);
      if (p >= 0) put_bounded(A.SNK + A.voff[p], pos, A.voff[p + 1] - A.voff[p], (int32_t)u, A.ctl);
    });
    sums.flush(out);
    return;
  }
  bnd_union(A, [&](auto &&f) { grid_items(A, A.vpre, f); });
}

// Takes the next pair of the queue for launch `it`; -1 when the queue is
// empty.  Pairs that stopped are skipped.  All threads call it.
// Entries in the phase `upto` or below qualify: 0 for a corridor that is
// due, 1 for a flow that starts or continues.
template <int TPB>
__device__ __forceinline__ int32_t next_pair(const KArgs &A, int32_t *queue,
                                             SolveShared<TPB> &sh, int32_t upto) {
  for (;;) {
    if (threadIdx.x == 0) sh.pair = atomicAdd(queue, 1);
    __syncthreads();
    const int32_t q = uni(sh.pair);
    __syncthreads();
    if (q >= A.P) return -1;
    const int32_t p = uni(A.order[q]);
    if (!A.ps[p].done && A.ps[p].phase <= upto) return p;
  }
}

// ---- bounded BFS corridor (Sec. 4.1): level-synchronous on both sides from
//      the boundary; a level that crosses the side's area bound is cut in
//      ascending vertex id.  Taken vertices get local ids (lg, vmap).
template <int TPB>
__device__ __forceinline__ void corr_pair(const KArgs &A, int32_t S, int32_t p, SolveShared<TPB> &sh,
                          PairState &st) {
  const PairView V = make_view(A, p);
  const int32_t a = V.a, b = V.b;
  int32_t *mk = mark_of(A, p), *vm = vmap_of(A, p);
  // the boundary pass ran once per pair, for its first entry p0: its sums,
  // and its list in p0's SNK slice (untouched until the network build)
  const int32_t p0 = p - p % A.W;
  const int64_t *pa = A.pacc + (int64_t)p0 * PA_N;
  int64_t t0 = wall_clock64();
  if (threadIdx.x == 0) {
    st = A.ps[p];
    sh.cnt[0] = min(A.pcnt[p0], (int32_t)V.nv);
    sh.cnt[1] = sh.cnt[2] = 0;
    sh.nr = 0;
    sh.W[0] = sh.W[1] = 0;
    sh.state[0] = sh.state[1] = 1;
    const int64_t base = A.base[st.alpha];
    sh.U[0] = base - st.cB > 0 ? base - st.cB : 0;
    sh.U[1] = base - st.cA > 0 ? base - st.cA : 0;
    if (st.cut0 < 0) st.cut0 = pa[PA_CUT];
    st.cut = pa[PA_CUT];
  }
  if (threadIdx.x < W_COUNT) sh.work[threadIdx.x] = 0ull;
  __syncthreads();
  {
    // level 0: the pair's boundary list into this entry's list, the other
    // slots also marking it in their own corridor marks (the first entry's
    // marks were set by the boundary pass)
    const int32_t *bl = A.SNK + A.voff[p0];
    const int32_t n0 = uni(sh.cnt[0]);
    for (int32_t i = threadIdx.x; i < n0; i += TPB) {
      const int32_t u = bl[i];
      V.LA[i] = u;
      if (p != p0) mk[u] = S;
    }
    __syncthreads();
  }
  int64_t Lw[2] = {pa[PA_BW0], pa[PA_BW1]}, Lc[2] = {pa[PA_BC0], pa[PA_BC1]};
  int32_t *cur = V.LA, *nxt = V.LB;
  int cc = 0;  // counter of the current list
  for (int32_t lev = 0;; lev++) {
    const int32_t cnt = uni(min(sh.cnt[cc], (int32_t)V.nv));
    if (threadIdx.x == 0) {
      for (int s = 0; s < 2; s++) {
        sh.mode[s] = 0;
        if (!sh.state[s]) continue;
        if (Lc[s] == 0) {
          sh.state[s] = 0;
          continue;
        }
        if (A.area_mode == FR_AREA_DEPTH) {
          sh.mode[s] = 1;
          sh.W[s] += Lw[s];
          if (lev >= A.depth) sh.state[s] = 0;
        } else if (sh.W[s] + Lw[s] <= sh.U[s]) {
          sh.mode[s] = 1;
          sh.W[s] += Lw[s];
        } else {
          sh.mode[s] = 2;  // the bound is crossed inside this level
          sh.state[s] = 0;
        }
      }
      sh.cnt[(cc + 1) % 3] = 0;
      st.bfs_levels += 1;
    }
    __syncthreads();
    for (int s = 0; s < 2; s++)
      if (sh.mode[s] == 2) cut_level<TPB>(A, mk, s ? b : a, cur, cnt, sh.U[s] - sh.W[s], S, sh);
    // the taken part of this level joins the corridor
    BLOCK_WAVE_LOOP(i, cnt) {
      bool take = false;
      int32_t u = 0;
      if (i < cnt) {
        u = cur[i];
        const int s = A.part[u] == b;
        take = sh.mode[s] == 1 || (sh.mode[s] == 2 && mk[u] == S);
      }
      const int pos = wave_append(&sh.nr, take);
      if (take) {
        put_bounded(V.lg, pos, V.nv, u, A.ctl);
        vm[u] = pos;
      }
    }
    if (!sh.state[0] && !sh.state[1]) break;
    // expand the sides that go on
    int64_t acc2[4] = {0, 0, 0, 0};  // weight a, weight b, count a, count b
    int32_t *ncnt = &sh.cnt[(cc + 1) % 3];
    // GTF lanes per frontier vertex, KF arcs per lane: the neighbours'
    // block, mark and weight are loaded together, ahead of the claims
    by_width(cnt, [&](auto L) {
      constexpr int GW = decltype(L)::g, KW = decltype(L)::k;
      for_groups<GW>(cnt, [&](int item, bool valid, int gl) {
        const int32_t u = valid ? cur[item] : 0;
        const int32_t x = valid ? A.part[u] : -1;
        const int32_t e0 = valid ? A.xadj[u] : 0, e1 = valid ? A.xadj[u + 1] : 0;
        const int s = x == b;
        const bool go = valid && sh.state[s];
        count_work(sh, W_BFS_ITEMS, (go && gl == 0) ? 1 : 0);
        count_work(sh, W_BFS_ARCS, (go && gl == 0) ? e1 - e0 : 0);
        const int32_t ee = go ? e1 : e0;
        for (int32_t c0 = e0; c0 < ee; c0 += GW * KW) {
          int32_t v[KW], xv[KW], mv[KW], wv[KW];
#pragma unroll
          for (int k = 0; k < KW; k++) {
            const int32_t e = c0 + k * GW + gl;
            v[k] = e < ee ? A.adjncy[e] : -1;
          }
#pragma unroll
          for (int k = 0; k < KW; k++) {
            xv[k] = v[k] >= 0 ? A.part[v[k]] : -1;
            mv[k] = v[k] >= 0 ? mk[v[k]] : S;
            wv[k] = v[k] >= 0 ? A.vwgt[v[k]] : 0;
          }
#pragma unroll
          for (int k = 0; k < KW; k++) {
            bool claim = false;
            if (v[k] >= 0 && xv[k] == x && mv[k] < S) claim = atomicMax(&mk[v[k]], S) < S;
            const int pos = wave_append(ncnt, claim);
            if (claim) {
              put_bounded(nxt, pos, V.nv, v[k], A.ctl);
              acc2[s] += wv[k];
              acc2[2 + s] += 1;
            }
          }
        }
      });
    });
    block_sums<4>(acc2, sh.red);
    Lw[0] = acc2[0];
    Lw[1] = acc2[1];
    Lc[0] = acc2[2];
    Lc[1] = acc2[3];
    int32_t *t = cur;
    cur = nxt;
    nxt = t;
    cc = (cc + 1) % 3;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    st.nr = min(sh.nr, (int32_t)V.nv);
    for (int j = 0; j < W_COUNT; j++) st.work[j] += (int64_t)sh.work[j];
    st.t_corridor += wall_clock64() - t0;
    A.ps[p] = st;
  }
  __syncthreads();
}

template <int TPB>
__global__ void __launch_bounds__(TPB) k_corr(KArgs A, int32_t it) {
  __shared__ SolveShared<TPB> sh;
  __shared__ PairState st;
  for (;;) {
    const int32_t p = next_pair<TPB>(A, A.queue + 4 * (it % A.max_iters), sh, 0);
    if (p < 0) break;
    corr_pair<TPB>(A, stamp_of(A, p), p, sh, st);
  }
}

// ---- corridor network G' (Sec. 4.1), pass 1: arcs of each corridor vertex
//      inside the corridor (edges of G[B], capacity omega both ways), border
//      flag (a neighbour in A u B outside the corridor: merged into s or t).
//      With contracted terminals no vertex is pinned: the weight into a
//      outside the corridor is the capacity of s -> u (written as u's initial
//      excess), the weight into b outside that of u -> t (written to SNK),
//      and the old a-b edges with one end outside count as decided too.
template <typename Items>
__device__ __forceinline__ void net_count(const KArgs &A, Items &&items) {
  const bool term = A.terminals != 0;
  unsigned long long *acc = (unsigned long long *)A.pacc;
  unsigned long long *psw = (unsigned long long *)A.ps;
  // corridor arcs, capacity sum, decided old a-b weight, vertices, arcs
  // scanned, capacity out of s
  KeyedSums<6> sums;
  auto out = [&](int j, int key, int64_t v) {
    if (j < 3) wave_add_by_key(acc, PA_N, PA_RARCS + j, key, v);
    else if (j == 5) wave_add_by_key(acc, PA_N, PA_CS, key, v);
    else wave_add_by_key(psw, PS_WORDS, PS_WORK + (j == 3 ? W_NET_VERTS : W_NET_ARCS), key, v);
  };
  items([&](int32_t p, int64_t item) {
    const int64_t i = p >= 0 ? A.voff[p] + item : 0;  // arena slot
    const bool on = p >= 0;
    const int32_t a = on ? A.pairs[2 * p] : 0, b = on ? A.pairs[2 * p + 1] : 0;
    const int32_t u = on ? A.lg[i] : 0;
    const int side = on && A.part[u] == b;
    const int32_t *mk = on ? mark_of(A, p) : A.mark;
    const int32_t S = on ? stamp_of(A, p) : 0;
    const int32_t e0 = on ? A.xadj[u] : 0, e1 = on ? A.xadj[u + 1] : 0;
    int64_t cnt = 0, cap = 0, cin = 0, cs = 0, ct = 0;
    bool border = false;
    for (int32_t e = e0; e < e1; e++) {
      const int32_t v = A.adjncy[e];
      const int32_t xv = A.part[v];
      if (xv != a && xv != b) continue;
      if (mk[v] == S) {
        cnt++;
        cap += A.adjwgt[e];
        if (!side && xv == b) cin += A.adjwgt[e];
      } else {
        border = true;
        if (xv == a) cs += A.adjwgt[e];
        else ct += A.adjwgt[e];
        if (term && xv != (side ? b : a)) cin += A.adjwgt[e];
      }
    }
    border = border && !term;
    if (term) cap += cs + ct;
    else cs = 0;
    const bool lead = on;
    if (lead) {
      A.lo[i + p + 1] = (int32_t)cnt;  // the pair's offsets start at voff[p] + p
      A.lflag[i] = (uint8_t)((side ? LF_SIDE_B : 0u) | (border ? LF_BORDER : 0u));
      if (term) {  // clamped: past 2^31 the pair reports FR_E_OVERFLOW before any use
        A.ex[i] = (int32_t)min<int64_t>(cs, 0x7fffffffLL);
        A.SNK[i] = (int32_t)min<int64_t>(ct, 0x7fffffffLL);
      }
    }
    const int64_t x[6] = {cnt, cap, cin, 1, e1 - e0, cs};
    sums.add(lead ? p : -1, x, out);
  });
  sums.flush(out);
}

__global__ void __launch_bounds__(256) k_net_count(KArgs A, int32_t it) {
  (void)it;
  net_count(A, [&](auto &&f) { grid_items(A, A.cpre, f); });
}

// pass 2 (one block per pair): inclusive scan of the arc counts into CSR
// offsets, 4 values per thread per tile
// s_scan: blockDim.x / 64 + 1 LDS words.  All threads call it.
__device__ __forceinline__ void net_scan_pair(const KArgs &A, int32_t p, int64_t *s_scan) {
  const int32_t nr = uni(A.ps[p].nr);
  int32_t *lo = A.lo + A.voff[p] + p;
  int64_t carry = 0;
  const int tile = 4 * (int)blockDim.x;
  for (int32_t t0 = 0; t0 < nr; t0 += tile) {
    const int32_t i0 = t0 + 4 * (int)threadIdx.x;
    int32_t v[4];
    int64_t mine = 0;
#pragma unroll
    for (int j = 0; j < 4; j++) {
      v[j] = i0 + j < nr ? lo[i0 + j + 1] : 0;
      mine += v[j];
    }
    int64_t tot;
    int64_t run = carry + block_exscan64(mine, &tot, s_scan);
#pragma unroll
    for (int j = 0; j < 4; j++) {
      run += v[j];
      if (i0 + j < nr) lo[i0 + j + 1] = (int32_t)run;
    }
    carry += tot;
  }
  if (threadIdx.x == 0) {
    lo[0] = 0;
    A.ps[p].last_nr = nr;
  }
}

__global__ void __launch_bounds__(1024) k_net_scan(KArgs A, int32_t it) {
  __shared__ int64_t s_scan[17];
  (void)it;
  const int32_t p = blockIdx.x;
  if (p >= A.P || A.ps[p].done || A.ps[p].phase != 0) return;
  net_scan_pair(A, p, s_scan);
}

// pass 3: arcs (local head and capacity) in the order of the global adjacency
template <typename Items>
__device__ __forceinline__ void net_fill(const KArgs &A, Items &&items) {
  items([&](int32_t p, int64_t item) {
    if (p < 0) return;
    const int32_t S = stamp_of(A, p);
    const int64_t i = A.voff[p] + item;  // arena slot
    const int32_t a = A.pairs[2 * p], b = A.pairs[2 * p + 1];
    const int32_t u = A.lg[i];
    const int32_t *mk = mark_of(A, p);
    const int32_t *vm = vmap_of(A, p);
    const int32_t e0 = A.xadj[u], e1 = A.xadj[u + 1];
    const int64_t ab = A.aoff[p];
    const int64_t na = A.aoff[p + 1] - ab;
    int32_t k = A.lo[i + p];
    // four arcs per step, their loads issued together
    for (int32_t c = e0; c < e1; c += 4) {
      int32_t v[4], w[4], xv[4], mv[4];
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const bool in = c + q < e1;
        v[q] = in ? A.adjncy[c + q] : 0;
        w[q] = in ? A.adjwgt[c + q] : 0;
      }
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const bool in = c + q < e1;
        xv[q] = in ? A.part[v[q]] : -1;
        mv[q] = in ? mk[v[q]] : S - 1;
      }
#pragma unroll
      for (int q = 0; q < 4; q++) {
        if ((xv[q] == a || xv[q] == b) && mv[q] == S) {
          if (k < na) {
            Arc &x = A.arc[ab + k];
            x.lh = vm[v[q]];
            x.rc = res_pair(w[q], w[q]);
          }
          k++;
        }
      }
    }
  });
}

__global__ void __launch_bounds__(256) k_net_fill(KArgs A, int32_t it) {
  (void)it;
  net_fill(A, [&](auto &&f) { grid_items(A, A.cpre, f); });
}

// pass 4: reverse arcs, the initial preflow (every arc out of the source
// border is saturated), cleared closure marks, the sink list
template <typename Items>
__device__ __forceinline__ void net_rev(const KArgs &A, Items &&items) {
  items([&](int32_t p, int64_t item64) {
    const bool on = p >= 0;
    const int32_t item = (int32_t)item64;
    bool overflow = false;
    int64_t vb = 0, ab = 0;
    if (on) {
      overflow = A.pacc[(int64_t)p * PA_N + PA_RCAP] >= 0x7fffffffLL;
      vb = A.voff[p];
      ab = A.aoff[p];
    }
    const int32_t *lo = A.lo + vb + (on ? p : 0);
    Arc *arc = A.arc + ab;
    const uint8_t *fl = A.lflag + vb;
    const uint32_t f = on ? fl[item] : 0u;
    const bool src = on && LF_SRC(f);
    const bool snk = on && LF_SNK(f);
    const int32_t b0 = on ? lo[item] : 0, e0 = on ? lo[item + 1] : 0;
    int64_t ex = 0;
    for (int32_t ar = b0; ar < e0; ar++) {
      const int32_t j = arc[ar].lh;
      const int32_t je = lo[j + 1];
      int32_t r = lo[j];
      // the reverse arc: the head's arc list is short; four heads per step
      for (; r + 3 < je; r += 4) {
        const int32_t h0 = arc[r].lh, h1 = arc[r + 1].lh, h2 = arc[r + 2].lh, h3 = arc[r + 3].lh;
        if (h0 == item) break;
        if (h1 == item) { r += 1; break; }
        if (h2 == item) { r += 2; break; }
        if (h3 == item) { r += 3; break; }
      }
      while (r < je && arc[r].lh != item) r++;
      if (r == je) {  // asymmetric input slipped past validation
        A.ctl->err = FR_E_INVALID_GRAPH;
        A.ctl->diag = DIAG_REV;
        r = ar;
      }
      arc[ar].lr = r;
      if (!src && LF_SRC(fl[j]) && !overflow) {
        const int32_t c = res_own(arc[ar].rc);
        ex += c;
        arc[ar].rc = res_pair(2 * c, 0);
        arc[r].rc = res_pair(0, 2 * c);
      }
    }
    if (on) {
      if (!A.terminals) A.ex[vb + item] = src ? 0 : (int32_t)ex;  // else: the s -> u capacity
      A.ins[vb + item] = 0;
      if (overflow) {
        A.ctl->err = FR_E_OVERFLOW;
        A.ctl->diag = DIAG_OVERFLOW;
      }
    }
    const int pos = wave_append_by_key(A.pcnt + A.P, snk ? p : -1);
    if (snk) put_bounded(A.SNK + vb, pos, A.voff[p + 1] - vb, item, A.ctl);
  });
}

__global__ void __launch_bounds__(256) k_net_rev(KArgs A, int32_t it) {
  (void)it;
  net_rev(A, [&](auto &&f) { grid_items(A, A.cpre, f); });
}

// ---- maximum preflow, smallest source set, balance check, write-back and
//      the adaptive factor (Sec. 4.1), one workgroup per pair.
//      lc (sliced rounds): this launch's running and started flow entries.
template <int TPB>
__device__ __forceinline__ void flow_pair(const KArgs &A, int32_t p, SolveShared<TPB> &sh,
                                          PairState &st, const int32_t *lc = nullptr) {
  const PairView V = make_view(A, p);
  const int32_t a = V.a, b = V.b;
  int64_t *pa = A.pacc + (int64_t)p * PA_N;
  if (threadIdx.x == 0) {
    st = A.ps[p];
    sh.cnt[0] = sh.cnt[1] = sh.cnt[2] = 0;
    sh.nsnk = min(A.pcnt[A.P + p], (int32_t)V.nv);
    if (st.phase == 0) {  // a new solve (else it continues from a sliced launch)
      st.solve_sweeps = 0;
      st.rp_eff = A.relabel_period;
    }
  }
  if (threadIdx.x < W_COUNT) sh.work[threadIdx.x] = 0ull;
  __syncthreads();
  const int32_t nr = uni(st.nr);
  int64_t t0 = wall_clock64(), t1;
  const int64_t t_start = t0;
  bool sliced = false;
  int64_t t_rel = 0, t_push = 0;
  const int32_t NL = nr + 2;
  const bool lds = nr <= 32 * FR_BM_WORDS;
  const int32_t nw = (nr + 31) >> 5;
  const bool overflow = pa[PA_RCAP] >= 0x7fffffffLL;
  Rot R;
  int64_t gr_levels = 0, sweeps = 0, relabels = 0, cl_levels = 0;
  if (!overflow) {
    // one relabel call site (the relabel is inlined; one copy keeps the
    // kernel within its registers): at the start, when the active list
    // runs dry and after rp_eff passes
    int32_t cnt = 0;
    ListRef cur, nxt;
    int since = 0;
    // sweeps until the next global relabel: half the last relabel's BFS
    // depth (a deep corridor's relabel costs more), within [period / 4,
    // 2 period] of the tuning's period
    int32_t rp_eff = uni(st.rp_eff);
    const int32_t rp_lo = max(1, A.relabel_period / 4), rp_hi = 2 * A.relabel_period;
    const int64_t sweeps0 = uni(st.solve_sweeps);  // of this solve, in earlier launches
    bool relabel = true;
    for (;;) {
      if (relabel && A.slice_ticks > 0 && relabels > 0) {
        // sliced rounds: once this launch's time is used up, stop where a
        // global relabel is due anyway; the next launch starts with it
        // (only while at most a quarter of the launch's entries still run:
        // the others are waiting for it)
        if (threadIdx.x == 0) {
          int32_t stop = 0;
          if (lc && wall_clock64() - t_start >= A.slice_ticks) {
            const int32_t run = __hip_atomic_load(lc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const int32_t sta =
                __hip_atomic_load(lc + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            stop = 4 * run <= sta ? 1 : 0;
          }
          sh.slice_end = stop;
        }
        __syncthreads();
        sliced = uni(sh.slice_end) != 0;
        __syncthreads();
        if (sliced) break;
      }
      if (relabel) {
        t1 = wall_clock64();
        t_push += t1 - t0;
        t0 = t1;
        {
          const int64_t lev0 = gr_levels;
          cnt = global_relabel<TPB>(A, V, nr, NL, sh, R, gr_levels, lds);
          rp_eff = (int32_t)min((int64_t)rp_hi, max((int64_t)rp_lo, (gr_levels - lev0) / 2));
        }
        t1 = wall_clock64();
        t_rel += t1 - t0;
        t0 = t1;
        relabels++;
        cur = flist(V, sh, 0, lds);
        nxt = flist(V, sh, 1, lds);
        since = 0;
        relabel = false;
      }
      if (cnt == 0) {
        if (since == 0) break;  // an exact relabel found no active vertex
        relabel = true;
        continue;
      }
      if (sweeps0 + sweeps >= A.max_sweeps) {
        if (threadIdx.x == 0) {
          A.ctl->err = FR_E_SOLVER_LIMIT;
          A.ctl->diag = DIAG_SWEEPS;
        }
        break;
      }
      // queued marks of this pass in bm[(since + 1) & 1]; the other bitmap
      // (the previous pass's marks, or the relabel's visited marks) is
      // cleared now and serves the next pass
      uint32_t *qbm = nullptr;
      if (lds) {
        qbm = sh.u.f.bm[(since + 1) & 1];
        uint32_t *old = sh.u.f.bm[since & 1];
        for (int w = threadIdx.x; w < nw; w += TPB) old[w] = 0u;
      }
      pr_sweep_any<TPB>(A, V, cur, cnt, nxt, &sh.cnt[(R.c + 1) % 3], NL, sh.work, qbm);
      if (threadIdx.x == 0) sh.cnt[(R.c + 2) % 3] = 0;
      __syncthreads();
      R.c = (R.c + 1) % 3;
      cnt = uni(min(sh.cnt[R.c], (int32_t)V.nv));
      const ListRef t = cur;
      cur = nxt;
      nxt = t;
      sweeps++;
      if (++since >= rp_eff) relabel = true;
    }
    t1 = wall_clock64();
    t_push += t1 - t0;
    t0 = t1;
    if (sliced) {
      // the solve continues in the next launch: its counters so far, its
      // relabel interval; the network, labels and excesses stay in place
      if (threadIdx.x == 0) {
        st.sweeps += sweeps;
        st.relabels += relabels;
        st.gr_levels += gr_levels;
        for (int j = 0; j < W_COUNT; j++) st.work[j] += (int64_t)sh.work[j];
        st.t_relabel += t_rel;
        st.t_push += t_push;
        st.solve_sweeps = sweeps0 + sweeps;
        st.rp_eff = rp_eff;
        st.phase = 1;
        st.slices++;
        A.ps[p] = st;
      }
      __syncthreads();
      return;
    }
    // ---- smallest source set (Sec. 4.1.1): closure of the source border
    //      and of every vertex left with excess, over arcs with residual
    //      capacity
    {
      uint32_t *vis = sh.u.f.bm[0];
      cur = flist(V, sh, 0, lds);
      nxt = flist(V, sh, 1, lds);
      int32_t *ncnt = &sh.cnt[(R.c + 1) % 3];
      BLOCK_WAVE_LOOP(i, nr) {
        bool seed = false;
        if (i < nr) {
          const uint32_t f = V.fl[i];
          seed = LF_SRC(f) || (!LF_SNK(f) && V.ex[i] > 0);
          if (seed) V.ins[i] = 1;
        }
        if (lds) {
          const unsigned long long m = __ballot(seed);
          if (lane64() == 0) vis[i >> 5] = (uint32_t)m;
          if (lane64() == 32) vis[i >> 5] = (uint32_t)(m >> 32);
        }
        const int pos = wave_append(ncnt, seed);
        if (seed) lput(cur, pos, V.nv, (int32_t)i, A.ctl);
      }
      if (threadIdx.x == 0) sh.cnt[(R.c + 2) % 3] = 0;
      __syncthreads();
      R.c = (R.c + 1) % 3;
      int32_t cnt2 = uni(min(sh.cnt[R.c], (int32_t)V.nv));
      while (cnt2 > 0) {
        int32_t *ncnt2 = &sh.cnt[(R.c + 1) % 3];
        for_groups<GTF>(cnt2, [&](int item, bool valid, int gl) {
          const int32_t u = valid ? lget(cur, item) : 0;
          const int32_t e0 = valid ? V.lo[u] : 0, e1 = valid ? V.lo[u + 1] : 0;
          count_work(sh, W_CL_ITEMS, (valid && gl == 0) ? 1 : 0);
          count_work(sh, W_CL_ARCS, (valid && gl == 0) ? e1 - e0 : 0);
          for (int32_t c0 = e0; c0 < e1; c0 += GTF * KF) {
            int32_t v[KF], r[KF];
#pragma unroll
            for (int k = 0; k < KF; k++) {
              const int32_t ar = c0 + k * GTF + gl;
              Arc x = {0, 0, 0ull};
              if (ar < e1) x = V.arc[ar];
              r[k] = res_own(x.rc);
              v[k] = x.lh;
            }
#pragma unroll
            for (int k = 0; k < KF; k++) {
              bool claim = false;
              if (r[k] > 0) {
                if (lds) {
                  const bool seen = (vis[v[k] >> 5] >> (v[k] & 31)) & 1u;
                  if (!seen) {
                    claim = bm_claim(vis, v[k]);
                    if (claim) V.ins[v[k]] = 1;
                  }
                } else if (V.ins[v[k]] == 0) {
                  claim = atomicCAS(&V.ins[v[k]], 0, 1) == 0;
                }
              }
              const int pos = wave_append(ncnt2, claim);
              if (claim) lput(nxt, pos, V.nv, v[k], A.ctl);
            }
          }
        });
        if (threadIdx.x == 0) sh.cnt[(R.c + 2) % 3] = 0;
        __syncthreads();
        R.c = (R.c + 1) % 3;
        cnt2 = uni(min(sh.cnt[R.c], (int32_t)V.nv));
        const ListRef t = cur;
        cur = nxt;
        nxt = t;
        cl_levels++;
      }
    }
  }
  t1 = wall_clock64();
  const int64_t t_cl = t1 - t0;
  t0 = t1;
  // ---- candidate partition and its balance check (Sec. 2.1); for the most
  //      balanced cut, also the free vertices (neither in the smallest
  //      source set nor able to reach the sink: exact label NL), listed in
  //      LB with LA[i] = i for them and -1 for every other corridor vertex
  // flow, moved a->b, moved b->a, source side; the same three for the
  // largest minimum source side (label >= NL: cannot reach the sink)
  int64_t acc[7] = {0, 0, 0, 0, 0, 0, 0};
  const bool term = A.terminals != 0;
  const bool mb = A.mb_reps > 0 && !overflow;
  const int side_mode = (A.mb_reps > 0 || overflow) ? 0 : A.cut_side;
  if (mb) {
    if (threadIdx.x == 0) sh.nfree = 0;
    __syncthreads();
  }
  if (!overflow) {
    BLOCK_WAVE_LOOP(i, nr) {
      bool fv = false;
      if (i < nr) {
        const uint32_t f = V.fl[i];
        const int32_t w = A.vwgt[V.lg[i]];
        const bool in = V.ins[i] != 0;
        // the closure reached the sink: the preflow was not maximal
        if (in && (term ? V.SNK[i] > 0 : LF_SNK(f))) {
          A.ctl->err = FR_E_DEVICE;
          A.ctl->diag = DIAG_CLOSURE;
        }
        // flow: what reached the sink border; contracted terminals: what
        // left s and stayed nowhere in the corridor
        if (term) acc[0] -= V.ex[i];
        else if (LF_SNK(f)) acc[0] += V.ex[i];
        if (!(f & LF_SIDE_B) && !in) acc[1] += w;
        if ((f & LF_SIDE_B) && in) acc[2] += w;
        acc[3] += in ? 1 : 0;
        if (side_mode) {
          const bool inx = V.lab[i] >= NL;
          if (!(f & LF_SIDE_B) && !inx) acc[4] += w;
          if ((f & LF_SIDE_B) && inx) acc[5] += w;
          acc[6] += inx ? 1 : 0;
        }
        if (mb) {
          fv = !in && !(f & LF_BORDER) && V.lab[i] == NL;
          V.LA[i] = fv ? (int32_t)i : -1;
        }
      }
      if (mb) {
        const int pos = wave_append(&sh.nfree, fv);
        if (fv) V.LB[pos] = (int32_t)i;
      }
    }
  }
  block_sums<7>(acc, sh.red);
  // the record of this solve; the adaptive rule and the write-back run in
  // k_select, over all slots of the pair
  if (threadIdx.x == 0) {
    st.sweeps += sweeps;
    st.relabels += relabels;
    st.gr_levels += gr_levels;
    st.cl_levels += cl_levels;
    for (int j = 0; j < W_COUNT; j++) st.work[j] += (int64_t)sh.work[j];
    st.t_relabel += t_rel;
    st.t_push += t_push;
    st.t_closure += t_cl;
    fr_solve rec;
    const int64_t cut = st.cut;
    rec.alpha = st.alpha;
    if (term) acc[0] += pa[PA_CS];
    rec.flow = acc[0];
    rec.region_vertices = nr;
    rec.region_edges = pa[PA_RARCS] / 2;
    rec.source_side = acc[3];
    rec.cut_before = cut;
    int64_t cand = cut - pa[PA_RCIN] + acc[0];
    int64_t wa = st.cA - acc[1] + acc[2];
    int64_t wb = st.cB + acc[1] - acc[2];
    sh.use_max = 0;
    if (side_mode && cut != 0) {  // the largest minimum source side instead
      const int64_t wa2 = st.cA - acc[4] + acc[5], wb2 = st.cB + acc[4] - acc[5];
      const bool f1 = wa <= A.lmax && wb <= A.lmax, f2 = wa2 <= A.lmax && wb2 <= A.lmax;
      if (side_mode == 1 || (!f1 && f2)) {
        sh.use_max = 1;
        wa = wa2;
        wb = wb2;
        rec.source_side = acc[6];
      }
    }
    int dec;
    if (cut == 0) {
      dec = FR_DEC_NOT_ADJACENT;
      cand = 0;
      wa = st.cA;
      wb = st.cB;
      rec.flow = 0;
    } else {
      const bool feas = wa <= A.lmax && wb <= A.lmax;
      dec = !feas ? FR_DEC_INFEASIBLE : (cand < cut ? FR_DEC_APPLY : FR_DEC_EQUAL);
    }
    rec.cut_candidate = cand;
    rec.wa = wa;
    rec.wb = wb;
    rec.decision = dec;
    A.srec[p] = rec;
    st.t_finish += wall_clock64() - t0;
    for (int j = 0; j < PA_N; j++) pa[j] = 0;
    A.pcnt[p] = mb ? sh.nfree : 0;  // the most balanced cut kernel reads and clears it
    A.pcnt[A.P + p] = 0;
    st.phase = 2;
    A.ps[p] = st;
  }
  __syncthreads();
  if (sh.use_max) {  // the source side becomes every vertex that cannot reach the sink
    BLOCK_WAVE_LOOP(i, nr) {
      if (i < nr) V.ins[i] = V.lab[i] >= NL ? 1 : 0;
    }
    __syncthreads();
  }
}

template <int TPB>
__global__ void __launch_bounds__(TPB) k_flow(KArgs A, int32_t it) {
  __shared__ SolveShared<TPB> sh;
  __shared__ PairState st;
  for (;;) {
    int32_t *lc = A.queue + 4 * (it % A.max_iters) + 2;  // running, started
    const int32_t p = next_pair<TPB>(A, lc - 1, sh, 1);
    if (p < 0) break;
    if (threadIdx.x == 0 && A.slice_ticks > 0) {
      atomicAdd(lc, 1);
      atomicAdd(lc + 1, 1);
    }
    flow_pair<TPB>(A, p, sh, st, lc);
    if (threadIdx.x == 0 && A.slice_ticks > 0) atomicSub(lc, 1);
  }
}

// ---- the adaptive factor (Sec. 4.1), one block per pair: walk the slots
//      solved in this launch in halving order as the sequential loop would
//      (an applied solve doubles alpha, an infeasible one halves it and the
//      next slot holds that solve, a feasible solve that does not improve
//      stops), record the walked solves, write the applied candidate back and
//      set every slot's factor for the next launch
// Pair p of the round (entries p * W ...); s_sel: 3 LDS words (chosen slot,
// first entry, stopped).  All threads call it.
__device__ __forceinline__ void select_pair(const KArgs &A, int32_t p, int32_t *s_sel) {
  const int32_t W = A.W;
  const int32_t v0 = p * W;
  if (A.ps[v0].done) return;
  // sliced rounds: the pair moves on once every slot it runs has solved
  bool ready = true;
  for (int s = 0; s < W; s++) ready = ready && (A.ps[v0 + s].done || A.ps[v0 + s].phase == 2);
  if (!ready) {
    if (threadIdx.x == 0) s_sel[2] = 0;
    return;
  }
  if (threadIdx.x == 0) {
    PairState &R = A.ps[v0];  // updated in place (a copy would live in scratch)
    bool stop = false;
    int chosen = -1;
    int32_t next_alpha = R.alpha;
    for (int s = 0; s < W; s++) {
      const int32_t v = v0 + s;
      if (A.ps[v].done) break;  // not solved in this launch
      if (A.ctl->err != 0) {
        stop = true;
        break;
      }
      const fr_solve rec = A.srec[v];
      if (A.trace) A.trace[(int64_t)p * A.max_iters + R.iters] = rec;
      R.iters++;
      R.rv_sum += rec.region_vertices;
      R.re_sum += rec.region_edges;
      R.final_alpha = rec.alpha;
      R.flow_last = rec.flow;
      R.last_dec = rec.decision;
      R.last_slot = s;
      if (rec.decision == FR_DEC_APPLY) {
        R.applied++;
        R.cA = rec.wa;
        R.cB = rec.wb;
        R.cut = rec.cut_candidate;
        chosen = s;
        if (!A.adaptive) stop = true;
        else next_alpha = 2 * rec.alpha < A.alpha_max ? 2 * rec.alpha : A.alpha_max;
      } else if (rec.decision == FR_DEC_INFEASIBLE) {
        if (!A.adaptive || rec.alpha == 1) stop = true;
        else next_alpha = rec.alpha / 2 > 1 ? rec.alpha / 2 : 1;
      } else if (rec.decision == FR_DEC_EQUAL && R.applied == 0 && !R.restarted &&
                 R.start_alpha < A.restart_alpha) {
        R.restarted = 1;  // the plain search decides before the pair gives up
        next_alpha = A.restart_alpha;
      } else {
        stop = true;
      }
      if (!stop && R.iters >= A.max_iters) {
        stop = true;
        R.iter_cap = 1;
      }
      if (stop || rec.decision != FR_DEC_INFEASIBLE) break;
    }
    R.alpha = next_alpha;
    R.done = stop ? 1 : 0;
    R.phase = 0;
    R.iter++;
    for (int s = 1; s < W; s++) {
      PairState &q = A.ps[v0 + s];
      q.alpha = next_alpha >> s;
      q.done = (stop || q.alpha < 1) ? 1 : 0;
      q.cA = R.cA;
      q.cB = R.cB;
      q.cut = R.cut;
      q.phase = 0;
      q.iter = R.iter;
    }
    s_sel[0] = A.ctl->err == 0 ? chosen : -1;
    s_sel[1] = v0;
    s_sel[2] = stop ? 1 : 0;
  }
  __syncthreads();
  const int chosen = s_sel[0];
  if (chosen < 0) return;
  const int32_t vc = s_sel[1] + chosen;
  const int32_t a = A.pairs[2 * vc], b = A.pairs[2 * vc + 1];
  const int64_t vb = A.voff[vc];
  const int32_t nr = A.ps[vc].nr;
  for (int32_t i = threadIdx.x; i < nr; i += blockDim.x)
    A.part[A.lg[vb + i]] = A.ins[vb + i] ? a : b;
}

// Entries still iterating, for the host's count of further launches of a
// sliced round (0 once a device error stopped the round).  One block.
__global__ void __launch_bounds__(1024) k_live(KArgs A) {
  __shared__ int32_t s_live;
  if (threadIdx.x == 0) s_live = 0;
  __syncthreads();
  int32_t cnt = 0;
  for (int32_t i = threadIdx.x; i < A.P; i += blockDim.x) cnt += A.ps[i].done ? 0 : 1;
  if (cnt) atomicAdd(&s_live, cnt);
  __syncthreads();
  if (threadIdx.x == 0) A.ctl->live = A.ctl->err != 0 ? 0 : s_live;
}

__global__ void __launch_bounds__(1024) k_select(KArgs A, int32_t it) {
  __shared__ int32_t s_sel[3];
  (void)it;
  select_pair(A, blockIdx.x, s_sel);
}

// ---- a whole round in one launch: each workgroup takes a pair (one entry
//      per pair, W = 1) and runs its adaptive loop -- boundary, corridor,
//      network, flow, the adaptive rule -- to the end without waiting for the
//      other pairs.  The phases are the bodies of the per-iteration kernels
//      over the pair's own items; a pair's buffers are touched by its
//      workgroup only, so barriers order the phases.
template <int TPB>
__global__ void __launch_bounds__(TPB) k_round(KArgs A) {
  __shared__ SolveShared<TPB> sh;
  __shared__ PairState st;
  __shared__ int32_t s_sel[3];
  for (;;) {
    const int32_t p = next_pair<TPB>(A, A.queue, sh, 1);
    if (p < 0) break;
    const int64_t nu = A.voff[p + 1] - A.voff[p];
    for (int32_t it = 0; it < A.max_iters; it++) {
      bnd_union(A, [&](auto &&f) { pair_items(p, nu, f); });
      __syncthreads();
      corr_pair<TPB>(A, stamp_of(A, p), p, sh, st);
      const int32_t nr = uni(st.nr);
      net_count(A, [&](auto &&f) { pair_items(p, nr, f); });
      __syncthreads();
      net_scan_pair(A, p, sh.scan);
      __syncthreads();
      net_fill(A, [&](auto &&f) { pair_items(p, nr, f); });
      __syncthreads();
      net_rev(A, [&](auto &&f) { pair_items(p, nr, f); });
      __syncthreads();
      flow_pair<TPB>(A, p, sh, st);
      __syncthreads();
      select_pair(A, p, s_sel);
      __syncthreads();
      if (uni(s_sel[2])) break;
    }
  }
}

// side codes of the last solve of pair 0 (single-pair calls)
__global__ void __launch_bounds__(256) k_side_fill(KArgs A) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < A.n;
       u += (int64_t)gridDim.x * blockDim.x)
    A.side_out[u] = -1;
}

__global__ void __launch_bounds__(256) k_side_scatter(KArgs A) {
  const int32_t v = A.ps[0].last_slot;
  const int32_t nr = A.ps[v].last_nr;
  const int64_t vb = A.voff[v];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nr;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t f = A.lflag[vb + i];
    const int code = ((f & LF_BORDER) ? 2 : 0) + (A.ins[vb + i] ? 0 : 1);
    A.side_out[A.lg[vb + i]] = (int8_t)code;
  }
}

// quotient graph adjacency: qadj[x*k + y] = 1 for blocks x < y sharing an edge
__global__ void __launch_bounds__(256) k_quotient(KArgs A, uint8_t *qadj) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < A.n;
       u += (int64_t)gridDim.x * blockDim.x) {
    const int32_t x = A.part[u];
    for (int32_t e = A.xadj[u]; e < A.xadj[u + 1]; e++) {
      const int32_t y = A.part[A.adjncy[e]];
      if (x < y) qadj[(int64_t)x * A.k + y] = 1;
    }
  }
}

// total cut sum_{i<j} omega(E_ij), counted at the lower-id end of each edge
__global__ void __launch_bounds__(256) k_total_cut(KArgs A, int64_t *out) {
  __shared__ int64_t s_red[16];
  int64_t c = 0;
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < A.n;
       u += (int64_t)gridDim.x * blockDim.x) {
    const int32_t x = A.part[u];
    for (int32_t e = A.xadj[u]; e < A.xadj[u + 1]; e++) {
      const int32_t v = A.adjncy[e];
      if (v > u && A.part[v] != x) c += A.adjwgt[e];
    }
  }
  int64_t v[1] = {c};
  block_sums<1>(v, s_red);
  if (threadIdx.x == 0 && v[0]) atomicAdd((unsigned long long *)out, (unsigned long long)v[0]);
}
