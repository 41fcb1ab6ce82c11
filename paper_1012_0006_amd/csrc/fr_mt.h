// Multi-try FM (Sanders & Schulz, Section 4.2) on the GPU: after the
// pairwise improvements of a round, one round of localized k-way searches per
// pair, in pair order.
//
// The k-way local search of Section 2.2 moves a vertex to the adjacent block
// with the largest gain, so a search of one pair can reach any block: the
// searches of a round's pairs are not independent, and they run one after
// the other, in one wave.  Around them the work is spread over the chip:
//   k_mt_weights  block weights of all k blocks (grid-wide)
//   k_mt_todo     each pair's todo list: the vertices of its two blocks with
//                 a neighbour in another block, as sort keys (upper 32 bits
//                 of a SplitMix64 output, then the id), grid-wide
//   k_mt_sort     each todo list in key order (one workgroup per pair:
//                 bitonic in LDS, a tiled rank sort beyond)
//   k_mt          the searches (one wave): an addressable max-heap over
//                 (gain, key) in LDS that spills to device memory, each
//                 neighbour's k-way gain computed by a lane of its own, lane 0
//                 making every decision; KaSPar's stopping rule in exact
//                 integer arithmetic; rollback to the best state.
// The counters of the keys (SplitMix64 outputs from mt_seed): todo order of v
// 2^40 + v + 1, queue order of v 2^41 + v + 1, tie key of target block P of v
// 2^42 + v k + P + 1.
#pragma once
#include "fr_kernels.h"

#define MT_SORT_TPB 1024
#define MT_LSORT 8192   // todo keys sorted in LDS
#define MT_LHEAP 4096   // heap slots in LDS (the rest in device memory)
#define MT_LBLK 2048    // block weights held in LDS
#define MT_CH 16        // arcs of a vertex examined together by its lane

__device__ __forceinline__ uint64_t mt_splitmix(uint64_t seed, uint64_t n) {
  uint64_t z = seed + n * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t mt_key(uint64_t seed, int which, uint64_t x) {
  return mt_splitmix(seed, (1ull << (40 + which)) + x + 1ull);
}

// Block weights of every block (cleared by k_mt_clear).
__global__ void __launch_bounds__(256) k_mt_weights(KArgs A) {
  for (int64_t b0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) & ~(int64_t)63; b0 < A.n;
       b0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t u = b0 + lane64();
    const int key = u < A.n ? A.part[u] : -1;
    const int64_t w = u < A.n ? A.vwgt[u] : 0;
    wave_add_by_key(reinterpret_cast<unsigned long long *>(A.mtw), 1, 0, key, w);
  }
}

// Clears the weights and the todo counters of the round (one block).
__global__ void __launch_bounds__(1024) k_mt_clear(KArgs A) {
  for (int i = threadIdx.x; i < A.k; i += blockDim.x) A.mtw[i] = 0;
  for (int i = threadIdx.x; i < A.P; i += blockDim.x) A.ucnt[i] = 0;
}

// Todo keys: every vertex of a round pair's blocks with a neighbour in
// another block, appended to the pair's slice (its first entry's arena).
__global__ void __launch_bounds__(256) k_mt_todo(KArgs A) {
  const uint64_t seed = (uint64_t)(uint32_t)A.mt_seed;
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < A.n;
       u += (int64_t)gridDim.x * blockDim.x) {
    const int32_t x = A.part[u];
    const int32_t p = A.blk2pair[x];
    if (p < 0) continue;
    const int32_t e1 = A.xadj[u + 1];
    bool bnd = false;
    for (int32_t e = A.xadj[u]; e < e1 && !bnd; e++) bnd = A.part[A.adjncy[e]] != x;
    if (!bnd) continue;
    const uint64_t k = ((mt_key(seed, 0, (uint64_t)u) >> 32) << 32) | (uint64_t)(uint32_t)u;
    const int32_t pos = atomicAdd(&A.ucnt[p], 1);
    if (A.voff[p] + pos < A.voff[p + 1]) A.mtk[A.voff[p] + pos] = k;
  }
}

// Each pair's todo keys in ascending order (one workgroup per pair).
__global__ void __launch_bounds__(MT_SORT_TPB) k_mt_sort(KArgs A) {
  __shared__ unsigned long long s[MT_LSORT];
  const int32_t p = blockIdx.x * A.W;  // the pair's first entry
  const int32_t T = min((int64_t)A.ucnt[p], A.voff[p + 1] - A.voff[p]);
  unsigned long long *key = A.mtk + A.voff[p];
  if (T <= 1) return;
  if (T <= MT_LSORT) {
    int32_t N = 1;
    while (N < T) N <<= 1;
    for (int32_t i = threadIdx.x; i < N; i += blockDim.x) s[i] = i < T ? key[i] : ~0ull;
    __syncthreads();
    for (int32_t len = 2; len <= N; len <<= 1)
      for (int32_t st = len >> 1; st > 0; st >>= 1) {
        for (int32_t i = threadIdx.x; i < N; i += blockDim.x) {
          const int32_t j = i ^ st;
          if (j > i) {
            const bool up = (i & len) == 0;
            const unsigned long long a = s[i], b = s[j];
            if ((a > b) == up) {
              s[i] = b;
              s[j] = a;
            }
          }
        }
        __syncthreads();
      }
    for (int32_t i = threadIdx.x; i < T; i += blockDim.x) key[i] = s[i];
    return;
  }
  // a long list: the rank of every key (the keys are distinct) by comparing
  // with all keys, tile by tile through LDS, written to the second buffer and
  // copied back
  unsigned long long *out = A.mtk2 + A.voff[p];
  for (int32_t b0 = 0; b0 < T; b0 += blockDim.x) {
    const int32_t i = b0 + threadIdx.x;
    const unsigned long long mine = i < T ? key[i] : 0ull;
    int32_t rank = 0;
    for (int32_t t0 = 0; t0 < T; t0 += MT_LSORT) {
      const int32_t tn = min(MT_LSORT, T - t0);
      __syncthreads();
      for (int32_t j = threadIdx.x; j < tn; j += blockDim.x) s[j] = key[t0 + j];
      __syncthreads();
      if (i < T)
        for (int32_t j = 0; j < tn; j++) rank += s[j] < mine ? 1 : 0;
    }
    if (i < T) out[rank] = mine;
  }
  __syncthreads();
  for (int32_t i = threadIdx.x; i < T; i += blockDim.x) key[i] = out[i];
}

// The search state of the one wave.
struct MTShared {
  int32_t hv[MT_LHEAP];  // heap slots in LDS: vertex, gain
  int32_t hg[MT_LHEAP];
  int64_t bw[MT_LBLK];   // block weights (k <= MT_LBLK)
};

struct MTState {
  const KArgs *A;
  MTShared *sh;
  int64_t *gbw;      // block weights when k > MT_LBLK
  int32_t *ghv, *ghg;  // heap slots beyond MT_LHEAP
  int32_t hn;        // heap size
  uint64_t seed;
  __device__ __forceinline__ int64_t &bw(int32_t b) { return A->k <= MT_LBLK ? sh->bw[b] : gbw[b]; }
  __device__ __forceinline__ int32_t &hvs(int32_t i) { return i < MT_LHEAP ? sh->hv[i] : ghv[i]; }
  __device__ __forceinline__ int32_t &hgs(int32_t i) { return i < MT_LHEAP ? sh->hg[i] : ghg[i]; }
  __device__ __forceinline__ uint64_t qkey(int32_t v) const { return mt_key(seed, 1, (uint64_t)(uint32_t)v); }
  // (gu, u) before (gv, v): larger gain, then larger queue key
  __device__ __forceinline__ bool above(int32_t gu, int32_t u, int32_t gv, int32_t v) const {
    return gu != gv ? gu > gv : qkey(u) > qkey(v);
  }
  __device__ void place(int32_t i, int32_t v, int32_t g) {
    hvs(i) = v;
    hgs(i) = g;
    A->mtq[v] = i;
  }
  __device__ void up(int32_t i) {
    const int32_t v = hvs(i), g = hgs(i);
    while (i > 0) {
      const int32_t pa = (i - 1) >> 1;
      const int32_t w = hvs(pa), gw = hgs(pa);
      if (!above(g, v, gw, w)) break;
      place(i, w, gw);
      i = pa;
    }
    place(i, v, g);
  }
  __device__ void down(int32_t i) {
    const int32_t v = hvs(i), g = hgs(i);
    for (;;) {
      const int32_t l = 2 * i + 1;
      if (l >= hn) break;
      int32_t c = l, cv = hvs(l), cg = hgs(l);
      if (l + 1 < hn) {
        const int32_t rv = hvs(l + 1), rg = hgs(l + 1);
        if (above(rg, rv, cg, cv)) {
          c = l + 1;
          cv = rv;
          cg = rg;
        }
      }
      if (!above(cg, cv, g, v)) break;
      place(i, cv, cg);
      i = c;
    }
    place(i, v, g);
  }
  __device__ void push(int32_t v, int32_t g) {
    hvs(hn) = v;
    hgs(hn) = g;
    A->mtq[v] = hn;
    hn++;
    up(hn - 1);
  }
  __device__ void remove(int32_t i) {  // slot i leaves the heap
    A->mtq[hvs(i)] = -1;
    hn--;
    if (i == hn) return;
    const int32_t v = hvs(hn), g = hgs(hn);
    place(i, v, g);
    if (i > 0 && above(g, v, hgs((i - 1) >> 1), hvs((i - 1) >> 1))) up(i);
    else down(i);
  }
  __device__ void update(int32_t i, int32_t g) {  // new gain of slot i
    const int32_t old = hgs(i);
    hgs(i) = g;
    if (g > old) up(i);
    else if (g < old) down(i);
  }
};

// The k-way gain of vertex y (any lane, for its own y; y < 0: none): over the
// blocks other than y's own that hold a neighbour of y, the largest weight to
// that block minus the weight to y's own block; the block reaching it is the
// target (equal gains: the smaller tie key).  Returns the target or -1 when y
// has no neighbour outside its block; *ovf is set when a weighted degree
// reaches 2^31.  Arcs are read MT_CH at a time; with more than MT_CH arcs the
// block sums of each candidate are re-read over all arcs.
__device__ int32_t mt_gain(const KArgs &A, int32_t y, uint64_t seed, int32_t *gain, bool *ovf) {
  if (y < 0) return -1;
  const int32_t e0 = A.xadj[y], e1 = A.xadj[y + 1];
  const int32_t own = A.part[y];
  const int32_t deg = e1 - e0;
  int32_t best = -1;
  int64_t bg = 0;
  uint64_t bk = 0;
  auto consider = [&](int32_t P, int64_t gP) {
    const uint64_t kP = mt_key(seed, 2, (uint64_t)(uint32_t)y * (uint64_t)A.k + (uint64_t)P);
    if (best < 0 || gP > bg || (gP == bg && kP < bk)) {
      best = P;
      bg = gP;
      bk = kP;
    }
  };
  int64_t wown = 0, wtot = 0;
  if (deg <= MT_CH) {
    int32_t b[MT_CH];
    int32_t w[MT_CH];
#pragma unroll
    for (int j = 0; j < MT_CH; j++) {
      const int32_t e = e0 + j;
      b[j] = -1;
      w[j] = 0;
      if (e < e1) {
        w[j] = A.adjwgt[e];
        b[j] = A.adjncy[e];
      }
    }
#pragma unroll
    for (int j = 0; j < MT_CH; j++) b[j] = b[j] >= 0 ? A.part[b[j]] : -1;
#pragma unroll
    for (int j = 0; j < MT_CH; j++) {
      wtot += w[j];
      if (b[j] == own) wown += w[j];
    }
#pragma unroll
    for (int j = 0; j < MT_CH; j++) {
      if (b[j] < 0 || b[j] == own) continue;
      bool first = true;  // count each block once, at its first arc
      int64_t s = 0;
#pragma unroll
      for (int i = 0; i < MT_CH; i++) {
        if (b[i] == b[j]) {
          s += w[i];
          if (i < j) first = false;
        }
      }
      if (first) consider(b[j], s - wown);
    }
  } else {
    for (int32_t e = e0; e < e1; e++) {
      const int32_t w = A.adjwgt[e];
      wtot += w;
      if (A.part[A.adjncy[e]] == own) wown += w;
    }
    for (int32_t e = e0; e < e1; e++) {
      const int32_t P = A.part[A.adjncy[e]];
      if (P == own) continue;
      bool first = true;
      int64_t s = 0;
      for (int32_t f = e0; f < e1; f++) {
        if (A.part[A.adjncy[f]] == P) {
          s += A.adjwgt[f];
          if (f < e) first = false;
        }
      }
      if (first) consider(P, s - wown);
    }
  }
  if (wtot >= 0x7fffffffLL) *ovf = true;
  *gain = (int32_t)bg;
  return best;
}

// KaSPar's stopping rule: p moves since the last best state with gain sum S1
// and square sum S2 stop the search when p mu^2 > alpha sigma^2 + ln n, i.e.
// 2^16 (p S1^2 - alpha (p S2 - S1^2)) > beta_fx p^2 with beta_fx = floor(ln n
// 2^16).
__device__ __forceinline__ bool mt_stop(int64_t p, __int128 S1, __int128 S2, int32_t alpha,
                                        int64_t beta_fx) {
  const __int128 lhs =
      ((__int128)p * S1 * S1 - (__int128)alpha * ((__int128)p * S2 - S1 * S1)) * 65536;
  return lhs > (__int128)beta_fx * p * p;
}

// The multi-try rounds of all pairs of the round, in pair order (one wave).
__global__ void __launch_bounds__(WAVE) k_mt(KArgs A) {
  __shared__ MTShared sh;
  const int lane = lane64();
  const uint64_t seed = (uint64_t)(uint32_t)A.mt_seed;
  if (A.ctl->err != 0) return;
  MTState H;
  H.A = &A;
  H.sh = &sh;
  H.gbw = A.mtw;
  H.ghv = A.mth;
  H.ghg = A.mth + A.n;
  H.hn = 0;
  H.seed = seed;
  // block weights and the blocks above L_max
  int64_t over = 0;
  for (int32_t b = lane; b < A.k; b += WAVE) {
    const int64_t w = A.mtw[b];
    if (A.k <= MT_LBLK) sh.bw[b] = w;
    over += w > A.lmax ? 1 : 0;
  }
  for (int o = 32; o > 0; o >>= 1) over += __shfl_xor(over, o);
  bool ovf = false;
  const int32_t npair = A.P / A.W;
  for (int32_t q = 0; q < npair; q++) {
    const int32_t p0 = q * A.W;
    const int32_t stamp = A.mt_stamp0 + q + 1;
    const int32_t T = (int32_t)min((int64_t)A.ucnt[p0], A.voff[p0 + 1] - A.voff[p0]);
    const unsigned long long *todo = A.mtk + A.voff[p0];
    int64_t searches = 0, moves = 0, kept = 0;
    for (int32_t ti = 0; ti < T; ti++) {
      const int32_t v = (int32_t)(uint32_t)todo[ti];
      if (A.mtt[v] == stamp) continue;
      int32_t gv = 0;
      bool o1 = false;
      const int32_t tv = mt_gain(A, lane == 0 ? v : -1, seed, &gv, &o1);
      ovf |= o1;
      if (__shfl(tv, 0) < 0) continue;  // no longer a boundary vertex
      // the start set: v and its untouched boundary neighbours, a lane each
      int64_t delta = 0, best = 0, best_over = over;
      int64_t nmv = 0, best_n = 0, pcount = 0;
      __int128 S1 = 0, S2 = 0;
      {
        const int32_t e0 = A.xadj[v], e1 = A.xadj[v + 1];
        for (int32_t c0 = e0 - 1; c0 < e1; c0 += WAVE) {
          const int32_t e = c0 + lane;
          int32_t y = -1;
          if (e == e0 - 1) y = v;
          else if (e < e1) y = A.adjncy[e];
          if (y >= 0 && y != v && A.mtt[y] == stamp) y = -1;
          int32_t g = 0;
          bool o2 = false;
          const int32_t t = mt_gain(A, y, seed, &g, &o2);
          ovf |= o2;
          if (t >= 0) {
            A.mtt[y] = stamp;
            A.mtb[y] = t;
          }
          // lane 0 queues them in lane order
          unsigned long long m = __ballot(t >= 0);
          while (m) {
            const int l = __ffsll(m) - 1;
            m &= m - 1;
            const int32_t yl = __shfl(y, l), gl = __shfl(g, l);
            if (lane == 0) H.push(yl, gl);
          }
        }
      }
      searches++;
      // the moves
      for (;;) {
        int32_t x = -1, to = -1, gx = 0, from = -1;
        int skip = 0;
        if (lane == 0 && H.hn > 0) {
          x = H.hvs(0);
          gx = H.hgs(0);
          H.remove(0);
          to = A.mtb[x];
          from = A.part[x];
          const int64_t cx = A.vwgt[x];
          if (H.bw(to) + cx > A.lmax) {
            skip = 1;  // the move would overload its target
          } else {
            if (H.bw(from) > A.lmax && H.bw(from) - cx <= A.lmax) over--;
            H.bw(from) -= cx;
            H.bw(to) += cx;
            A.part[x] = to;
            A.mtv[nmv] = x;
            A.mtf[nmv] = from;
          }
        }
        x = __shfl(x, 0);
        if (x < 0) break;
        if (__shfl(skip, 0)) continue;
        gx = __shfl(gx, 0);
        over = __shfl(over, 0);
        nmv++;
        delta -= gx;
        if (over < best_over || (over == best_over && delta < best)) {
          best = delta;
          best_over = over;
          best_n = nmv;
          pcount = 0;
          S1 = S2 = 0;
        } else {
          pcount++;
          S1 += gx;
          S2 += (__int128)gx * gx;
          if (mt_stop(pcount, S1, S2, A.mt_alpha, A.mt_beta)) break;
        }
        // x's neighbours: queued ones get their gain again (or leave without
        // a target), untouched boundary ones join; a lane each
        const int32_t e0 = A.xadj[x], e1 = A.xadj[x + 1];
        for (int32_t c0 = e0; c0 < e1; c0 += WAVE) {
          const int32_t e = c0 + lane;
          int32_t y = e < e1 ? A.adjncy[e] : -1;
          int32_t slot = -1;
          if (y >= 0) {
            slot = A.mtq[y];
            if (slot < 0 && A.mtt[y] == stamp) y = -1;  // touched, not queued
          }
          int32_t g = 0;
          bool o2 = false;
          const int32_t t = mt_gain(A, y, seed, &g, &o2);
          ovf |= o2;
          if (t >= 0) A.mtb[y] = t;
          unsigned long long m = __ballot(y >= 0);
          while (m) {
            const int l = __ffsll(m) - 1;
            m &= m - 1;
            const int32_t yl = __shfl(y, l), gl = __shfl(g, l), tl = __shfl(t, l);
            if (lane == 0) {
              const int32_t sl = A.mtq[yl];  // current slot (earlier updates move entries)
              if (sl >= 0) {
                if (tl < 0) H.remove(sl);
                else H.update(sl, gl);
              } else if (tl >= 0) {
                A.mtt[yl] = stamp;
                H.push(yl, gl);
              }
            }
          }
        }
      }
      // the queue ends empty; roll back the moves after the best state
      if (lane == 0) {
        while (H.hn > 0) H.remove(H.hn - 1);
        for (int64_t j = nmv - 1; j >= best_n; j--) {
          const int32_t y = A.mtv[j], fr = A.mtf[j], tb = A.part[y];
          const int64_t cy = A.vwgt[y];
          H.bw(tb) -= cy;
          if (H.bw(fr) <= A.lmax && H.bw(fr) + cy > A.lmax) over++;
          H.bw(fr) += cy;
          A.part[y] = fr;
        }
        for (int64_t j = 0; j < best_n; j++) {
          A.mtchg[A.mtf[j]] = 1;
          A.mtchg[A.part[A.mtv[j]]] = 1;
        }
      }
      over = __shfl(over, 0);
      moves += nmv;
      kept += best_n;
    }
    if (lane == 0) {
      PairState &ps = A.ps[p0];
      ps.mt_searches += searches;
      ps.mt_moves += moves;
      ps.mt_kept += kept;
    }
  }
  for (int o = 32; o > 0; o >>= 1) ovf |= __shfl_xor((int)ovf, o) != 0;
  if (lane == 0 && ovf) {
    A.ctl->err = FR_E_OVERFLOW;
    A.ctl->diag = DIAG_MT;
  }
}
