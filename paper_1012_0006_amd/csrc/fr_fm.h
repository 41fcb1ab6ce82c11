// 2-way FM local search with TopGain (Sanders & Schulz, Section 2.2; KaPPa's
// pairwise local search) on the GPU: the pairwise improvement that runs on
// each pair of a round before its adaptive flow iterations.
//
// A grid-wide pass computes the gains of all vertices of the round's pairs
// and lists each pair's boundary vertices; then one workgroup per pair builds
// its two queues level by level.  The moves themselves are sequential by
// nature: lane 0 makes every decision and heap update, the rest of its wave
// fetches each moved vertex's neighbourhood at once:
//   - one queue per block: a binary max-heap in the pair's arena ordered by
//     (gain, key), the key a per-vertex SplitMix64 output, so the order does
//     not depend on how the heap was built; heap positions (or -1 = not
//     queued, -2 = moved) and gains live in per-vertex arrays;
//   - TopGain: the block with the larger top gain moves (a random bit on
//     ties), the heavier block while one is overloaded;
//   - after a move, the unmoved neighbours in the pair get their gains
//     changed by +-2 w and are queued if they were not;
//   - stop after fm_limit moves without a better state (feasible before
//     infeasible, then smaller cut, or a lighter heavier block while
//     infeasible) or when both queues are empty; roll back to the first best
//     state.
#pragma once
#include "fr_kernels.h"

#define FM_TPB 256

__device__ __forceinline__ uint64_t fm_splitmix(uint64_t seed, uint64_t n) {
  uint64_t z = seed + n * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Addressable binary max-heap of vertex ids over (gain, key).  Each slot
// keeps its vertex's gain beside the id (hv, hg), so a level of a sift is
// one round of independent loads.
struct FMHeap {
  int32_t *hv;       // heap slots: vertex
  int32_t *hg;       // heap slots: its gain
  int32_t n;
  int32_t *pos;      // per vertex: slot, -1 not queued, -2 moved
  uint64_t seed;
  __device__ __forceinline__ uint64_t key(int32_t v) const {
    return fm_splitmix(seed, (uint64_t)(uint32_t)v + 1);
  }
  // true when (gu, u) comes before (gv, v)
  __device__ __forceinline__ bool above(int32_t gu, int32_t u, int32_t gv, int32_t v) const {
    return gu != gv ? gu > gv : key(u) > key(v);
  }
  __device__ void up(int32_t i) {
    const int32_t v = hv[i], gv = hg[i];
    while (i > 0) {
      const int32_t pa = (i - 1) >> 1;
      const int32_t w = hv[pa], gw = hg[pa];
      if (!above(gv, v, gw, w)) break;
      hv[i] = w;
      hg[i] = gw;
      pos[w] = i;
      i = pa;
    }
    hv[i] = v;
    hg[i] = gv;
    pos[v] = i;
  }
  __device__ void down(int32_t i) {
    const int32_t v = hv[i], gv = hg[i];
    for (;;) {
      int32_t c = 2 * i + 1;
      if (c >= n) break;
      int32_t w = hv[c], gw = hg[c];
      if (c + 1 < n) {
        const int32_t w2 = hv[c + 1], g2 = hg[c + 1];
        if (above(g2, w2, gw, w)) {
          c++;
          w = w2;
          gw = g2;
        }
      }
      if (!above(gw, w, gv, v)) break;
      hv[i] = w;
      hg[i] = gw;
      pos[w] = i;
      i = c;
    }
    hv[i] = v;
    hg[i] = gv;
    pos[v] = i;
  }
  __device__ void push(int32_t v, int32_t g) {
    hv[n] = v;
    hg[n] = g;
    pos[v] = n;
    up(n++);
  }
  __device__ int32_t pop() {
    const int32_t top = hv[0];
    --n;
    if (n > 0) {
      const int32_t last = hv[n];
      hv[0] = last;
      hg[0] = hg[n];
      pos[last] = 0;
      down(0);
    }
    return top;
  }
  // the vertex in slot i has the new gain g, up (grew) or down
  __device__ void changed(int32_t i, int32_t g, bool grew) {
    hg[i] = g;
    if (grew) up(i);
    else down(i);
  }
};

// Queues of the pair's two blocks in the first entry's arena (vertex and gain
// per slot), whose per-iteration arrays are free until the flow iterations;
// the move log follows them.
#define FM_QUEUES(A, vb)                                                        \
  int32_t *hvA = (A).ex + (vb), *hgA = (A).lab + (vb), *hvB = (A).LA + (vb),  \
          *hgB = (A).SNK + (vb), *log = (A).LB + (vb)

// Gains of every vertex in a block of a pair of the round (weight to the other
// block minus weight inside its own), queue position -1, the pair's boundary
// vertices (a neighbour in the other block) listed per side in the queue
// slots (counts in pcnt[p] and pcnt[P + p]), the pair's cut summed into
// pacc[p][PA_CUT] and vertices whose weighted degree does not fit int32
// counted in pacc[p][PA_BW0].  The FM kernel reads and clears these sums.
__global__ void __launch_bounds__(256) k_fm_gain(KArgs A) {
  unsigned long long *acc = (unsigned long long *)A.pacc;
  for (int64_t b0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) & ~(int64_t)63;
       b0 < A.n; b0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t u = b0 + lane64();
    int32_t p = -1, side = 0;
    int64_t ext = 0, in = 0;
    if (u < A.n) {
      const int32_t pv = A.part[u];
      p = A.blk2pair[pv];
      if (p >= 0) {
        side = pv == A.pairs[2 * p] ? 0 : 1;
        const int32_t other = A.pairs[2 * p + 1 - side];
        for (int32_t e = A.xadj[u]; e < A.xadj[u + 1]; e++) {
          const int32_t pu = A.part[A.adjncy[e]];
          if (pu == other) ext += A.adjwgt[e];
          else if (pu == pv) in += A.adjwgt[e];
        }
        A.fmg[u] = (int32_t)(ext - in);
        A.fmq[u] = -1;
      }
    }
    wave_add_by_key(acc, PA_N, PA_CUT, p >= 0 && side == 0 ? p : -1, ext);
    wave_add_by_key(acc, PA_N, PA_BW0, p >= 0 && ext + in > 0x7fffffffLL ? p : -1, 1);
    const int key = p >= 0 && ext > 0 ? (side ? A.P + p : p) : -1;
    const int slot = wave_append_by_key(A.pcnt, key);
    if (key >= 0) {
      const int64_t vb = A.voff[p];
      if (slot < A.voff[p + 1] - vb) {
        FM_QUEUES(A, vb);
        (side ? hvB : hvA)[slot] = (int32_t)u;
        (side ? hgB : hgA)[slot] = (int32_t)(ext - in);
      }
    }
  }
}

__global__ void __launch_bounds__(FM_TPB) k_fm(KArgs A) {
  __shared__ int32_t s_n[2];
  __shared__ int64_t s_cut;
  __shared__ int32_t s_bad;
  const int32_t q = blockIdx.x;  // pair of the round
  const int32_t v0 = q * A.W;   // its first entry
  const int32_t a = A.pairs[2 * v0], b = A.pairs[2 * v0 + 1];
  const int64_t vb = A.voff[v0];
  FM_QUEUES(A, vb);
  int32_t *gain = A.fmg, *pos = A.fmq;
  if (threadIdx.x == 0) {  // the gain pass's sums, cleared for the flow iterations
    const int64_t cap = A.voff[v0 + 1] - vb;
    int64_t *pa = A.pacc + (int64_t)v0 * PA_N;
    s_n[0] = (int32_t)min<int64_t>(A.pcnt[v0], cap);
    s_n[1] = (int32_t)min<int64_t>(A.pcnt[A.P + v0], cap);
    s_cut = pa[PA_CUT];
    s_bad = pa[PA_BW0] != 0;  // gains must fit int32
    pa[PA_CUT] = pa[PA_BW0] = 0;
    A.pcnt[v0] = A.pcnt[A.P + v0] = 0;
  }
  __syncthreads();
  if (s_bad) {
    if (threadIdx.x == 0) {
      A.ctl->err = FR_E_OVERFLOW;
      A.ctl->diag = DIAG_FM;
    }
    return;
  }
  const uint64_t seed = (uint64_t)(uint32_t)A.fm_seed;
  // two named heaps (an array indexed at run time would live in scratch)
  FMHeap HA{hvA, hgA, s_n[0], pos, seed}, HB{hvB, hgB, s_n[1], pos, seed};
  // heap build: slots, then sift-downs one tree level at a time from the
  // deepest internal level up (the subtrees of one level are disjoint)
  for (int32_t i = threadIdx.x; i < HA.n + HB.n; i += blockDim.x) {
    if (i < HA.n) pos[HA.hv[i]] = i;
    else pos[HB.hv[i - HA.n]] = i - HA.n;
  }
  __syncthreads();
  const int32_t ia = HA.n / 2, ib = HB.n / 2;  // internal nodes: [0, n / 2)
  for (int d = 30; d >= 0; d--) {
    const int32_t lo = (1 << d) - 1;  // level d: [lo, 2 lo + 1)
    if (lo >= ia && lo >= ib) continue;
    const int32_t ca = max(0, min(2 * lo + 1, ia) - lo), cb = max(0, min(2 * lo + 1, ib) - lo);
    for (int32_t j = threadIdx.x; j < ca + cb; j += blockDim.x) {
      if (j < ca) HA.down(lo + j);
      else HB.down(lo + j - ca);
    }
    __syncthreads();
  }
  // the moves: the first wave; lane 0 keeps the state and makes every
  // decision, the other lanes fetch the moved vertex's neighbourhood
  if (threadIdx.x >= WAVE) return;
  const int lane = lane64();
  int64_t cut = s_cut;
  const int64_t lmax = A.lmax;
  int64_t wa = A.ps[v0].cA, wb = A.ps[v0].cB;
  const int64_t cut0 = cut;
  int best_inf = !(wa <= lmax && wb <= lmax);
  int64_t best_val = best_inf ? (wa > wb ? wa : wb) : cut;
  int32_t steps = 0, best_step = 0, since = 0;
  for (;;) {
    int32_t v = -1, side = 0;
    if (lane == 0 && since < A.fm_limit) {
      const int32_t tA = HA.n > 0 ? HA.hv[0] : -1, tB = HB.n > 0 ? HB.hv[0] : -1;
      if (tA >= 0 || tB >= 0) {
        if ((wa > lmax || wb > lmax) && wa != wb) side = wa > wb ? 0 : 1;
        else if (tA < 0 || tB < 0) side = tA < 0 ? 1 : 0;
        else if (HA.hg[0] != HB.hg[0]) side = HA.hg[0] > HB.hg[0] ? 0 : 1;
        else side = (int)(fm_splitmix(seed, (1ull << 32) + (uint64_t)steps + 1) & 1ull);
        if ((side ? tB : tA) < 0) side = 1 - side;
        v = side ? HB.pop() : HA.pop();
        A.part[v] = side ? a : b;
        pos[v] = -2;
        cut -= gain[v];
        const int64_t wv = A.vwgt[v];
        if (side == 0) {
          wa -= wv;
          wb += wv;
        } else {
          wb -= wv;
          wa += wv;
        }
        log[steps++] = v;
      }
    }
    v = __builtin_amdgcn_readfirstlane(v);
    side = __builtin_amdgcn_readfirstlane(side);
    if (v < 0) break;
    const int32_t from = side ? b : a;
    // the neighbours, one per lane, then lane 0 updates them in adjacency
    // order (their heap slots re-read: an earlier update may move them)
    const int32_t e0 = A.xadj[v], e1 = A.xadj[v + 1];
    for (int32_t c0 = e0; c0 < e1; c0 += WAVE) {
      const int32_t e = c0 + lane;
      int32_t u = 0, w = 0, pu = -1, gu = 0;
      if (e < e1) {
        u = A.adjncy[e];
        w = A.adjwgt[e];
        pu = A.part[u];
        gu = gain[u];
        const int32_t pq = pos[u];  // brings the line close for lane 0
        asm volatile("" ::"v"(pq));
      }
      const int32_t cnt = min(WAVE, e1 - c0);
      for (int32_t j = 0; j < cnt; j++) {
        const int32_t uj = __builtin_amdgcn_readlane(u, j);
        const int32_t pj = __builtin_amdgcn_readlane(pu, j);
        if (pj != a && pj != b) continue;
        const int32_t wj = __builtin_amdgcn_readlane(w, j);
        const int32_t gj = __builtin_amdgcn_readlane(gu, j);
        if (lane == 0) {
          const int32_t pq = pos[uj];
          if (pq != -2) {
            const bool grew = pj == from;  // an internal edge of u became a cut edge
            const int32_t g2 = gj + (grew ? 2 * wj : -2 * wj);
            gain[uj] = g2;
            if (pj == a) {
              if (pq >= 0) HA.changed(pq, g2, grew);
              else HA.push(uj, g2);
            } else {
              if (pq >= 0) HB.changed(pq, g2, grew);
              else HB.push(uj, g2);
            }
          }
        }
      }
    }
    if (lane == 0) {
      const int inf = !(wa <= lmax && wb <= lmax);
      const int64_t val = inf ? (wa > wb ? wa : wb) : cut;
      if (inf < best_inf || (inf == best_inf && val < best_val)) {
        best_inf = inf;
        best_val = val;
        best_step = steps;
        since = 0;
      } else {
        since++;
      }
    }
  }
  if (lane != 0) return;
  // roll back the moves after the best state
  for (int32_t i = steps - 1; i >= best_step; i--) {
    const int32_t v = log[i];
    const int32_t back = A.part[v] == a ? b : a;
    A.part[v] = back;
    const int64_t wv = A.vwgt[v];
    if (back == a) {
      wa += wv;
      wb -= wv;
    } else {
      wb += wv;
      wa -= wv;
    }
  }
  for (int32_t s = 0; s < A.W; s++) {
    PairState &ps = A.ps[v0 + s];
    ps.cA = wa;
    ps.cB = wb;
    ps.cut0 = cut0;
  }
  A.ps[v0].fm_steps += steps;
  A.ps[v0].fm_kept += best_step;
}
