// Device code of libflowrefine: max-flow min-cut pair refinement
// (Sanders & Schulz, Section 4.1) for gfx950.
//
// All pairs of one call are solved together: their corridors are disjoint
// (each pair owns two blocks), so the union of their flow networks is one
// flow network with many sources and sinks whose components never touch.
// Every stage is a grid-stride pass over that union, so one launch serves any
// number of pairs of uneven sizes.  Each round (one flow solve per active
// pair) runs four persistent kernels launched cooperatively:
//   k_corridor  boundary nodes, the two bounded BFS per pair, the id-ordered
//               cut of the last BFS level (radix select on vertex ids)
//   k_build     corridor compaction to local ids (ascending global id), the
//               local CSR with reverse-arc index, border flags, initial
//               preflow out of the source border
//   k_flow      push/relabel sweeps over an active-vertex frontier with
//               periodic global relabelling (backward BFS from the sink
//               border over residual arcs), then the residual closure that
//               yields the smallest source set
//   k_finish    per-pair reductions, balance check and adaptive factor
//               update, write-back of accepted cuts
// Inside a kernel, phases are separated by a software grid barrier.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fr_internal.h"

#define WAVE 64

// ------------------------------------------------------------------------
// small wave / block helpers

__device__ __forceinline__ int lane64() { return (int)__lane_id(); }

// Append for lanes with want=true among the ACTIVE lanes of the wave: one
// atomic per wave.  Returns the slot (or -1).
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

// Store v at list[pos] if the slot exists; a slot past the capacity means a
// logic error, recorded in *err instead of written out of bounds.
__device__ __forceinline__ void put_bounded(int32_t *list, int pos, int64_t cap, int32_t v,
                                            Ctl *ctl) {
  if (pos >= 0 && pos < cap) {
    list[pos] = v;
  } else if (pos >= 0) {
    ctl->err = FR_E_DEVICE;
    ctl->diag = DIAG_LIST;
  }
}

// Sum over all 64 lanes (the wave must be converged).
__device__ __forceinline__ int64_t wave_sum64(int64_t v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Add v into base[key*stride + slot] for every lane with key >= 0 and v != 0;
// one atomic per wave when all lanes agree on the key (the common case,
// because frontier lists are filled by whole waves).  Converged wave only.
__device__ __forceinline__ void wave_add_keyed(int64_t *base, int stride, int slot, int key,
                                               int64_t v) {
  int k0 = __shfl(key, 0);
  bool same = __ballot(key != k0 && v != 0) == 0ull;
  if (same) {
    int64_t s = wave_sum64(k0 >= 0 ? v : 0);
    if (lane64() == 0 && k0 >= 0 && s != 0)
      atomicAdd((unsigned long long *)&base[(int64_t)k0 * stride + slot], (unsigned long long)s);
  } else if (key >= 0 && v != 0) {
    atomicAdd((unsigned long long *)&base[(int64_t)key * stride + slot], (unsigned long long)v);
  }
}

// Exclusive scan of one int64 per thread over the block; *total gets the sum.
// lds must hold blockDim.x/64 + 1 entries.  Every thread of the block calls it.
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

__device__ int64_t block_sum64(int64_t v, int64_t *lds) {
  int64_t tot;
  block_exscan64(v, &tot, lds);
  return tot;
}

// ------------------------------------------------------------------------
// grid barrier with a bounded wait: if a wait exceeds spin_limit ticks of
// the constant-rate wall clock, the barrier sets abort and every block leaves
// at its next barrier, so no wave can wait forever.

__device__ bool grid_sync(const KArgs &A) {
  __shared__ int s_ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = 1;
    GridBar *b = A.bar;
    uint32_t nb = gridDim.x;
    uint32_t g = __hip_atomic_load(&b->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
    uint32_t arrived =
        __hip_atomic_fetch_add(&b->count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (arrived == nb - 1) {
      __hip_atomic_store(&b->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&b->gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      uint64_t t0 = (uint64_t)wall_clock64();
      while (__hip_atomic_load(&b->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
        __builtin_amdgcn_s_sleep(2);
        if (__hip_atomic_load(&b->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          ok = 0;
          break;
        }
        if ((uint64_t)wall_clock64() - t0 > A.spin_limit) {
          __hip_atomic_store(&b->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
      }
    }
    if (__hip_atomic_load(&b->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) ok = 0;
    __threadfence();
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}

// wave-uniform grid-stride iteration: every lane of a wave runs the same
// number of iterations (idx may be out of range on the last one)
#define GRID_WAVE_LOOP(i, N)                                                          \
  for (int64_t _b = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) & ~(int64_t)63, \
               _s = (int64_t)gridDim.x * blockDim.x;                                  \
       _b < (int64_t)(N); _b += _s)                                                   \
    for (int64_t i = _b + lane64(), _once = 1; _once; _once = 0)

// ------------------------------------------------------------------------
// setup: vertex-weight totals, block weights, partition range check

__global__ void __launch_bounds__(256) k_setup(KArgs A, int64_t *bw) {
  __shared__ int64_t s_red[8];
  __shared__ unsigned long long s_hist[4096];
  const bool priv = A.k <= 4096;
  if (priv)
    for (int i = threadIdx.x; i < A.k; i += blockDim.x) s_hist[i] = 0ull;
  __syncthreads();
  int64_t sum = 0;
  int32_t mx = 0;
  int bad = 0;
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < A.n;
       u += (int64_t)gridDim.x * blockDim.x) {
    int32_t w = A.vwgt[u];
    int32_t x = A.part[u];
    sum += w;
    mx = w > mx ? w : mx;
    if (w < 0) bad = 2;
    if (x < 0 || x >= A.k) {
      bad |= 1;
      continue;
    }
    if (priv) atomicAdd(&s_hist[x], (unsigned long long)(int64_t)w);
    else atomicAdd((unsigned long long *)&bw[x], (unsigned long long)(int64_t)w);
  }
  int64_t tot = block_sum64(sum, s_red);
  if (threadIdx.x == 0) atomicAdd((unsigned long long *)&A.ctl->cV, (unsigned long long)tot);
  for (int o = 32; o > 0; o >>= 1) {
    int32_t t = __shfl_xor(mx, o);
    mx = t > mx ? t : mx;
  }
  if (lane64() == 0 && mx > 0) atomicMax((long long *)&A.ctl->maxc, (long long)mx);
  if (bad & 1) atomicOr(&A.ctl->bad_part, 1);
  if (bad & 2) atomicOr(&A.ctl->bad_graph, 1);
  __syncthreads();
  if (priv)
    for (int i = threadIdx.x; i < A.k; i += blockDim.x)
      if (s_hist[i]) atomicAdd((unsigned long long *)&bw[i], s_hist[i]);
}

// CSR checks: ids in range, no self loop, no repeated neighbour, weights in
// [1, 2^30), symmetric with equal weights.
__global__ void __launch_bounds__(256) k_validate(KArgs A, int64_t narcs) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < A.n;
       u += (int64_t)gridDim.x * blockDim.x) {
    int32_t b = A.xadj[u], e = A.xadj[u + 1];
    if (b < 0 || e < b || e > narcs) {
      atomicOr(&A.ctl->bad_graph, 1);
      continue;
    }
    for (int32_t j = b; j < e; j++) {
      int32_t v = A.adjncy[j], w = A.adjwgt[j];
      bool ok = v >= 0 && v < A.n && v != (int32_t)u && w >= 1 && w < (1 << 30);
      for (int32_t q = b; ok && q < j; q++)
        if (A.adjncy[q] == v) ok = false;
      if (ok) {
        bool found = false;
        int32_t vb = A.xadj[v], ve = A.xadj[v + 1];
        for (int32_t q = vb; q < ve; q++)
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

// initial per-pair state; one block
__global__ void __launch_bounds__(256) k_pair_init(KArgs A, const int32_t *pairs,
                                                   const int64_t *bw, const int32_t *alpha0) {
  for (int p = threadIdx.x; p < A.P; p += blockDim.x) {
    PairState s;
    s.a = pairs[2 * p];
    s.b = pairs[2 * p + 1];
    int al = alpha0 ? alpha0[p] : 1;
    al = al < 1 ? 1 : (al > A.alpha_max ? A.alpha_max : al);
    s.alpha = al;
    s.start_alpha = al;
    s.final_alpha = al;
    s.active = 1;
    s.iters = s.applied = s.last_dec = s.iter_cap = 0;
    s.stopped = 0;
    s.pad = 0;
    s.cA = bw[s.a];
    s.cB = bw[s.b];
    s.cut = -1;
    s.cut0 = -1;
    s.flow_last = 0;
    s.rv_sum = s.re_sum = 0;
    int64_t base = A.base[al];
    s.U[0] = base - s.cB > 0 ? base - s.cB : 0;
    s.U[1] = base - s.cA > 0 ? base - s.cA : 0;
    A.ps[p] = s;
    for (int j = 0; j < FR_NACC; j++) A.acc[p * FR_NACC + j] = 0;
    for (int j = 0; j < 3; j++)
      for (int sd = 0; sd < 2; sd++) {
        A.lvlw[(j * A.P + p) * 2 + sd] = 0;
        A.lvlc[(j * A.P + p) * 2 + sd] = 0;
      }
  }
  if (threadIdx.x == 0) {
    A.ctl->cnt[0] = A.ctl->cnt[1] = A.ctl->cnt[2] = 0;
    A.ctl->active_pairs = A.P;
  }
}

// ------------------------------------------------------------------------
// k_corridor

// Among the vertices of `list` that belong to side si (block x), find the
// first vertex y0 in ascending id whose inclusive weight prefix exceeds R and
// exclude every vertex with id >= y0 (mark = S + 1).  Radix descent over the
// id bits, 11 + 10 + 10 bits; one block.
__device__ void select_level_prefix(const KArgs &A, int32_t x, const int32_t *list, int32_t cnt,
                                    int64_t R, int32_t S, unsigned long long *hist,
                                    int64_t *lds_scan, int *s_digit, int64_t *s_before) {
  uint32_t prefix = 0, mask = 0;
  int64_t rem = R;
  for (int pass = 0; pass < 3; pass++) {
    const int shift = pass == 0 ? 20 : (pass == 1 ? 10 : 0);
    const int nbk = pass == 0 ? 2048 : 1024;
    for (int i = threadIdx.x; i < nbk; i += blockDim.x) hist[i] = 0ull;
    __syncthreads();
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
      int32_t u = list[i];
      if (A.part[u] == x && ((uint32_t)u & mask) == prefix)
        atomicAdd(&hist[((uint32_t)u >> shift) & (nbk - 1)], (unsigned long long)(int64_t)A.vwgt[u]);
    }
    __syncthreads();
    const int per = nbk / blockDim.x;  // blockDim divides 1024
    int64_t mine = 0;
    for (int j = 0; j < per; j++) mine += (int64_t)hist[threadIdx.x * per + j];
    int64_t tot;
    int64_t before = block_exscan64(mine, &tot, lds_scan);
    if (threadIdx.x == 0) *s_digit = -1;
    __syncthreads();
    for (int j = 0; j < per; j++) {
      int64_t h = (int64_t)hist[threadIdx.x * per + j];
      if (before <= rem && before + h > rem) {
        *s_digit = threadIdx.x * per + j;
        *s_before = before;
      }
      before += h;
    }
    __syncthreads();
    int d = *s_digit;
    int64_t bef = *s_before;
    __syncthreads();
    if (d < 0) return;  // the whole side fits: nothing to exclude
    rem -= bef;
    prefix |= (uint32_t)d << shift;
    mask |= (uint32_t)(nbk - 1) << shift;
  }
  const int32_t y0 = (int32_t)prefix;
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
    int32_t u = list[i];
    if (A.part[u] == x && u >= y0) A.mark[u] = S + 1;
  }
  __syncthreads();
}

__global__ void __launch_bounds__(256) k_corridor(KArgs A) {
  __shared__ int8_t s_state[2 * FR_MAX_PAIRS];
  __shared__ int64_t s_W[2 * FR_MAX_PAIRS];
  __shared__ int16_t s_cross[2 * FR_MAX_PAIRS];
  __shared__ unsigned long long s_hist[2048];
  __shared__ int64_t s_scan[17];
  __shared__ int s_ncross, s_any, s_digit;
  __shared__ int64_t s_before;

  const int32_t S = A.ctl->stamp;
  const int P = A.P;
  const int NS = 2 * P;
  for (int i = threadIdx.x; i < NS; i += blockDim.x) {
    s_state[i] = A.ps[i >> 1].active ? SIDE_EXPAND : SIDE_DONE;
    s_W[i] = 0;
  }
  __syncthreads();

  // boundary nodes (level 0) and the pair cut
  GRID_WAVE_LOOP(u, A.n) {
    bool bnd = false;
    int key = -1;
    int64_t cw = 0, wv = 0;
    if (u < A.n) {
      int32_t x = A.part[u];
      int32_t p = A.blk2pair[x];
      if (p >= 0 && s_state[2 * p] == SIDE_EXPAND) {
        int32_t side = A.blk2side[x];
        int32_t y = side ? A.ps[p].a : A.ps[p].b;
        for (int32_t e = A.xadj[u]; e < A.xadj[u + 1]; e++)
          if (A.part[A.adjncy[e]] == y) {
            bnd = true;
            if (side == 0) cw += A.adjwgt[e];
          }
        if (bnd) {
          A.mark[u] = S;
          key = 2 * p + side;
          wv = A.vwgt[u];
        }
      }
    }
    int pos = wave_append(&A.ctl->cnt[0], bnd);
    if (bnd) put_bounded(A.f0, pos, A.n, (int32_t)u, A.ctl);
    // pair cut (side a only), boundary weights / counts per side
    wave_add_keyed(A.acc, FR_NACC, ACC_CUT, key >= 0 ? (key >> 1) : -1, cw);
    wave_add_keyed(A.lvlw, 1, 0, key, wv);
    {
      // boundary counts per side (one slot per call: the helper aggregates
      // lanes by key only)
      const bool sa = key >= 0 && (key & 1) == 0, sb = key >= 0 && (key & 1) == 1;
      wave_add_keyed(A.acc, FR_NACC, ACC_NDA, sa ? (key >> 1) : -1, sa ? 1 : 0);
      wave_add_keyed(A.acc, FR_NACC, ACC_NDB, sb ? (key >> 1) : -1, sb ? 1 : 0);
      wave_add_keyed(A.acc, FR_NACC, ACC_WDA, sa ? (key >> 1) : -1, wv);
    }
  }
  if (!grid_sync(A)) return;
  // level counts of level 0 come from the per-side boundary counts
  for (int lev = 0;; lev++) {
    const int cur = lev % 3, nxt = (lev + 1) % 3, nn2 = (lev + 2) % 3;
    const int32_t *flist = (lev & 1) ? A.f1 : A.f0;
    int32_t *nlist = (lev & 1) ? A.f0 : A.f1;
    const int32_t curcnt = min(A.ctl->cnt[cur], A.n);
    // decide, identically in every block
    for (int i = threadIdx.x; i < NS; i += blockDim.x) {
      if (s_state[i] != SIDE_EXPAND) continue;
      int64_t Lw = A.lvlw[cur * NS + i];
      int64_t Lc = lev == 0 ? A.acc[(i >> 1) * FR_NACC + ((i & 1) ? ACC_NDB : ACC_NDA)]
                            : (int64_t)A.lvlc[cur * NS + i];
      if (Lc == 0) {
        s_state[i] = SIDE_DONE;
        continue;
      }
      if (A.area_mode == FR_AREA_DEPTH) {
        s_W[i] += Lw;
        if (lev >= A.depth) s_state[i] = SIDE_DONE;
      } else {
        int64_t U = A.ps[i >> 1].U[i & 1];
        if (s_W[i] + Lw <= U) s_W[i] += Lw;
        else s_state[i] = SIDE_CROSS;
      }
    }
    __syncthreads();
    if (blockIdx.x == 0) {
      for (int i = threadIdx.x; i < NS; i += blockDim.x) {
        A.lvlw[nn2 * NS + i] = 0;
        A.lvlc[nn2 * NS + i] = 0;
      }
      if (threadIdx.x == 0) A.ctl->cnt[nn2] = 0;
    }
    // crossing sides in index order (deterministic across blocks)
    {
      const int per = (NS + blockDim.x - 1) / blockDim.x;
      int64_t mine = 0;
      for (int j = 0; j < per; j++) {
        int i = threadIdx.x * per + j;
        if (i < NS && s_state[i] == SIDE_CROSS) mine++;
      }
      int64_t tot;
      int64_t pos = block_exscan64(mine, &tot, s_scan);
      for (int j = 0; j < per; j++) {
        int i = threadIdx.x * per + j;
        if (i < NS && s_state[i] == SIDE_CROSS) s_cross[pos++] = (int16_t)i;
      }
      if (threadIdx.x == 0) s_ncross = (int)tot;
      __syncthreads();
    }
    for (int c = blockIdx.x; c < s_ncross; c += gridDim.x) {
      int i = s_cross[c];
      int p = i >> 1;
      int32_t x = (i & 1) ? A.ps[p].b : A.ps[p].a;
      select_level_prefix(A, x, flist, curcnt, A.ps[p].U[i & 1] - s_W[i], S, s_hist, s_scan,
                          &s_digit, &s_before);
    }
    __syncthreads();
    if (threadIdx.x == 0) s_any = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < NS; i += blockDim.x) {
      if (s_state[i] == SIDE_CROSS) s_state[i] = SIDE_DONE;
      if (s_state[i] == SIDE_EXPAND) s_any = 1;
    }
    __syncthreads();
    if (!s_any) break;
    // expand level lev -> lev + 1
    GRID_WAVE_LOOP(idx, curcnt) {
      int key = -1;
      int64_t wsum = 0, csum = 0;
      if (idx < curcnt) {
        int32_t u = flist[idx];
        int32_t x = A.part[u];
        int32_t p = A.blk2pair[x];
        int si = 2 * p + A.blk2side[x];
        if (s_state[si] == SIDE_EXPAND) {
          key = si;
          for (int32_t e = A.xadj[u]; e < A.xadj[u + 1]; e++) {
            int32_t v = A.adjncy[e];
            bool claim = false;
            if (A.part[v] == x && A.mark[v] < S) claim = atomicMax(&A.mark[v], S) < S;
            int pos = wave_append(&A.ctl->cnt[nxt], claim);
            if (claim) {
              put_bounded(nlist, pos, A.n, v, A.ctl);
              wsum += A.vwgt[v];
              csum += 1;
            }
          }
        }
      }
      wave_add_keyed(A.lvlw + nxt * NS, 1, 0, key, wsum);
      // counts (int32 array): rare mixed keys, plain atomics
      {
        int k0 = __shfl(key, 0);
        bool same = __ballot(key != k0 && csum != 0) == 0ull;
        if (same) {
          int64_t s = wave_sum64(k0 >= 0 ? csum : 0);
          if (lane64() == 0 && k0 >= 0 && s) atomicAdd(&A.lvlc[nxt * NS + k0], (int)s);
        } else if (key >= 0 && csum) {
          atomicAdd(&A.lvlc[nxt * NS + key], (int)csum);
        }
      }
    }
    if (threadIdx.x == 0 && blockIdx.x == 0) A.ctl->bfs_levels += 1;
    if (!grid_sync(A)) return;
  }
}

// ------------------------------------------------------------------------
// k_build

// Device-wide exclusive scan of flag/count values produced by `val(i)` for
// i in [0, N): writes out(i) for each i with the running prefix; returns the
// total (identical in every block).  Uses bsum[nblocks + 1].
template <typename ValF, typename OutF>
__device__ bool grid_exscan(const KArgs &A, int64_t N, ValF val, OutF out, int64_t *total,
                            int64_t *lds) {
  const int64_t T = blockDim.x;
  int64_t chunk = (N + gridDim.x - 1) / gridDim.x;
  chunk = (chunk + T - 1) / T * T;
  const int64_t lo = (int64_t)blockIdx.x * chunk;
  const int64_t hi = lo + chunk < N ? lo + chunk : N;
  int64_t mine = 0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += T) mine += val(i);
  int64_t bs = block_sum64(mine, lds);
  if (threadIdx.x == 0) A.bsum[blockIdx.x] = bs;
  if (!grid_sync(A)) return false;
  if (blockIdx.x == 0) {
    const int nb = gridDim.x;
    const int per = (nb + blockDim.x - 1) / blockDim.x;
    int64_t s = 0;
    for (int j = 0; j < per; j++) {
      int b = threadIdx.x * per + j;
      if (b < nb) s += A.bsum[b];
    }
    int64_t tot;
    int64_t run = block_exscan64(s, &tot, lds);
    for (int j = 0; j < per; j++) {
      int b = threadIdx.x * per + j;
      if (b < nb) {
        int64_t t = A.bsum[b];
        A.bsum[b] = run;
        run += t;
      }
    }
    if (threadIdx.x == 0) A.bsum[nb] = tot;
  }
  if (!grid_sync(A)) return false;
  int64_t run = A.bsum[blockIdx.x];
  *total = A.bsum[gridDim.x];
  for (int64_t t0 = lo; t0 < hi; t0 += T) {
    int64_t i = t0 + threadIdx.x;
    int64_t v = i < hi ? val(i) : 0;
    int64_t tt;
    int64_t ex = block_exscan64(v, &tt, lds);
    if (i < hi) out(i, run + ex, v);
    run += tt;
  }
  return grid_sync(A);
}

__global__ void __launch_bounds__(256) k_build(KArgs A) {
  __shared__ int64_t s_scan[17];
  const int32_t S = A.ctl->stamp;
  // 1. corridor vertices -> local ids in ascending global id
  int64_t nr = 0;
  if (!grid_exscan(
          A, A.n, [&](int64_t u) -> int64_t { return A.mark[u] == S ? 1 : 0; },
          [&](int64_t u, int64_t id, int64_t v) {
            if (v) {
              A.vmap[u] = (int32_t)id;
              A.lglob[id] = (int32_t)u;
            }
          },
          &nr, s_scan))
    return;
  if (blockIdx.x == 0 && threadIdx.x == 0) A.ctl->nr = (int32_t)nr;
  // 2. corridor degree, border flag, pair id, C_in
  GRID_WAVE_LOOP(i, nr) {
    int key = -1;
    int64_t cin = 0, cnt = 0, cap = 0;
    if (i < nr) {
      int32_t u = A.lglob[i];
      int32_t x = A.part[u];
      int32_t p = A.blk2pair[x];
      int32_t side = A.blk2side[x];
      uint32_t border = 0;
      for (int32_t e = A.xadj[u]; e < A.xadj[u + 1]; e++) {
        int32_t v = A.adjncy[e];
        int32_t xv = A.part[v];
        if (A.blk2pair[xv] != p) continue;
        if (A.mark[v] == S) {
          cnt++;
          cap += A.adjwgt[e];
          if (side == 0 && xv != x) cin += A.adjwgt[e];
        } else {
          border = LF_BORDER;
        }
      }
      A.ldeg[i] = (int32_t)cnt;
      A.lflag[i] = (uint8_t)((side ? LF_SIDE_B : 0u) | border);
      A.lpair[i] = p;
      key = p;
    }
    wave_add_keyed(A.acc, FR_NACC, ACC_CIN, key, cin);
    wave_add_keyed(A.acc, FR_NACC, ACC_RARCS, key, cnt);
    wave_add_keyed(A.acc, FR_NACC, ACC_CAP, key, cap);
    wave_add_keyed(A.acc, FR_NACC, ACC_RVERT, key, key >= 0 ? 1 : 0);
  }
  if (!grid_sync(A)) return;
  // 3. offsets of the local CSR
  int64_t na = 0;
  if (!grid_exscan(
          A, nr, [&](int64_t i) -> int64_t { return A.ldeg[i]; },
          [&](int64_t i, int64_t off, int64_t) { A.loff[i] = (int32_t)off; }, &na, s_scan))
    return;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    A.loff[nr] = (int32_t)na;
    A.ctl->na = (int32_t)na;
    A.ctl->nsink = 0;
  }
  // 4. arcs: head (local id) and capacity = edge weight in both directions
  GRID_WAVE_LOOP(i, nr) {
    if (i < nr) {
      int32_t u = A.lglob[i];
      int32_t p = A.lpair[i];
      int32_t k = A.loff[i];
      for (int32_t e = A.xadj[u]; e < A.xadj[u + 1]; e++) {
        int32_t v = A.adjncy[e];
        if (A.blk2pair[A.part[v]] == p && A.mark[v] == S) {
          A.lhead[k] = A.vmap[v];
          A.rcap[k] = A.adjwgt[e];
          k++;
        }
      }
    }
  }
  if (!grid_sync(A)) return;
  // 5. reverse arcs, initial preflow (every arc out of the source border is
  //    saturated), labels, sink list, closure marks
  const int32_t NL = (int32_t)nr + 2;
  GRID_WAVE_LOOP(i, nr) {
    bool snk = false;
    if (i < nr) {
      uint32_t f = A.lflag[i];
      bool src = LF_SRC(f);
      snk = LF_SNK(f);
      int32_t b = A.loff[i], e = A.loff[i + 1];
      int32_t ex = 0;
      for (int32_t a = b; a < e; a++) {
        int32_t j = A.lhead[a];
        int32_t jb = A.loff[j], je = A.loff[j + 1];
        int32_t r = jb;
        while (r < je && A.lhead[r] != (int32_t)i) r++;
        if (r == je) {  // asymmetric input slipped past validation
          A.ctl->err = FR_E_INVALID_GRAPH;
          A.ctl->diag = DIAG_REV;
          r = a;
        }
        A.lrev[a] = r;
        if (!src && LF_SRC(A.lflag[j])) {
          int32_t c = A.rcap[a];
          ex += c;
          A.rcap[a] = 2 * c;
          A.rcap[r] = 0;
        }
      }
      A.excess[i] = src ? 0 : ex;
      A.label[i] = snk ? 0 : (src ? NL + 1 : NL);
      A.ins[i] = 0;
    }
    int pos = wave_append(&A.ctl->nsink, snk);
    if (snk) put_bounded(A.sinks, pos, A.n, (int32_t)i, A.ctl);
  }
}

// ------------------------------------------------------------------------
// k_flow: push/relabel to a maximum preflow, then the smallest source set

struct FlowLoop {
  int ci;  // counter index: cnt[ci] = size of the current list
  int li;  // current list: li ? fb : fa
};

__device__ __forceinline__ int32_t *flist_of(const KArgs &A, int li) { return li ? A.fb : A.fa; }

// One push/relabel pass over the active list with `tpv` lanes per vertex
// (lock-free pushes: residuals and excess by atomics; labels read without
// synchronisation -- they only grow, and the exact global relabel decides
// termination).  Appends newly activated vertices and still-active ones to
// the next list.
template <int T>
__device__ void pr_sweep(const KArgs &A, const int32_t *cur, int32_t cnt, int32_t *next,
                         int32_t *next_cnt, int32_t NL) {
  const int lane = lane64();
  const int gl = lane & (T - 1);
  const int64_t gid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / T;
  const int64_t gstride = (int64_t)gridDim.x * blockDim.x / T;
  // wave-uniform trip count
  const int64_t wave_first = (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) & ~(int64_t)63) / T;
  for (int64_t base = wave_first; base < cnt; base += gstride) {
    const int64_t item = base + (gid - wave_first);
    bool valid = item < cnt;
    int32_t u = valid ? cur[item] : 0;
    // the group leader reads label and excess once and shares them: excess
    // may grow concurrently, and every lane must push against the same value
    int32_t d = NL, e = 0;
    if (valid && gl == 0) {
      d = A.label[u];
      e = A.excess[u];
    }
    if (T > 1) {
      d = __shfl(d, 0, T);
      e = __shfl(e, 0, T);
    }
    bool work = valid && d < NL && e > 0;
    int64_t erem = e;
    int64_t pushed = 0;
    int32_t minres = 0x7fffffff;
    int32_t ab = 0, ae = 0;
    if (work) {
      ab = A.loff[u];
      ae = A.loff[u + 1];
    }
    // all lanes of a group share ab/ae, so group-level shuffles stay converged
    for (int32_t a0 = ab; a0 < ae; a0 += T) {
      const int32_t a = a0 + gl;
      const bool in = a < ae;
      int32_t h = in ? A.lhead[a] : 0;
      int32_t r = in ? A.rcap[a] : 0;
      int32_t dh = (in && r > 0) ? A.label[h] : 0x7fffffff;
      int64_t adm = (r > 0 && dh < d) ? (int64_t)r : 0;
      // inclusive scan of adm inside the group
      int64_t inc = adm;
      if (T > 1) {
        for (int o = 1; o < T; o <<= 1) {
          int64_t t = __shfl_up(inc, o, T);
          if (gl >= o) inc += t;
        }
      }
      int64_t pre = inc - adm;
      int64_t tot = T > 1 ? __shfl(inc, T - 1, T) : inc;
      int64_t amt = 0;
      if (adm > 0 && erem > pre) amt = adm < erem - pre ? adm : erem - pre;
      if (amt > 0) {
        atomicSub(&A.rcap[a], (int32_t)amt);
        atomicAdd(&A.rcap[A.lrev[a]], (int32_t)amt);
        int32_t old = atomicAdd(&A.excess[h], (int32_t)amt);
        int pos = wave_append(next_cnt, old == 0 && dh > 0);
        if (old == 0 && dh > 0) put_bounded(next, pos, A.n, h, A.ctl);
      }
      if (r - amt > 0 && dh < minres) minres = dh;
      int64_t used = tot < erem ? tot : erem;
      erem -= used;
      pushed += used;
    }
    if (T > 1) {
      for (int o = T >> 1; o > 0; o >>= 1) {
        int32_t t = __shfl_xor(minres, o, T);
        minres = t < minres ? t : minres;
      }
    }
    bool again = false;
    if (work && gl == 0) {
      int32_t nd = d;
      if (erem > 0) {
        int64_t cand = minres == 0x7fffffff ? (int64_t)NL : (int64_t)minres + 1;
        if (cand > NL) cand = NL;
        if (cand > d) {
          nd = (int32_t)cand;
          A.label[u] = nd;
        }
      }
      int64_t left = e;
      if (pushed > 0) left = (int64_t)atomicSub(&A.excess[u], (int32_t)pushed) - pushed;
      again = left > 0 && nd < NL;
    }
    int pos = wave_append(next_cnt, again);
    if (again) put_bounded(next, pos, A.n, u, A.ctl);
  }
}

__device__ void pr_sweep_dispatch(const KArgs &A, const int32_t *cur, int32_t cnt, int32_t *next,
                                  int32_t *next_cnt, int32_t NL) {
  switch (A.tpv) {
    case 1: pr_sweep<1>(A, cur, cnt, next, next_cnt, NL); break;
    case 2: pr_sweep<2>(A, cur, cnt, next, next_cnt, NL); break;
    case 4: pr_sweep<4>(A, cur, cnt, next, next_cnt, NL); break;
    case 8: pr_sweep<8>(A, cur, cnt, next, next_cnt, NL); break;
    default: pr_sweep<16>(A, cur, cnt, next, next_cnt, NL); break;
  }
}

// Exact distance labels: BFS from the sink border backwards over residual
// arcs (v gets d+1 if the arc v -> w to a labelled w has residual capacity).
// Unreached vertices keep NL (inactive).  Leaves the active list (excess > 0,
// label < NL, not a terminal) as the current list.  Returns false on abort.
__device__ bool global_relabel(const KArgs &A, FlowLoop &L, int32_t NL, int32_t nr) {
  Ctl *C = A.ctl;
  GRID_WAVE_LOOP(i, nr) {
    if (i < nr) {
      uint32_t f = A.lflag[i];
      A.label[i] = LF_SNK(f) ? 0 : (LF_SRC(f) ? NL + 1 : NL);
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) C->cnt[(L.ci + 2) % 3] = 0;
  if (!grid_sync(A)) return false;
  const int32_t *cur = A.sinks;
  int32_t cnt = min(C->nsink, A.n);
  int32_t lev = 0;
  bool first = true;
  while (cnt > 0) {
    int32_t *next = flist_of(A, first ? L.li : (L.li ^ 1));
    int32_t *ncnt = &C->cnt[(L.ci + 1) % 3];
    GRID_WAVE_LOOP(idx, cnt) {
      if (idx < cnt) {
        int32_t w = cur[idx];
        for (int32_t a = A.loff[w]; a < A.loff[w + 1]; a++) {
          int32_t v = A.lhead[a];
          bool claim = false;
          if (A.label[v] == NL && A.rcap[A.lrev[a]] > 0)
            claim = atomicCAS(&A.label[v], NL, lev + 1) == NL;
          int pos = wave_append(ncnt, claim);
          if (claim) put_bounded(next, pos, A.n, v, C);
        }
      }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      C->cnt[(L.ci + 2) % 3] = 0;
      C->gr_levels += 1;
    }
    if (!grid_sync(A)) return false;
    L.ci = (L.ci + 1) % 3;
    if (!first) L.li ^= 1;
    first = false;
    cur = flist_of(A, L.li);
    cnt = min(C->cnt[L.ci], A.n);
    lev++;
  }
  // active list
  {
    int32_t *next = flist_of(A, L.li ^ 1);
    int32_t *ncnt = &C->cnt[(L.ci + 1) % 3];
    GRID_WAVE_LOOP(i, nr) {
      bool act = false;
      if (i < nr) {
        uint32_t f = A.lflag[i];
        act = !(f & LF_BORDER) && A.excess[i] > 0 && A.label[i] < NL;
      }
      int pos = wave_append(ncnt, act);
      if (act) put_bounded(next, pos, A.n, (int32_t)i, C);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      C->cnt[(L.ci + 2) % 3] = 0;
      C->relabels += 1;
    }
    if (!grid_sync(A)) return false;
    L.ci = (L.ci + 1) % 3;
    L.li ^= 1;
  }
  return true;
}

template <int TPB>
__global__ void __launch_bounds__(TPB) k_flow(KArgs A) {
  Ctl *C = A.ctl;
  const int32_t nr = C->nr;
  const int32_t NL = nr + 2;
  // capacity guard: every corridor's capacities must stay below 2^31
  for (int p = 0; p < A.P; p++)
    if (A.acc[p * FR_NACC + ACC_CAP] >= 0x7fffffffLL) {
      if (blockIdx.x == 0 && threadIdx.x == 0) C->err = FR_E_OVERFLOW;
      return;
    }
  if (blockIdx.x == 0 && threadIdx.x == 0) C->cnt[0] = C->cnt[1] = C->cnt[2] = 0;
  if (!grid_sync(A)) return;
  FlowLoop L{0, 0};
  if (!global_relabel(A, L, NL, nr)) return;
  int32_t cnt = min(C->cnt[L.ci], A.n);
  int since = 0;
  int64_t sweeps = 0;
  for (;;) {
    if (cnt == 0) {
      if (since == 0) break;
      if (!global_relabel(A, L, NL, nr)) return;
      since = 0;
      cnt = min(C->cnt[L.ci], A.n);
      continue;
    }
    if (sweeps >= A.max_sweeps) {
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        C->err = FR_E_SOLVER_LIMIT;
        C->diag = DIAG_SWEEPS;
      }
      return;
    }
    pr_sweep_dispatch(A, flist_of(A, L.li), cnt, flist_of(A, L.li ^ 1), &C->cnt[(L.ci + 1) % 3],
                      NL);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      C->cnt[(L.ci + 2) % 3] = 0;
      C->sweeps += 1;
    }
    if (!grid_sync(A)) return;
    L.ci = (L.ci + 1) % 3;
    L.li ^= 1;
    cnt = min(C->cnt[L.ci], A.n);
    sweeps++;
    if (++since >= A.relabel_period) {
      if (!global_relabel(A, L, NL, nr)) return;
      since = 0;
      cnt = min(C->cnt[L.ci], A.n);
    }
  }
  // smallest source set: closure of the source border and of every vertex
  // left with excess, over arcs with residual capacity
  {
    int32_t *next = flist_of(A, L.li ^ 1);
    int32_t *ncnt = &C->cnt[(L.ci + 1) % 3];
    GRID_WAVE_LOOP(i, nr) {
      bool seed = false;
      if (i < nr) {
        uint32_t f = A.lflag[i];
        seed = LF_SRC(f) || (!LF_SNK(f) && A.excess[i] > 0);
        if (seed) A.ins[i] = 1;
      }
      int pos = wave_append(ncnt, seed);
      if (seed) put_bounded(next, pos, A.n, (int32_t)i, C);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) C->cnt[(L.ci + 2) % 3] = 0;
    if (!grid_sync(A)) return;
    L.ci = (L.ci + 1) % 3;
    L.li ^= 1;
    cnt = min(C->cnt[L.ci], A.n);
  }
  while (cnt > 0) {
    const int32_t *cur = flist_of(A, L.li);
    int32_t *next = flist_of(A, L.li ^ 1);
    int32_t *ncnt = &C->cnt[(L.ci + 1) % 3];
    GRID_WAVE_LOOP(idx, cnt) {
      if (idx < cnt) {
        int32_t u = cur[idx];
        for (int32_t a = A.loff[u]; a < A.loff[u + 1]; a++) {
          bool claim = false;
          int32_t v = 0;
          if (A.rcap[a] > 0) {
            v = A.lhead[a];
            if (A.ins[v] == 0) claim = atomicCAS(&A.ins[v], 0, 1) == 0;
          }
          if (claim && LF_SNK(A.lflag[v])) {  // the preflow was not maximal
            C->err = FR_E_DEVICE;
            C->diag = DIAG_CLOSURE;
          }
          int pos = wave_append(ncnt, claim);
          if (claim) put_bounded(next, pos, A.n, v, C);
        }
      }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      C->cnt[(L.ci + 2) % 3] = 0;
      C->cl_levels += 1;
    }
    if (!grid_sync(A)) return;
    L.ci = (L.ci + 1) % 3;
    L.li ^= 1;
    cnt = min(C->cnt[L.ci], A.n);
  }
}

// ------------------------------------------------------------------------
// k_finish: reductions, decision, apply

__global__ void __launch_bounds__(256) k_finish(KArgs A, int32_t round) {
  __shared__ int64_t s_scan[17];
  Ctl *C = A.ctl;
  const int32_t nr = C->nr;
  GRID_WAVE_LOOP(i, nr) {
    int key = -1;
    int64_t fl = 0, ab = 0, ba = 0, src = 0;
    if (i < nr) {
      uint32_t f = A.lflag[i];
      key = A.lpair[i];
      int32_t w = A.vwgt[A.lglob[i]];
      bool in = A.ins[i] != 0;
      if (LF_SNK(f)) fl = A.excess[i];
      if (!(f & LF_SIDE_B) && !in) ab = w;
      if ((f & LF_SIDE_B) && in) ba = w;
      src = in ? 1 : 0;
    }
    wave_add_keyed(A.acc, FR_NACC, ACC_FLOW, key, fl);
    wave_add_keyed(A.acc, FR_NACC, ACC_MOVAB, key, ab);
    wave_add_keyed(A.acc, FR_NACC, ACC_MOVBA, key, ba);
    wave_add_keyed(A.acc, FR_NACC, ACC_SRC, key, src);
  }
  if (!grid_sync(A)) return;
  if (blockIdx.x == 0) {
    int64_t nact = 0;
    for (int p = threadIdx.x; p < A.P; p += blockDim.x) {
      PairState s = A.ps[p];
      int64_t *acc = A.acc + p * FR_NACC;
      if (s.active) {
        fr_solve rec;
        int64_t cut = acc[ACC_CUT];
        if (s.cut0 < 0) s.cut0 = cut;
        rec.alpha = s.alpha;
        rec.flow = acc[ACC_FLOW];
        rec.region_vertices = acc[ACC_RVERT];
        rec.region_edges = acc[ACC_RARCS] / 2;
        rec.source_side = acc[ACC_SRC];
        rec.cut_before = cut;
        int64_t cand = cut - acc[ACC_CIN] + acc[ACC_FLOW];
        int64_t wa = s.cA - acc[ACC_MOVAB] + acc[ACC_MOVBA];
        int64_t wb = s.cB + acc[ACC_MOVAB] - acc[ACC_MOVBA];
        int dec;
        if (cut == 0) {
          dec = FR_DEC_NOT_ADJACENT;
          cand = 0;
          wa = s.cA;
          wb = s.cB;
          rec.flow = 0;
        } else {
          bool feas = wa <= A.lmax && wb <= A.lmax;
          dec = !feas ? FR_DEC_INFEASIBLE : (cand < cut ? FR_DEC_APPLY : FR_DEC_EQUAL);
        }
        rec.cut_candidate = cand;
        rec.wa = wa;
        rec.wb = wb;
        rec.decision = dec;
        A.trace[(int64_t)p * A.max_iters + s.iters] = rec;
        s.iters++;
        s.final_alpha = s.alpha;
        s.flow_last = rec.flow;
        s.rv_sum += rec.region_vertices;
        s.re_sum += rec.region_edges;
        s.last_dec = dec;
        s.cut = cut;
        bool stop = false;
        if (dec == FR_DEC_APPLY) {
          s.applied++;
          s.cA = wa;
          s.cB = wb;
          s.cut = cand;
          if (!A.adaptive) stop = true;
          else s.alpha = 2 * s.alpha < A.alpha_max ? 2 * s.alpha : A.alpha_max;
        } else if (dec == FR_DEC_INFEASIBLE) {
          if (!A.adaptive || s.alpha == 1) stop = true;
          else s.alpha = s.alpha / 2 > 1 ? s.alpha / 2 : 1;
        } else {
          stop = true;
        }
        if (!stop && s.iters >= A.max_iters) {
          stop = true;
          s.iter_cap = 1;
        }
        s.stopped = stop;
        s.active = stop ? 0 : 1;
        if (!stop) {
          int64_t base = A.base[s.alpha];
          s.U[0] = base - s.cB > 0 ? base - s.cB : 0;
          s.U[1] = base - s.cA > 0 ? base - s.cA : 0;
        }
        A.ps[p] = s;
      }
      for (int j = 0; j < FR_NACC; j++) acc[j] = 0;
      for (int j = 0; j < 3; j++)
        for (int sd = 0; sd < 2; sd++) {
          A.lvlw[(j * A.P + p) * 2 + sd] = 0;
          A.lvlc[(j * A.P + p) * 2 + sd] = 0;
        }
      nact += A.ps[p].active;
    }
    int64_t tot = block_sum64(nact, s_scan);
    if (threadIdx.x == 0) {
      C->active_pairs = (int32_t)tot;
      C->cnt[0] = C->cnt[1] = C->cnt[2] = 0;
    }
  }
  if (!grid_sync(A)) return;
  GRID_WAVE_LOOP(i, nr) {
    if (i < nr) {
      int32_t p = A.lpair[i];
      const PairState &s = A.ps[p];
      if (s.last_dec == FR_DEC_APPLY && s.iters == round + 1)
        A.part[A.lglob[i]] = A.ins[i] ? s.a : s.b;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) C->stamp += 2;
}

// side codes of the last solve (single-pair calls)
__global__ void __launch_bounds__(256) k_side_out(KArgs A) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < A.n;
       u += (int64_t)gridDim.x * blockDim.x)
    A.side_out[u] = -1;
  __threadfence();
}

__global__ void __launch_bounds__(256) k_side_out2(KArgs A) {
  const int32_t nr = A.ctl->nr;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nr;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t f = A.lflag[i];
    int code = ((f & LF_BORDER) ? 2 : 0) + (A.ins[i] ? 0 : 1);
    A.side_out[A.lglob[i]] = (int8_t)code;
  }
}

// quotient graph adjacency: qadj[x*k + y] = 1 for blocks x < y sharing an edge
__global__ void __launch_bounds__(256) k_quotient(KArgs A, uint8_t *qadj) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < A.n;
       u += (int64_t)gridDim.x * blockDim.x) {
    int32_t x = A.part[u];
    for (int32_t e = A.xadj[u]; e < A.xadj[u + 1]; e++) {
      int32_t y = A.part[A.adjncy[e]];
      if (x < y) qadj[(int64_t)x * A.k + y] = 1;
    }
  }
}

// total cut sum_{i<j} omega(E_ij), counted from the lower-id end of each edge
__global__ void __launch_bounds__(256) k_total_cut(KArgs A, int64_t *out) {
  __shared__ int64_t s_red[17];
  int64_t c = 0;
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < A.n;
       u += (int64_t)gridDim.x * blockDim.x) {
    int32_t x = A.part[u];
    for (int32_t e = A.xadj[u]; e < A.xadj[u + 1]; e++) {
      int32_t v = A.adjncy[e];
      if (v > u && A.part[v] != x) c += A.adjwgt[e];
    }
  }
  int64_t t = block_sum64(c, s_red);
  if (threadIdx.x == 0 && t) atomicAdd((unsigned long long *)out, (unsigned long long)t);
}
