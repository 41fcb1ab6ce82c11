// Learned area factor: a small MLP that proposes the start factor alpha of
// each pair's adaptive flow iterations.  It has no counterpart in the paper;
// the plain adaptive search (Sec. 4.1) keeps running from the proposed
// factor, so the flow results stay exact; the search from alpha' is the
// reference for cut quality.
//
// Network: 8 features -> 64 -> 64 -> 5 classes (alpha = 1, 2, 4, 8, 16),
// ReLU hidden layers, softmax cross-entropy.  FP32 throughout, plain FMA
// (5 k parameters, no dense contraction worth a matrix core).  Parameters are
// one float array: W1[8][64], b1[64], W2[64][64], b2[64], W3[64][5], b3[5]
// (row-major [in][out]).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fr_internal.h"

#define MLP_IN 8
#define MLP_H 64
#define MLP_OUT 5
#define MLP_W1 0
#define MLP_B1 (MLP_W1 + MLP_IN * MLP_H)
#define MLP_W2 (MLP_B1 + MLP_H)
#define MLP_B2 (MLP_W2 + MLP_H * MLP_H)
#define MLP_W3 (MLP_B2 + MLP_H)
#define MLP_B3 (MLP_W3 + MLP_H * MLP_OUT)
#define MLP_NPARAMS (MLP_B3 + MLP_OUT)
#define MLP_SAMPLES_PER_BLOCK 16  // 16 samples x 64 units = 1024 threads

// Per-pair boundary statistics for the features: [P][4] = boundary vertices
// of a, of b, boundary weight of a, pair cut.  Grid over all vertices.
__global__ void __launch_bounds__(256) k_feature_stats(KArgs A, int64_t *acc) {
  __shared__ uint32_t s_bnd[256];
  __shared__ unsigned long long s_cw[256];
  const int lane = lane64();
  const int wl = (int)(threadIdx.x & ~63u);
  unsigned long long *ac = (unsigned long long *)acc;
  // boundary count a / b, boundary weight a, cut weight; keyed by pair
  KeyedSums<4> sums;
  auto out = [&](int j, int key, int64_t v) { wave_add_by_key(ac, 4, j, key, v); };
  wave_chunk_runs(A, [&](int64_t u0, int32_t blk, int32_t x0) {
    const int64_t u = u0 + lane;
    const int64_t last = min((int64_t)A.n, u0 + 64);
    int32_t p = -1, y2 = -1;
    int64_t w = 0;
    if (u < last) {
      const int32_t x = blk;
      p = A.blk2pair[x];
      if (p >= 0) {
        const int32_t a = A.pairs[2 * p], b = A.pairs[2 * p + 1];
        const int side = x == b;
        y2 = ((side ? a : b) << 1) | side;
        w = A.vwgt[u];
      }
    }
    bool bnd;
    int64_t cw;
    chunk_boundary(A, x0, y2, __shfl(x0, 0), A.xadj[last], s_bnd + wl, s_cw + wl, bnd, cw);
    const int side = y2 & 1;
    const int64_t x[4] = {bnd && !side ? 1 : 0, bnd && side ? 1 : 0, bnd && !side ? w : 0, cw};
    sums.add(p, x, out);
  });
  sums.flush(out);
}

// The 8 features of every pair (FP32): log2(1+|dA|), log2(1+|dB|), c(A)/W,
// c(B)/W, log2(1+cut), (Lmax-c(A))/W, (Lmax-c(B))/W, log2(1 + U_A(1)/c(dA))
// with W = c(V)/k and U_A(1) the alpha = 1 area bound of side a.
__global__ void __launch_bounds__(256) k_features(KArgs A, const int64_t *acc, float *feats) {
  const int64_t cV = A.ctl->cV;
  const double W = (double)cV / (double)A.k > 0 ? (double)cV / (double)A.k : 1.0;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < A.P; p += gridDim.x * blockDim.x) {
    const int32_t a = A.pairs[2 * p], b = A.pairs[2 * p + 1];
    const int64_t cA = A.bstat[a], cB = A.bstat[b];
    const int64_t *s = acc + 4 * p;
    int64_t u1 = A.base[1] - cB;
    u1 = u1 > 0 ? u1 : 0;
    const double wda = s[2] > 1 ? (double)s[2] : 1.0;
    float *f = feats + (int64_t)MLP_IN * p;
    f[0] = (float)log2(1.0 + (double)s[0]);
    f[1] = (float)log2(1.0 + (double)s[1]);
    f[2] = (float)((double)cA / W);
    f[3] = (float)((double)cB / W);
    f[4] = (float)log2(1.0 + (double)s[3]);
    f[5] = (float)((double)(A.lmax - cA) / W);
    f[6] = (float)((double)(A.lmax - cB) / W);
    f[7] = (float)log2(1.0 + (double)u1 / wda);
  }
}

// Forward pass: MLP_SAMPLES_PER_BLOCK samples per block, one thread per
// (sample, hidden unit).  Writes the class probabilities and, when act is
// given, the activations a1, h1, a2, h2 ([n][64] each, in that order) for
// the backward pass.
__global__ void __launch_bounds__(1024) k_mlp_forward(const float *prm, const float *x, int32_t n,
                                                      float *probs, float *act) {
  __shared__ float s_x[MLP_SAMPLES_PER_BLOCK][MLP_IN];
  __shared__ float s_h1[MLP_SAMPLES_PER_BLOCK][MLP_H];
  __shared__ float s_h2[MLP_SAMPLES_PER_BLOCK][MLP_H];
  __shared__ float s_z[MLP_SAMPLES_PER_BLOCK][MLP_OUT];
  const int ls = threadIdx.x / MLP_H, j = threadIdx.x % MLP_H;
  const int s = blockIdx.x * MLP_SAMPLES_PER_BLOCK + ls;
  const bool ok = s < n;
  if (j < MLP_IN) s_x[ls][j] = ok ? x[(int64_t)s * MLP_IN + j] : 0.f;
  __syncthreads();
  float a1 = prm[MLP_B1 + j];
  for (int i = 0; i < MLP_IN; i++) a1 = fmaf(s_x[ls][i], prm[MLP_W1 + i * MLP_H + j], a1);
  const float h1 = a1 > 0.f ? a1 : 0.f;
  s_h1[ls][j] = h1;
  __syncthreads();
  float a2 = prm[MLP_B2 + j];
  for (int i = 0; i < MLP_H; i++) a2 = fmaf(s_h1[ls][i], prm[MLP_W2 + i * MLP_H + j], a2);
  const float h2 = a2 > 0.f ? a2 : 0.f;
  s_h2[ls][j] = h2;
  __syncthreads();
  if (j < MLP_OUT) {
    float z = prm[MLP_B3 + j];
    for (int i = 0; i < MLP_H; i++) z = fmaf(s_h2[ls][i], prm[MLP_W3 + i * MLP_OUT + j], z);
    s_z[ls][j] = z;
  }
  __syncthreads();
  if (ok && j == 0) {
    float zm = s_z[ls][0];
    for (int c = 1; c < MLP_OUT; c++) zm = fmaxf(zm, s_z[ls][c]);
    float e[MLP_OUT], sum = 0.f;
    for (int c = 0; c < MLP_OUT; c++) {
      e[c] = expf(s_z[ls][c] - zm);
      sum += e[c];
    }
    for (int c = 0; c < MLP_OUT; c++) probs[(int64_t)s * MLP_OUT + c] = e[c] / sum;
  }
  if (ok && act) {
    const int64_t base = (int64_t)s * MLP_H + j, stride = (int64_t)n * MLP_H;
    act[base] = a1;
    act[stride + base] = h1;
    act[2 * stride + base] = a2;
    act[3 * stride + base] = h2;
  }
}

// Backward through the activations of each sample, for the mean softmax
// cross-entropy (labels): dz = (p - onehot) / n; or, with per-class costs
// [n][5], for the mean expected cost sum_c p_c cost_c: dz_j = p_j (cost_j -
// sum_c p_c cost_c) / n.  Then da2 = (dz W3^T) * [a2 > 0], da1 = (da2 W2^T) *
// [a1 > 0].  dact = dz [n][5], da2 [n][64], da1 [n][64].
__global__ void __launch_bounds__(1024) k_mlp_backward(const float *prm, const float *probs,
                                                       const int32_t *labels, const float *costs,
                                                       int32_t n, const float *act, float *dact) {
  __shared__ float s_dz[MLP_SAMPLES_PER_BLOCK][MLP_OUT];
  __shared__ float s_da2[MLP_SAMPLES_PER_BLOCK][MLP_H];
  const int ls = threadIdx.x / MLP_H, j = threadIdx.x % MLP_H;
  const int s = blockIdx.x * MLP_SAMPLES_PER_BLOCK + ls;
  const bool ok = s < n;
  const int64_t stride = (int64_t)n * MLP_H;
  if (j < MLP_OUT) {
    float dz = 0.f;
    if (ok && costs) {
      const float *pr = probs + (int64_t)s * MLP_OUT, *cs = costs + (int64_t)s * MLP_OUT;
      float pc = 0.f;
      for (int c = 0; c < MLP_OUT; c++) pc = fmaf(pr[c], cs[c], pc);
      dz = pr[j] * (cs[j] - pc) / (float)n;
    } else if (ok) {
      dz = (probs[(int64_t)s * MLP_OUT + j] - (labels[s] == j ? 1.f : 0.f)) / (float)n;
    }
    s_dz[ls][j] = dz;
    if (ok) dact[(int64_t)s * MLP_OUT + j] = dz;
  }
  __syncthreads();
  float dh2 = 0.f;
  for (int c = 0; c < MLP_OUT; c++) dh2 = fmaf(s_dz[ls][c], prm[MLP_W3 + j * MLP_OUT + c], dh2);
  const float a2 = ok ? act[2 * stride + (int64_t)s * MLP_H + j] : 0.f;
  const float da2 = a2 > 0.f ? dh2 : 0.f;
  s_da2[ls][j] = da2;
  __syncthreads();
  float dh1 = 0.f;
  for (int k2 = 0; k2 < MLP_H; k2++) dh1 = fmaf(s_da2[ls][k2], prm[MLP_W2 + j * MLP_H + k2], dh1);
  const float a1 = ok ? act[(int64_t)s * MLP_H + j] : 0.f;
  const float da1 = a1 > 0.f ? dh1 : 0.f;
  if (ok) {
    const int64_t o = (int64_t)n * MLP_OUT;
    dact[o + (int64_t)s * MLP_H + j] = da2;
    dact[o + stride + (int64_t)s * MLP_H + j] = da1;
  }
}

// Parameter gradients, one thread per parameter, summing over the samples in
// index order (deterministic): dW1 = x^T da1, db1 = sum da1, dW2 = h1^T da2,
// db2 = sum da2, dW3 = h2^T dz, db3 = sum dz.
__global__ void __launch_bounds__(256) k_mlp_grad(const float *x, const float *act,
                                                  const float *dact, int32_t n, float *grad) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= MLP_NPARAMS) return;
  const int64_t stride = (int64_t)n * MLP_H;
  const float *dz = dact, *da2 = dact + (int64_t)n * MLP_OUT, *da1 = da2 + stride;
  const float *h1 = act + stride, *h2 = act + 3 * stride;
  float g = 0.f;
  if (t < MLP_B1) {
    const int i = t / MLP_H, j = t % MLP_H;
    for (int s = 0; s < n; s++) g = fmaf(x[(int64_t)s * MLP_IN + i], da1[(int64_t)s * MLP_H + j], g);
  } else if (t < MLP_W2) {
    const int j = t - MLP_B1;
    for (int s = 0; s < n; s++) g += da1[(int64_t)s * MLP_H + j];
  } else if (t < MLP_B2) {
    const int i = (t - MLP_W2) / MLP_H, j = (t - MLP_W2) % MLP_H;
    for (int s = 0; s < n; s++) g = fmaf(h1[(int64_t)s * MLP_H + i], da2[(int64_t)s * MLP_H + j], g);
  } else if (t < MLP_W3) {
    const int j = t - MLP_B2;
    for (int s = 0; s < n; s++) g += da2[(int64_t)s * MLP_H + j];
  } else if (t < MLP_B3) {
    const int i = (t - MLP_W3) / MLP_OUT, c = (t - MLP_W3) % MLP_OUT;
    for (int s = 0; s < n; s++) g = fmaf(h2[(int64_t)s * MLP_H + i], dz[(int64_t)s * MLP_OUT + c], g);
  } else {
    const int c = t - MLP_B3;
    for (int s = 0; s < n; s++) g += dz[(int64_t)s * MLP_OUT + c];
  }
  grad[t] = g;
}

// mean cross-entropy of n samples (labels), or their mean expected cost
// (costs [n][5]); one block
__global__ void __launch_bounds__(256) k_mlp_loss(const float *probs, const int32_t *labels,
                                                  const float *costs, int32_t n, float *loss) {
  __shared__ double s_red[256];
  double acc = 0.0;
  for (int s = threadIdx.x; s < n; s += blockDim.x) {
    if (costs) {
      for (int c = 0; c < MLP_OUT; c++)
        acc += (double)probs[(int64_t)s * MLP_OUT + c] * (double)costs[(int64_t)s * MLP_OUT + c];
    } else {
      const float p = probs[(int64_t)s * MLP_OUT + labels[s]];
      acc -= log((double)fmaxf(p, 1e-30f));
    }
  }
  s_red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) s_red[threadIdx.x] += s_red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = (float)(s_red[0] / (n > 0 ? n : 1));
}

// Adam (Kingma & Ba 2015) with bias correction; t >= 1.
__global__ void __launch_bounds__(256) k_adam(float *prm, const float *grad, float *m, float *v,
                                              float lr, float b1, float b2, float eps, int32_t t) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= MLP_NPARAMS) return;
  const float g = grad[i];
  const float mi = b1 * m[i] + (1.f - b1) * g;
  const float vi = b2 * v[i] + (1.f - b2) * g * g;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / (1.f - powf(b1, (float)t));
  const float vh = vi / (1.f - powf(b2, (float)t));
  prm[i] -= lr * mh / (sqrtf(vh) + eps);
}

// rows idx[0..m) of (x, labels or costs) into (xb, lb or cb)
static_assert(MLP_IN >= MLP_OUT, "a row's costs are gathered by its feature lanes");
__global__ void __launch_bounds__(256) k_gather_rows(const float *x, const int32_t *labels,
                                                     const float *costs, const int32_t *idx,
                                                     int32_t m, float *xb, int32_t *lb,
                                                     float *cb) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m * MLP_IN) return;
  const int r = t / MLP_IN, c = t % MLP_IN;
  xb[t] = x[(int64_t)idx[r] * MLP_IN + c];
  if (costs) {
    if (c < MLP_OUT) cb[r * MLP_OUT + c] = costs[(int64_t)idx[r] * MLP_OUT + c];
  } else if (c == 0) {
    lb[r] = labels[idx[r]];
  }
}

// start factor of each pair from the predicted class (first maximum, i.e.
// the smaller factor on ties)
__global__ void __launch_bounds__(256) k_alpha_from_probs(const float *probs, int32_t P,
                                                          int32_t *alpha0) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  int best = 0;
  for (int c = 1; c < MLP_OUT; c++)
    if (probs[(int64_t)p * MLP_OUT + c] > probs[(int64_t)p * MLP_OUT + best]) best = c;
  alpha0[p] = 1 << best;
}
