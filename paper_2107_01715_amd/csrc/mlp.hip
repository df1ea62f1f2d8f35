// Batch-BFS over a learned forward model: the fully connected stand-in for a
// learned simulator of the paper's runtime study (Sec. 4.1: three hidden
// layers of width 100 fed a 100-dimensional state and a one-hot action).
//
// The model maps x = [s ; onehot(a)] through three ReLU layers of width 100
// to a linear output of 101 units (next state, then reward); a leaf state is
// valued by the linear head Q(s, .) = Wq s + bq.  All roots of one call share
// A and the depth, so child c of level k has parent c / A at level k - 1 and
// the leaves of root r, root action a0 form the contiguous block
// [(r A + a0) A^(d-1), (r A + a0 + 1) A^(d-1)).
//
// FP32 throughout.  On CDNA4 the FP32 matrix cores have the same peak as the
// FP32 vector units (157.3 TFLOP/s), and at width 100 the work per child is
// small next to its state traffic, so the layers run as register-tiled FMA
// loops: a workgroup takes 64 children (8 on small levels), keeps their
// activations in LDS and each thread owns one output unit of 32 (4) children.  Every sum runs in a fixed
// order (bias, the action column, then k = 0..99), so results do not depend
// on batching.
#include "bcts_internal.h"

namespace bcts {
namespace {

constexpr int kS = 100;          // state / hidden width
constexpr int kMT = 64;          // children per tile (large levels)
constexpr int kMTs = 8;          // children per tile (small levels)
constexpr int kXS = 104;         // LDS row stride in floats (16-byte aligned rows)
constexpr int kThreads = 256;

// Y[r][col] for this thread's R rows: bias[col] (+ extra[r]) + sum_k W[col][k] X[r][k].
// Large tiles (R = 32) read their weight row one float4 per K step; small
// tiles (R <= 8, used when a level has few children and a lone tile is
// latency-bound) request the whole row at once into registers.
template <bool RELU, int R>
__device__ __forceinline__ void dense(const float* __restrict__ W, const float* __restrict__ bias, int nout,
                                      const float* X, float* Y, int col, int rh, const float* extra) {
  if (col < nout) {
    float acc[R];
    const float b = bias[col];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = b + (extra ? extra[r] : 0.f);
    const float4* wr = reinterpret_cast<const float4*>(W + (size_t)col * kS);
    if constexpr (R <= 8) {
      float4 wv[kS / 4];
#pragma unroll
      for (int k4 = 0; k4 < kS / 4; ++k4) wv[k4] = wr[k4];
#pragma unroll
      for (int k4 = 0; k4 < kS / 4; ++k4) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const float4 x = *reinterpret_cast<const float4*>(X + (rh * R + r) * kXS + 4 * k4);
          acc[r] = fmaf(wv[k4].x, x.x, acc[r]);
          acc[r] = fmaf(wv[k4].y, x.y, acc[r]);
          acc[r] = fmaf(wv[k4].z, x.z, acc[r]);
          acc[r] = fmaf(wv[k4].w, x.w, acc[r]);
        }
      }
    } else {
      for (int k4 = 0; k4 < kS / 4; ++k4) {
        const float4 w = wr[k4];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const float4 x = *reinterpret_cast<const float4*>(X + (rh * R + r) * kXS + 4 * k4);
          acc[r] = fmaf(w.x, x.x, acc[r]);
          acc[r] = fmaf(w.y, x.y, acc[r]);
          acc[r] = fmaf(w.z, x.z, acc[r]);
          acc[r] = fmaf(w.w, x.w, acc[r]);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) Y[(rh * R + r) * kXS + col] = RELU ? fmaxf(acc[r], 0.f) : acc[r];
  }
}

// One level of the tree: children c in [0, n) of parents c / A.
//   ps    parent states [n / A][100] (the roots at level 1), pret their
//         returns (null at level 1: the root's return is 0)
//   gpow  gamma^(k-1), the discount of this level's reward
//   os    child states (null: not kept), oret child returns (null: not kept)
//   ov    max_a Q(child, a) (null: not needed)
//   oleaf return + gamma^d max_a Q (null: not a leaf level)
template <int MT>
__global__ void __launch_bounds__(kThreads) mlp_level_kernel(MlpDev m, long long n, const float* __restrict__ ps,
                                                             const float* __restrict__ pret, float gpow,
                                                             float* __restrict__ os, float* __restrict__ oret,
                                                             float* __restrict__ ov, float* __restrict__ oleaf,
                                                             float gamma_d) {
  constexpr int R = MT / 2;                    // rows per thread: 2 row halves x 128 units
  __shared__ __attribute__((aligned(16))) float xa[MT * kXS];
  __shared__ __attribute__((aligned(16))) float xb[MT * kXS];
  __shared__ float rwd[MT];
  const int tid = threadIdx.x, col = tid & 127, rh = tid >> 7;
  const int A = m.A;
  const bool head = ov || oleaf;
  for (long long c0 = (long long)blockIdx.x * MT; c0 < n; c0 += (long long)gridDim.x * MT) {
    // parent states; rows past n repeat the last child (computed, never stored)
    for (int e = tid; e < MT * (kS / 4); e += kThreads) {
      const int row = e / (kS / 4), q = e % (kS / 4);
      const long long c = (c0 + row < n) ? c0 + row : n - 1;
      const float4 v = reinterpret_cast<const float4*>(ps + (c / A) * kS)[q];
      *reinterpret_cast<float4*>(&xa[row * kXS + 4 * q]) = v;
    }
    __syncthreads();
    // layer 1: the one-hot action selects one column of l1.w
    {
      float extra[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        long long c = c0 + rh * R + r;
        if (c >= n) c = n - 1;
        extra[r] = col < kS ? m.w1a[(size_t)(c % A) * kS + col] : 0.f;
      }
      dense<true, R>(m.w1s, m.b1, kS, xa, xb, col, rh, extra);
    }
    __syncthreads();
    dense<true, R>(m.w2, m.b2, kS, xb, xa, col, rh, nullptr);
    __syncthreads();
    dense<true, R>(m.w3, m.b3, kS, xa, xb, col, rh, nullptr);
    __syncthreads();
    dense<false, R>(m.wo, m.bo, kS + 1, xb, xa, col, rh, nullptr);   // units 0..99 next state, 100 reward
    __syncthreads();
    if (tid < MT) rwd[tid] = xa[tid * kXS + kS];
    __syncthreads();
    // returns and states
    if (tid < MT && c0 + tid < n) {
      const long long c = c0 + tid;
      const float r = fmaf(gpow, rwd[tid], pret ? pret[c / A] : 0.f);
      rwd[tid] = r;                           // now the child's return
      if (oret) oret[c] = r;
    } else if (tid < MT) {
      rwd[tid] = 0.f;
    }
    if (os)
      for (int e = tid; e < MT * (kS / 4); e += kThreads) {
        const int row = e / (kS / 4), q = e % (kS / 4);
        if (c0 + row < n)
          reinterpret_cast<float4*>(os + (c0 + row) * kS)[q] = *reinterpret_cast<const float4*>(&xa[row * kXS + 4 * q]);
      }
    __syncthreads();
    // leaf head: 4 lanes per child, actions a = part, part + 4, ...
    if (head) {
      const int row = (tid >> 2) < MT ? (tid >> 2) : MT - 1, part = tid & 3;
      float vmax = -INFINITY;
      for (int a = part; a < A; a += 4) {
        float acc = m.bq[a];
        const float4* wr = reinterpret_cast<const float4*>(m.wq + (size_t)a * kS);
        for (int k4 = 0; k4 < kS / 4; ++k4) {
          const float4 w = wr[k4];
          const float4 x = *reinterpret_cast<const float4*>(&xa[row * kXS + 4 * k4]);
          acc = fmaf(w.x, x.x, acc);
          acc = fmaf(w.y, x.y, acc);
          acc = fmaf(w.z, x.z, acc);
          acc = fmaf(w.w, x.w, acc);
        }
        vmax = fmaxf(vmax, acc);
      }
      vmax = fmaxf(vmax, __shfl_xor(vmax, 1));
      vmax = fmaxf(vmax, __shfl_xor(vmax, 2));
      if (part == 0 && (tid >> 2) < MT && c0 + row < n) {
        const long long c = c0 + row;
        if (ov) ov[c] = vmax;
        if (oleaf) oleaf[c] = fmaf(gamma_d, vmax, rwd[row]);
      }
    }
    __syncthreads();
  }
}

// q_d[b] = max over leaf block b (block elements contiguous)
__global__ void __launch_bounds__(kThreads) mlp_blockmax_kernel(long long block, const float* __restrict__ leaf,
                                                                float* __restrict__ qd) {
  __shared__ float red[kThreads];
  const long long b = blockIdx.x;
  float v = -INFINITY;
  for (long long i = threadIdx.x; i < block; i += kThreads) v = fmaxf(v, leaf[b * block + i]);
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) qd[b] = red[0];
}

// Per root (one wavefront): Q0 = Wq s + bq, then for d >= 1 the BCTS
// correction (Eq. 3 with B = pen_e d_e - pen_o d_o of Eq. 6 or Lemma 3.2):
// pi_o = argmax Q0 (lowest index), delta_a = r_a + gamma max Q(s1^a) - Q0_a
// from the level-1 returns and head values, d_o = |delta_pi_o|, d_e the mean
// of |delta_a| over a != pi_o (summed in index order); every a != pi_o moves
// by scale gamma^d B.  Output q [n][A] and the argmax action (lowest index).
__global__ void __launch_bounds__(64) mlp_root_kernel(MlpDev m, int d, const float* __restrict__ states,
                                                      const float* __restrict__ ret1,
                                                      const float* __restrict__ v1,
                                                      const float* __restrict__ qd, float gamma, float gamma_d,
                                                      float pen_e, float pen_o, int corr, float scale,
                                                      int32_t* __restrict__ act, float* __restrict__ q) {
  __shared__ float q0s[kMaxA], dels[kMaxA], outs[kMaxA];
  const int r = blockIdx.x, lane = threadIdx.x, A = m.A;
  if (lane < A) {
    float acc = m.bq[lane];
    const float* s = states + (size_t)r * kS;
    for (int k = 0; k < kS; ++k) acc = fmaf(m.wq[(size_t)lane * kS + k], s[k], acc);
    q0s[lane] = acc;
    if (d >= 1 && corr) dels[lane] = fmaf(gamma, v1[(size_t)r * A + lane], ret1[(size_t)r * A + lane]) - acc;
  }
  __syncthreads();
  if (lane == 0) {
    if (d == 0) {
      for (int a = 0; a < A; ++a) outs[a] = q0s[a];
    } else {
      for (int a = 0; a < A; ++a) outs[a] = qd[(size_t)r * A + a];
      if (corr) {
        int pi = 0;
        for (int a = 1; a < A; ++a)
          if (q0s[a] > q0s[pi]) pi = a;
        const float dobs = fabsf(dels[pi]);
        float se = 0.f;
        for (int a = 0; a < A; ++a)
          if (a != pi) se += fabsf(dels[a]);
        const float de = se / (float)(A - 1);
        // one rounding of pen_e d_e - pen_o d_o (the host search does the same)
        const float shift = scale * gamma_d * fmaf(pen_e, de, -(pen_o * dobs));
        for (int a = 0; a < A; ++a)
          if (a != pi) outs[a] -= shift;
      }
    }
    int best = 0;
    for (int a = 1; a < A; ++a)
      if (outs[best] < outs[a]) best = a;
    act[r] = best;
  }
  __syncthreads();
  if (lane < A) q[(size_t)r * A + lane] = outs[lane];
}

}  // namespace

void launch_mlp_level(const MlpDev& m, long long n, const float* ps, const float* pret, float gpow, float* os,
                      float* oret, float* ov, float* oleaf, float gamma_d, hipStream_t s) {
  if (n <= 0) return;
  // a level with fewer than ~2 large tiles per CU runs in small tiles: more
  // workgroups, 4 rows per thread, weights requested at once
  if (n < 2LL * 256 * kMT) {
    const long long tiles = (n + kMTs - 1) / kMTs;
    hipLaunchKernelGGL(mlp_level_kernel<kMTs>, dim3((unsigned)tiles), dim3(kThreads), 0, s, m, n, ps, pret, gpow,
                       os, oret, ov, oleaf, gamma_d);
    return;
  }
  const long long tiles = (n + kMT - 1) / kMT;
  const unsigned grid = (unsigned)(tiles < 65536 ? tiles : 65536);
  hipLaunchKernelGGL(mlp_level_kernel<kMT>, dim3(grid), dim3(kThreads), 0, s, m, n, ps, pret, gpow, os, oret, ov,
                     oleaf, gamma_d);
}

void launch_mlp_blockmax(long long n_blocks, long long block, const float* leaf, float* qd, hipStream_t s) {
  if (n_blocks <= 0) return;
  hipLaunchKernelGGL(mlp_blockmax_kernel, dim3((unsigned)n_blocks), dim3(kThreads), 0, s, block, leaf, qd);
}

void launch_mlp_root(const MlpDev& m, int n, int d, const float* states, const float* ret1, const float* v1,
                     const float* qd, float gamma, float gamma_d, float pen_e, float pen_o, int corr, float scale,
                     int32_t* act, float* q, hipStream_t s) {
  hipLaunchKernelGGL(mlp_root_kernel, dim3((unsigned)n), dim3(64), 0, s, m, d, states, ret1, v1, qd, gamma, gamma_d,
                     pen_e, pen_o, corr, scale, act, q);
}

}  // namespace bcts
