// Backup and root correction, one wavefront per root.
//
//  * Backup (Eq. 1 / Alg. 1, final steps): a leaf's value is its discounted
//    return plus gamma^d max_a Q(leaf, a); the leaves of root action a0 are
//    the contiguous block [a0 A^(d-1), (a0+1) A^(d-1)) of the root's leaves
//    (blocks of leaf_blk leaves when a beam cut the tree: the surviving
//    leaves stay grouped by root action), so Q_d(a0) is a max-reduction over
//    that block.
//  * Correction (Eq. 3 with B of Eq. 6 or the exact gap of Lemma 3.2):
//    pi_o = argmax of the network at the root, the depth-1 Bellman errors
//    delta(a) = r_a + gamma V(s_1^a) - Q_0(a) (Prop. 3.6), d_o = |delta(pi_o)|,
//    d_e = mean of |delta(a)| over the other actions, B = pen_e d_e - pen_o d_o
//    (pen_e, pen_o fixed by A and d, computed on the host); every a != pi_o
//    loses c gamma^d B.
//  * Action: argmax of the returned vector, lowest index on ties (Eq. 4).
// Everything is FP32; max is exact, so the result does not depend on the
// reduction order.
#include "bcts_internal.h"

namespace bcts {
namespace {

__device__ __forceinline__ float wave_max(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}

__global__ void __launch_bounds__(64)
backup_kernel(int n_roots, const RootInfo* __restrict__ roots, const float* __restrict__ V,
              const float* __restrict__ q0, LevelRet level_ret, float gamma, float corr_scale, int* __restrict__ out_action,
              float* __restrict__ out_q) {
  const int r = blockIdx.x;
  if (r >= n_roots) return;
  const int lane = threadIdx.x;
  const RootInfo ri = roots[r];
  const int A = ri.A, d = ri.d;
  __shared__ float q[kMaxA];

  if (d == 0) {
    if (lane < A) q[lane] = q0[(long long)r * kMaxA + lane];
  } else {
    const long long blk = ri.leaf_blk;          // A^(d-1), fewer when a beam cut the tree
    const float* ret = level_ret.ret[d] + ri.base[d];
    const float* v = V + ri.leaf_item;
    for (int a0 = 0; a0 < A; ++a0) {
      float m = -INFINITY;
      for (long long j = a0 * blk + lane; j < (a0 + 1) * blk; j += 64)
        m = fmaxf(m, ret[j] + ri.gamma_d * v[j]);
      m = wave_max(m);
      if (lane == 0) q[a0] = m;
    }
  }
  __syncthreads();

  if (lane == 0) {
    if (ri.corr) {
      const float* Q0 = q0 + (long long)r * kMaxA;
      const float* r1 = level_ret.ret[1] + ri.base[1];          // depth-1 returns = rewards
      const float* v1 = V + (ri.d1_item >= 0 ? ri.d1_item : ri.leaf_item);
      int pi_o = 0;
      for (int a = 1; a < A; ++a)
        if (Q0[a] > Q0[pi_o]) pi_o = a;
      float d_o = 0.f, d_e = 0.f;
      for (int a = 0; a < A; ++a) {
        const float dl = fabsf(r1[a] + gamma * v1[a] - Q0[a]);
        if (a == pi_o) d_o = dl; else d_e += dl;
      }
      d_e /= (float)(A - 1);
      const float B = ri.pen_e * d_e - ri.pen_o * d_o;
      const float shift = corr_scale * ri.gamma_d * B;
      for (int a = 0; a < A; ++a)
        if (a != pi_o) q[a] = q[a] - shift;
    }
    int best = 0;
    for (int a = 1; a < A; ++a)
      if (q[a] > q[best]) best = a;
    out_action[r] = best;
    float* o = out_q + (long long)r * ri.q_stride;
    for (int a = 0; a < A; ++a) o[a] = q[a];
    for (int a = A; a < ri.q_stride; ++a) o[a] = -INFINITY;
  }
}

}  // namespace

void launch_backup_correct(int n_roots, const RootInfo* roots, const float* V, const float* q0,
                           const LevelRet& level_ret, float gamma, float corr_scale,
                           int* out_action, float* out_q, hipStream_t s) {
  if (n_roots <= 0) return;
  hipLaunchKernelGGL(backup_kernel, dim3(n_roots), dim3(64), 0, s, n_roots, roots, V, q0,
                     level_ret, gamma, corr_scale, out_action, out_q);
}

}  // namespace bcts
