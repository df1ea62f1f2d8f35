// Host (CPU) levels of the forward-model search: the CPU side of the
// paper's CPU-to-GPU cross-over (Sec. 4.1 runtime study: the host is the
// faster device for the first levels of a small tree, so the search starts
// there and moves to the GPU at a cross-over depth).  Pure C++, no HIP.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <vector>

namespace bcts {

// The forward model for the host: weight matrices transposed to [in][out]
// (so one input's weights to all output units are contiguous), l1's action
// columns as rows w1a[a][o] = l1.w[o][100 + a], biases as they are.
struct MlpHost {
  int A = 0;
  std::vector<float> w1sT, w1a, b1, w2T, b2, w3T, b3, woT, bo, wqT, bq;
};

// From the device-order blob: w1s [100][100], w1a [A][100], b1, w2 [100][100],
// b2, w3, b3, wo [101][100], bo, wq [A][100], bq ([out][in] matrices).
void mlp_host_prepare(MlpHost& m, int A, const float* dev_blob);

// One level: children c in [0, n) of parents c / A (action c % A).
//   ps    parent states [n / A][100]; pret their returns (null at level 1)
//   gpow  gamma^(k-1)
//   os    child states [n][100], oret child returns [n], ov max_a Q(child, a)
//         [n] (null: not needed)
// Every output is the same FP32 arithmetic as the device's level kernel, in
// the same order (each sum starts from its bias -- plus the action column
// in layer 1 -- and adds k = 0..99 with fused multiply-adds; reward into the
// return by one fused multiply-add), so the two devices give the same bits.
void mlp_host_level(const MlpHost& m, long long n, const float* ps, const float* pret, float gpow, float* os,
                    float* oret, float* ov);

// The whole search of n roots on the host: the CPU BFS of the Sec. 4.1
// runtime study.  Levels 1..d as mlp_host_level; each leaf's value
// r + gamma^d max_a Q(leaf, a); their maximum per (root, root action) block
// (Eq. 1); the roots' Q0 = Wq s + bq; with `corr` the shift of Eq. 3 by
// scale gamma^d B, B = pen_e d_e - pen_o d_o (Prop. 3.6: d_o = |delta of
// pi_o|, d_e the mean |delta| of the other actions, delta_a = r_a +
// gamma max Q(s_1^a) - Q0_a).  act[n] gets the argmax (lowest index), q[n][A]
// the root vectors.  Every value is the device kernels' FP32 arithmetic in
// their order, so the results are the GPU search's bits.
void mlp_host_search(const MlpHost& m, int n, const float* states, int d, float gamma, bool corr, float pen_e,
                     float pen_o, float scale, int32_t* act, float* q);

}  // namespace bcts
