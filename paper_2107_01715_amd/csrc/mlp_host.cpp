// Host levels of the forward-model search (see mlp_host.h).  For one child
// the output units of a layer advance together over k (weights stored
// [in][out], so the units' weights for one k are contiguous and the
// compiler vectorises across units); each unit's sum keeps its own order
// (bias, action column, k = 0..99).
#include "mlp_host.h"

#include <cmath>
#include <vector>

namespace bcts {
namespace {

constexpr int kS = 100;

std::vector<float> transpose(const float* w, int rows, int cols) {   // [rows][cols] -> [cols][rows]
  std::vector<float> t((size_t)rows * cols);
  for (int r = 0; r < rows; ++r)
    for (int c = 0; c < cols; ++c) t[(size_t)c * rows + r] = w[(size_t)r * cols + c];
  return t;
}

// y[o] = act(init[o] + sum_k WT[k][o] x[k]) for o < nout
template <bool RELU, int NOUT>
inline __attribute__((always_inline)) void dense(const float* WT, const float* init, const float* x, float* y) {
  float acc[NOUT];
  for (int o = 0; o < NOUT; ++o) acc[o] = init[o];
  for (int k = 0; k < kS; ++k) {
    const float xk = x[k];
    const float* w = WT + (size_t)k * NOUT;
    for (int o = 0; o < NOUT; ++o) acc[o] = std::fmaf(w[o], xk, acc[o]);
  }
  for (int o = 0; o < NOUT; ++o) y[o] = RELU ? std::fmax(acc[o], 0.f) : acc[o];
}

template <int A>
inline __attribute__((always_inline)) float head_max(const MlpHost& m, const float* s) {
  float acc[A];
  for (int a = 0; a < A; ++a) acc[a] = m.bq[a];
  for (int k = 0; k < kS; ++k)
    for (int a = 0; a < A; ++a) acc[a] = std::fmaf(m.wqT[(size_t)k * A + a], s[k], acc[a]);
  float v = -INFINITY;
  for (int a = 0; a < A; ++a) v = std::fmax(v, acc[a]);
  return v;
}

float head_max_any(const MlpHost& m, const float* s) {
  float v = -INFINITY;
  for (int a = 0; a < m.A; ++a) {
    float acc = m.bq[a];
    for (int k = 0; k < kS; ++k) acc = std::fmaf(m.wqT[(size_t)k * m.A + a], s[k], acc);
    v = std::fmax(v, acc);
  }
  return v;
}

inline __attribute__((always_inline)) void level_body(const MlpHost& m, long long n, const float* ps,
                                                      const float* pret, float gpow, float* os, float* oret,
                                                      float* ov) {
  const int A = m.A;
  alignas(64) float init[kS], h1[kS], h2[kS], h3[kS], out[kS + 1];
  for (long long c = 0; c < n; ++c) {
    const float* s = ps + (c / A) * kS;
    const float* wa = m.w1a.data() + (size_t)(c % A) * kS;
    for (int o = 0; o < kS; ++o) init[o] = m.b1[o] + wa[o];
    dense<true, kS>(m.w1sT.data(), init, s, h1);
    dense<true, kS>(m.w2T.data(), m.b2.data(), h1, h2);
    dense<true, kS>(m.w3T.data(), m.b3.data(), h2, h3);
    dense<false, kS + 1>(m.woT.data(), m.bo.data(), h3, out);          // 0..99 state, 100 reward
    const float r = std::fmaf(gpow, out[kS], pret ? pret[c / A] : 0.f);
    if (oret) oret[c] = r;
    if (os)
      for (int k = 0; k < kS; ++k) os[c * kS + k] = out[k];
    if (ov) ov[c] = A == 2 ? head_max<2>(m, out) : A == 10 ? head_max<10>(m, out) : head_max_any(m, out);
  }
}

__attribute__((target("avx2,fma"))) void level_fma(const MlpHost& m, long long n, const float* ps, const float* pret,
                                                   float gpow, float* os, float* oret, float* ov) {
  level_body(m, n, ps, pret, gpow, os, oret, ov);
}

void level_generic(const MlpHost& m, long long n, const float* ps, const float* pret, float gpow, float* os,
                   float* oret, float* ov) {
  level_body(m, n, ps, pret, gpow, os, oret, ov);
}

}  // namespace

void mlp_host_prepare(MlpHost& m, int A, const float* d) {
  m.A = A;
  size_t o = 0;
  auto take = [&](size_t k) { const float* p = d + o; o += k; return p; };
  const float* w1s = take(kS * kS);
  const float* w1a = take((size_t)A * kS);
  const float* b1 = take(kS);
  const float* w2 = take(kS * kS);
  const float* b2 = take(kS);
  const float* w3 = take(kS * kS);
  const float* b3 = take(kS);
  const float* wo = take((kS + 1) * kS);
  const float* bo = take(kS + 1);
  const float* wq = take((size_t)A * kS);
  const float* bq = take(A);
  m.w1sT = transpose(w1s, kS, kS);
  m.w1a.assign(w1a, w1a + (size_t)A * kS);
  m.b1.assign(b1, b1 + kS);
  m.w2T = transpose(w2, kS, kS);
  m.b2.assign(b2, b2 + kS);
  m.w3T = transpose(w3, kS, kS);
  m.b3.assign(b3, b3 + kS);
  m.woT = transpose(wo, kS + 1, kS);
  m.bo.assign(bo, bo + kS + 1);
  m.wqT = transpose(wq, A, kS);
  m.bq.assign(bq, bq + A);
}

// vector units with fused multiply-add where the CPU has them, else the
// generic build: fmaf rounds the same either way
void mlp_host_level(const MlpHost& m, long long n, const float* ps, const float* pret, float gpow, float* os,
                    float* oret, float* ov) {
  static const bool fma = __builtin_cpu_supports("avx2") && __builtin_cpu_supports("fma");
  if (fma) level_fma(m, n, ps, pret, gpow, os, oret, ov);
  else level_generic(m, n, ps, pret, gpow, os, oret, ov);
}

void mlp_host_search(const MlpHost& m, int n, const float* states, int d, float gamma, bool corr, float pen_e,
                     float pen_o, float scale, int32_t* act, float* q) {
  const int A = m.A;
  const bool corr_on = corr && d >= 1;
  const float gamma_d = (float)std::pow((double)gamma, d);
  std::vector<float> ps(states, states + (size_t)n * kS), pr, ns, nr, nv, ret1, v1, qd;
  long long cnt = n;
  for (int k = 1; k <= d; ++k) {
    cnt *= A;
    const bool last = k == d;
    ns.resize(last ? 0 : (size_t)cnt * kS);
    nr.resize((size_t)cnt);
    nv.resize(last || (k == 1 && corr_on) ? (size_t)cnt : 0);
    mlp_host_level(m, cnt, ps.data(), k == 1 ? nullptr : pr.data(), (float)std::pow((double)gamma, (double)(k - 1)),
                   last ? nullptr : ns.data(), nr.data(), nv.empty() ? nullptr : nv.data());
    if (k == 1) {
      ret1 = nr;
      if (corr_on) v1 = nv;
    }
    if (last) {
      const long long block = cnt / ((long long)n * A);     // leaves per (root, root action)
      qd.assign((size_t)n * A, -INFINITY);
      for (long long c = 0; c < cnt; ++c) {
        float& b = qd[(size_t)(c / block)];
        b = std::fmax(b, std::fmaf(gamma_d, nv[c], nr[c]));
      }
    }
    ps.swap(ns);
    pr.swap(nr);
  }
  std::vector<float> q0s(A), dels(A), outs(A);
  for (int r = 0; r < n; ++r) {
    const float* s = states + (size_t)r * kS;
    for (int a = 0; a < A; ++a) {
      float acc = m.bq[a];
      for (int k = 0; k < kS; ++k) acc = std::fmaf(m.wqT[(size_t)k * A + a], s[k], acc);
      q0s[a] = acc;
      if (corr_on) dels[a] = std::fmaf(gamma, v1[(size_t)r * A + a], ret1[(size_t)r * A + a]) - acc;
    }
    if (d == 0) {
      outs = q0s;
    } else {
      for (int a = 0; a < A; ++a) outs[a] = qd[(size_t)r * A + a];
      if (corr_on) {
        int pi = 0;
        for (int a = 1; a < A; ++a)
          if (q0s[a] > q0s[pi]) pi = a;
        const float dobs = std::fabs(dels[pi]);
        float se = 0.f;
        for (int a = 0; a < A; ++a)
          if (a != pi) se += std::fabs(dels[a]);
        const float de = se / (float)(A - 1);
        const float shift = scale * gamma_d * std::fmaf(pen_e, de, -(pen_o * dobs));
        for (int a = 0; a < A; ++a)
          if (a != pi) outs[a] -= shift;
      }
    }
    int best = 0;
    for (int a = 1; a < A; ++a)
      if (outs[best] < outs[a]) best = a;
    act[r] = best;
    for (int a = 0; a < A; ++a) q[(size_t)r * A + a] = outs[a];
  }
}

}  // namespace bcts
