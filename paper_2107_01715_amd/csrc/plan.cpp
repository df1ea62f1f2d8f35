// Host-side planning of a batched search (see plan.h).
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace bcts {

// Eq. 6 penalty coefficients: B = pen_e d_e - pen_o d_o
void eq6_coeffs(int A, int d, double* pe, double* po) {
  const double s = std::sqrt(std::log((double)A)), r8 = 1.0 / std::sqrt(8.0);
  *pe = s * std::sqrt((double)d) - r8;
  *po = s * std::sqrt((double)(d - 1)) - r8;
}

// z with Phi(z) = 1 - p (upper tail p <= 1/2), by bisection on
// 0.5 erfc(z / sqrt 2) = p over [0, 40]; the tail function is monotone and
// erfc keeps full relative accuracy far into the tail.
double probit_upper_tail(double p) {
  double lo = 0.0, hi = 40.0;
  for (int it = 0; it < 200 && hi - lo > 1e-15 * hi; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (0.5 * std::erfc(mid / std::sqrt(2.0)) > p) lo = mid; else hi = mid;
  }
  return 0.5 * (lo + hi);
}

// Lemma 3.2: bias of the max of n Gaussians per unit sigma
double gev_bias(double n) {
  if (n <= 1.0) return 0.0;
  const double g = 0.57721566490153286060651209;
  return g * probit_upper_tail(1.0 / (M_E * n)) + (1.0 - g) * probit_upper_tail(1.0 / n);
}

// exact gap with sigma = |delta| / sqrt 2: B = pen_e d_e - pen_o d_o
void gev_coeffs(int A, int d, double* pe, double* po) {
  const double no = std::pow((double)A, d - 1), ne = std::pow((double)A, d) - no;
  *pe = gev_bias(ne) / std::sqrt(2.0);
  *po = gev_bias(no) / std::sqrt(2.0);
}

float discount_f32(float g, int n) {
  // g = m 2^e with a 24-bit integer m; m^n has at most 120 bits, so the power
  // is exact in 128-bit integers; keep its top 24 bits, round to nearest even
  if (n == 0) return 1.0f;
  int e = 0;
  const float fr = std::frexp(g, &e);                      // g = fr 2^e, fr in [0.5, 1)
  const unsigned long long m = (unsigned long long)std::ldexp((double)fr, 24);   // exact: 24 bits
  e -= 24;
  unsigned __int128 p = 1;
  for (int i = 0; i < n; ++i) p *= m;
  int bits = 0;
  for (unsigned __int128 t = p; t; t >>= 1) ++bits;
  int shift = bits - 24, ex = e * n;
  if (shift > 0) {
    const unsigned __int128 half = (unsigned __int128)1 << (shift - 1), rem = p & (((unsigned __int128)1 << shift) - 1);
    unsigned __int128 q = p >> shift;
    if (rem > half || (rem == half && (q & 1))) ++q;
    p = q;
    ex += shift;
  }
  return (float)std::ldexp((double)(unsigned long long)p, ex);   // p < 2^25 and the exponent in range: exact
}

size_t qnet_workspace_bytes(long long chunk, int prec) {
  const size_t el = prec == P_FP32 ? 4 : prec == P_BF16 ? 2 : 1;
  const size_t part = prec == P_FP32 ? (size_t)chunk * kFc1Split * 512 * 4 : 0;   // fc1's K slices
  return (size_t)chunk * (12800 + 5184 + 3136 + 512) * el + part + 256;
}

// fused path: x3 [chunk rounded up to fc1's 256-row tiles][3136] and
// h [chunk][512] in the operand type
size_t fused_x3_bytes(long long chunk, int prec) {
  const size_t el = prec == P_BF16 ? 2 : 1;
  return align_up((size_t)(fc1_padded_rows(chunk) / kFc1Rows) * (size_t)fc1_tile_bytes((int)el));
}
size_t fused_workspace_bytes(long long chunk, int prec) {
  const size_t el = prec == P_BF16 ? 2 : 1;
  return fused_x3_bytes(chunk, prec) + (size_t)chunk * 512 * el + 256;
}

void make_chunks(const Plan& p, int g, int g_end, long long target, std::vector<Plan::Chunk>& out, long long* most) {
  target = std::max(1LL, target);
  while (g < g_end) {
    Plan::Chunk ch;
    ch.g0 = g;
    ch.i0 = p.groups[g].item0;
    ch.max_group = 0;
    ch.group_stages = 0;
    long long items = 0;
    while (g < g_end && (items == 0 || items + p.groups[g].count <= target)) {
      items += p.groups[g].count;
      ch.max_group = std::max(ch.max_group, p.groups[g].count);
      ch.group_stages += 6 + 2LL * p.groups[g].count;
      ++g;
    }
    ch.g1 = g;
    ch.i1 = ch.i0 + items;
    *most = std::max(*most, items);
    out.push_back(ch);
  }
}

void make_plan(Plan& p, int n, const int32_t* depth, const int32_t* A, float gamma,
               const bcts_correction& corr, int q_stride, long long chunk_items, int prec,
               bool host_io, bool fused, int beam, bool corr_fp32, long long tail_chunk_items) {
  p = Plan();
  corr_fp32 = corr_fp32 && prec != P_FP32;
  p.beam = beam;
  p.fused = fused && prec != P_FP32;
  p.n = n;
  p.roots.resize(n);
  for (int r = 0; r < n; ++r) p.maxd = std::max(p.maxd, (int)depth[r]);
  // level node bases (root-major inside each level)
  for (int r = 0; r < n; ++r) {
    RootInfo& ri = p.roots[r];
    std::memset(&ri, 0, sizeof ri);
    ri.A = A[r];
    ri.d = depth[r];
    ri.gamma_d = (float)std::pow((double)gamma, (double)ri.d);
    ri.corr = (corr.enabled && ri.d >= 1) ? 1 : 0;
    ri.q_stride = q_stride;
    // nodes per level: A children of each kept node of the level above; a
    // beam cuts levels 2..d-1 to `beam` nodes per root action where a root
    // action's block is larger
    ri.lcnt[0] = 1;
    ri.kbase[0] = -1;
    long long kept = 1;
    for (int k = 1; k <= kMaxD; ++k) {
      ri.kbase[k] = -1;
      if (k <= ri.d) {
        const long long cnt = kept * ri.A;
        ri.lcnt[k] = cnt;
        ri.base[k] = p.lvl_count[k];
        p.lvl_root[k].push_back(r);
        p.lvl_start[k].push_back(p.lvl_count[k]);
        p.lvl_count[k] += cnt;
        kept = cnt;
        if (beam > 0 && k >= 2 && k <= ri.d - 1 && cnt / ri.A > beam) {
          ri.kbase[k] = p.keep_count[k];
          p.keep_count[k] += (long long)ri.A * beam;
          kept = (long long)ri.A * beam;
        }
      } else {
        ri.base[k] = -1;
        ri.lcnt[k] = 0;
      }
    }
    ri.leaf_blk = ri.d >= 1 ? ri.lcnt[ri.d] / ri.A : 0;
    if (ri.corr) {
      double pe, po;
      if (corr.mode == BCTS_CORR_EXACT_GEV) gev_coeffs(ri.A, ri.d, &pe, &po);
      else eq6_coeffs(ri.A, ri.d, &pe, &po);
      ri.pen_e = (float)pe;
      ri.pen_o = (float)po;
    }
  }
  // eval segments: per root, leaves, depth-1 nodes, root (with corr_fp32 the
  // depth-1 and root segments of corrected roots follow all the others)
  long long item = 0;
  // (at depth 1 the depth-1 nodes are the leaves: their values serve the
  // Bellman errors unless those are taken in FP32, which needs A FP32 evals)
  auto add_corr_segs = [&](int r) {
    RootInfo& ri = p.roots[r];
    if (ri.corr && (ri.d >= 2 || corr_fp32)) {
      p.segs.push_back(Seg{item, r, 1, ri.A, 1});
      ri.d1_item = item;
      item += ri.A;
    }
    if (ri.corr) {
      p.segs.push_back(Seg{item, r, 0, ri.A, 2});
      ri.root_item = item;
      item += 1;
    }
  };
  for (int r = 0; r < n; ++r) {
    RootInfo& ri = p.roots[r];
    ri.leaf_item = ri.d1_item = ri.root_item = -1;
    if (ri.d >= 1) {
      const long long cnt = ri.lcnt[ri.d];
      p.segs.push_back(Seg{item, r, ri.d, ri.A, 0});
      ri.leaf_item = item;
      item += cnt;
    }
    if (ri.d == 0) {                   // no search: the root eval is the result
      p.segs.push_back(Seg{item, r, 0, ri.A, 2});
      ri.root_item = item;
      item += 1;
    } else if (!corr_fp32) {
      add_corr_segs(r);
    }
  }
  const size_t main_segs = p.segs.size();
  p.tail_item0 = item;
  if (corr_fp32)
    for (int r = 0; r < n; ++r)
      if (p.roots[r].d >= 1) add_corr_segs(r);
  p.n_items = item;
  // sibling groups: the A children of each level-(d-1) node, the A depth-1
  // nodes of a root, a root alone; the main items' groups, then the tail's
  int main_groups = 0;
  for (size_t si = 0; si < p.segs.size(); ++si) {
    if (si == main_segs) main_groups = (int)p.groups.size();
    const Seg& sg = p.segs[si];
    const RootInfo& ri = p.roots[sg.root];
    const long long cnt = sg.kind == 2 ? 1 : (sg.kind == 1 ? ri.A : ri.lcnt[ri.d]);
    const int gsz = sg.kind == 2 ? 1 : ri.A;
    for (long long j = 0; j < cnt; j += gsz) p.groups.push_back(FusedGroup{sg.item0 + j, gsz, 0});
  }
  if (main_segs == p.segs.size()) main_groups = (int)p.groups.size();
  p.chunk = 1;
  make_chunks(p, 0, main_groups, chunk_items, p.chunks, &p.chunk);
  make_chunks(p, main_groups, (int)p.groups.size(), tail_chunk_items, p.tail_chunks, &p.tail_chunk);

  // arena layout
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o += align_up(bytes); return at; };
  p.o_roots = take(sizeof(RootInfo) * n);
  p.o_segs = take(sizeof(Seg) * p.segs.size());
  p.o_groups = take(sizeof(FusedGroup) * p.groups.size());
  for (int k = 1; k <= p.maxd; ++k) {
    p.o_lroot[k] = take(sizeof(int) * p.lvl_root[k].size());
    p.o_lstart[k] = take(sizeof(long long) * p.lvl_start[k].size());
  }
  p.table_bytes = o;
  if (host_io) {
    p.o_root_pos = take(sizeof(int32_t) * n * kSprites * 2);
    p.o_root_stack = take((size_t)n * 4 * kFrameBytes);
    p.o_act = take(sizeof(int32_t) * n);
    p.o_q = take(sizeof(float) * (size_t)n * q_stride);
  }
  for (int k = 1; k <= p.maxd; ++k) {
    p.o_pos[k] = take((size_t)p.lvl_count[k] * 16);
    p.o_frames[k] = take((size_t)p.lvl_count[k] * kFrameBytes);
    p.o_ret[k] = take((size_t)p.lvl_count[k] * sizeof(float));
    p.o_rew[k] = take((size_t)p.lvl_count[k]);
    if (p.keep_count[k] > 0) p.o_keep[k] = take(sizeof(int) * (size_t)p.keep_count[k]);
  }
  p.o_V = take(sizeof(float) * p.n_items);
  p.o_q0 = take(sizeof(float) * (size_t)n * kMaxA);
  p.o_desc = take(sizeof(ItemDesc) * std::max(p.chunk, p.tail_chunk));
  {
    size_t ws = p.chunks.empty() ? 0
                : (p.fused ? fused_workspace_bytes(p.chunk, prec) : qnet_workspace_bytes(p.chunk, prec));
    if (p.tail_chunk > 0) ws = std::max(ws, qnet_workspace_bytes(p.tail_chunk, P_FP32));
    p.o_ws = take(ws);
  }
  p.total = o;
}

size_t request_bytes(int d, int A) {
  // the plan of the request alone, with every evaluation the correction can
  // add and room for its host-side inputs, in the larger of the two layouts
  // (correction evaluations in the FP32 tail or among the sibling groups)
  const int32_t dd = d, aa = A;
  const bcts_correction corr{A >= 2 ? 1 : 0, 1.0f, 0};
  size_t b = 0;
  for (int prec : {P_FP32, P_BF16}) {     // FP32: its correction evaluations join the sibling groups
    Plan p;
    make_plan(p, 1, &dd, &aa, 0.99f, corr, kMaxA, 1, prec, true, prec != P_FP32, 0, true, 1);
    b = std::max(b, p.search_bytes());
  }
  return b;
}

void RangePool::reset(size_t capacity) {
  cap_ = capacity / kAlign * kAlign;
  used_ = 0;
  free_.clear();
  if (cap_ > 0) free_[0] = cap_;
}

bool RangePool::alloc(size_t bytes, size_t* off) {
  const size_t need = align_up(std::max<size_t>(bytes, 1));
  for (auto it = free_.begin(); it != free_.end(); ++it) {
    if (it->second < need) continue;
    const size_t at = it->first, len = it->second;
    free_.erase(it);
    if (len > need) free_[at + need] = len - need;
    used_ += need;
    *off = at;
    return true;
  }
  return false;
}

void RangePool::release(size_t off, size_t bytes) {
  const size_t len = align_up(std::max<size_t>(bytes, 1));
  used_ -= len;
  auto it = free_.emplace(off, len).first;
  auto nx = std::next(it);
  if (nx != free_.end() && it->first + it->second == nx->first) {
    it->second += nx->second;
    free_.erase(nx);
  }
  if (it != free_.begin()) {
    auto pv = std::prev(it);
    if (pv->first + pv->second == it->first) {
      pv->second += it->second;
      free_.erase(it);
    }
  }
}

size_t RangePool::largest_free() const {
  size_t m = 0;
  for (const auto& f : free_) m = std::max(m, f.second);
  return m;
}

}  // namespace bcts
