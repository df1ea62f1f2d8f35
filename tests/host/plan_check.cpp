// Host checks of the search planner and the pool allocator (plan.cpp), built
// with the address and undefined-behaviour sanitizers by
// tests/test_plan_host.py.  Exits non-zero at the first failed check.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <set>
#include <utility>
#include <vector>

#include "../../paper_2107_01715_amd/csrc/plan.h"

using namespace bcts;

static int g_checks = 0;
#define CHECK(cond, ...)                                               \
  do {                                                                 \
    ++g_checks;                                                        \
    if (!(cond)) {                                                     \
      std::fprintf(stderr, "FAILED %s:%d: %s: ", __FILE__, __LINE__, #cond); \
      std::fprintf(stderr, __VA_ARGS__);                               \
      std::fprintf(stderr, "\n");                                      \
      std::exit(1);                                                    \
    }                                                                  \
  } while (0)

struct Rng {   // xorshift64*: test inputs only
  uint64_t s;
  explicit Rng(uint64_t seed) : s(seed * 2654435761ULL + 1) {}
  uint64_t next() { s ^= s >> 12; s ^= s << 25; s ^= s >> 27; return s * 2685821657736338717ULL; }
  int uni(int lo, int hi) { return lo + (int)(next() % (uint64_t)(hi - lo + 1)); }
};

static long long ipow(long long a, int k) { long long r = 1; while (k--) r *= a; return r; }

// Nodes of one root at level k: A children of each kept node above; a beam
// keeps `beam` nodes per root action at cut levels 2..d-1.
static long long level_nodes(int A, int d, int beam, int k, bool* cut) {
  long long kept = 1, cnt = 0;
  for (int j = 1; j <= k; ++j) {
    cnt = kept * A;
    kept = cnt;
    *cut = false;
    if (beam > 0 && j >= 2 && j <= d - 1 && cnt / A > beam) { kept = (long long)A * beam; *cut = true; }
  }
  return cnt;
}

static void check_plan(const Plan& p, int n, const std::vector<int32_t>& dv, const std::vector<int32_t>& av,
                       const bcts_correction& corr, long long chunk_items, int prec, bool host_io, bool fused,
                       int beam, bool corr_fp32_req, long long tail_items) {
  const bool corr_fp32 = corr_fp32_req && prec != P_FP32;
  CHECK(p.n == n, "n");
  // ---- levels
  for (int k = 1; k <= kMaxD; ++k) {
    long long tot = 0, keep = 0;
    size_t li = 0;
    for (int r = 0; r < n; ++r) {
      const RootInfo& ri = p.roots[r];
      if (dv[r] < k) { CHECK(ri.lcnt[k] == 0 && ri.base[k] == -1, "root %d level %d", r, k); continue; }
      bool cut = false;
      const long long want = level_nodes(av[r], dv[r], beam, k, &cut);
      CHECK(ri.lcnt[k] == want, "root %d level %d: %lld nodes, want %lld", r, k, ri.lcnt[k], want);
      CHECK(ri.base[k] == tot, "root %d level %d base", r, k);
      CHECK(li < p.lvl_root[k].size() && p.lvl_root[k][li] == r && p.lvl_start[k][li] == tot, "level list");
      ++li;
      tot += want;
      if (cut) {
        CHECK(ri.kbase[k] == keep, "keep base");
        keep += (long long)av[r] * beam;
      } else {
        CHECK(ri.kbase[k] == -1, "uncut level has a keep list");
      }
    }
    CHECK(li == p.lvl_root[k].size(), "level %d lists %zu roots", k, p.lvl_root[k].size());
    CHECK(p.lvl_count[k] == tot && p.keep_count[k] == keep, "level %d totals", k);
  }
  // ---- eval segments: contiguous, one per (root, kind), at the expected places
  long long item = 0;
  bool in_tail = false;
  std::vector<int> seen(3 * n, 0);
  for (const Seg& sg : p.segs) {
    CHECK(sg.item0 == item, "segments are contiguous");
    CHECK(sg.root >= 0 && sg.root < n, "segment root");
    const RootInfo& ri = p.roots[sg.root];
    const int d = dv[sg.root], A = av[sg.root];
    const bool corrected = corr.enabled && d >= 1;
    long long cnt = 0;
    if (sg.kind == 0) {
      CHECK(d >= 1 && sg.level == d && ri.leaf_item == sg.item0, "leaf segment");
      cnt = ri.lcnt[d];
    } else if (sg.kind == 1) {
      CHECK(corrected && (d >= 2 || corr_fp32) && sg.level == 1 && ri.d1_item == sg.item0, "depth-1 segment");
      cnt = A;
    } else {
      CHECK(sg.kind == 2 && sg.level == 0 && ri.root_item == sg.item0 && (corrected || d == 0), "root segment");
      cnt = 1;
    }
    const bool tail_seg = corr_fp32 && corrected && sg.kind != 0;
    if (tail_seg) in_tail = true;
    CHECK(tail_seg == in_tail, "segment %lld: the FP32 correction evaluations come last", (long long)sg.item0);
    if (in_tail) CHECK(sg.item0 >= p.tail_item0, "tail segment before tail_item0");
    else CHECK(sg.item0 + cnt <= p.tail_item0, "main segment inside the tail");
    CHECK(++seen[3 * sg.root + sg.kind] == 1, "duplicate segment");
    item += cnt;
  }
  CHECK(item == p.n_items, "items %lld vs %lld", item, p.n_items);
  for (int r = 0; r < n; ++r) {
    const int d = dv[r];
    const bool corrected = corr.enabled && d >= 1;
    CHECK(seen[3 * r] == (d >= 1), "leaf segment of root %d", r);
    CHECK(seen[3 * r + 1] == (corrected && (d >= 2 || corr_fp32)), "depth-1 segment of root %d", r);
    CHECK(seen[3 * r + 2] == (corrected || d == 0), "root segment of root %d", r);
  }
  if (!corr_fp32) CHECK(p.tail_item0 == p.n_items && p.tail_chunks.empty(), "no tail expected");
  // ---- sibling groups: cover [0, n_items), each inside one segment, whole sibling sets
  long long g_item = 0;
  size_t si = 0;
  int main_groups = -1;
  for (const FusedGroup& g : p.groups) {
    if (g.item0 == p.tail_item0 && main_groups < 0) main_groups = (int)(&g - p.groups.data());
    CHECK(g.item0 == g_item && g.count >= 1, "groups are contiguous");
    while (si < p.segs.size() && p.segs[si].item0 + (p.segs[si].kind == 2 ? 1 : p.segs[si].kind == 1 ? av[p.segs[si].root] : p.roots[p.segs[si].root].lcnt[dv[p.segs[si].root]]) <= g.item0) ++si;
    CHECK(si < p.segs.size(), "group past the segments");
    const Seg& sg = p.segs[si];
    const int A = av[sg.root];
    const int want = sg.kind == 2 ? 1 : A;
    CHECK(g.count == want && (g.item0 - sg.item0) % want == 0, "group of %d at %lld (segment kind %d, A %d)", g.count,
          (long long)g.item0, sg.kind, A);
    g_item += g.count;
  }
  CHECK(g_item == p.n_items, "groups cover the items: %lld vs %lld", g_item, p.n_items);
  if (main_groups < 0) main_groups = (int)p.groups.size();
  // ---- chunks, then tail chunks: whole groups, bounded size
  long long maxg = 1;
  for (const auto& g : p.groups) maxg = std::max<long long>(maxg, g.count);
  auto check_chunks = [&](const std::vector<Plan::Chunk>& chunks, int g_from, int g_to, long long want,
                          long long most, const char* what) {
    int gi = g_from;
    for (const auto& ch : chunks) {
      CHECK(ch.g0 == gi && ch.g1 > ch.g0 && ch.g1 <= g_to, "%s groups", what);
      CHECK(ch.i0 == p.groups[ch.g0].item0, "%s start", what);
      long long items = 0, stages = 0;
      int most_g = 0;
      for (int g = ch.g0; g < ch.g1; ++g) {
        items += p.groups[g].count;
        stages += 6 + 2LL * p.groups[g].count;
        most_g = std::max(most_g, p.groups[g].count);
      }
      CHECK(ch.max_group == most_g && ch.group_stages == stages, "%s group statistics", what);
      CHECK(ch.i1 - ch.i0 == items && items <= std::max(std::max(1LL, want), maxg) && items <= most,
            "%s of %lld items", what, items);
      gi = ch.g1;
    }
    CHECK(gi == g_to, "%s cover their groups", what);
  };
  check_chunks(p.chunks, 0, main_groups, chunk_items, p.chunk, "chunk");
  check_chunks(p.tail_chunks, main_groups, (int)p.groups.size(), tail_items, p.tail_chunk, "tail chunk");
  if (!p.tail_chunks.empty()) CHECK(p.tail_chunks.front().i0 == p.tail_item0, "the tail chunks start at tail_item0");
  // ---- arena layout: aligned, disjoint, inside total, large enough
  std::vector<std::pair<size_t, size_t>> reg;   // (offset, bytes needed)
  auto add = [&](size_t off, size_t bytes) { if (bytes) reg.emplace_back(off, bytes); };
  add(p.o_roots, sizeof(RootInfo) * n);
  add(p.o_segs, sizeof(Seg) * p.segs.size());
  add(p.o_groups, sizeof(FusedGroup) * p.groups.size());
  for (int k = 1; k <= p.maxd; ++k) {
    add(p.o_lroot[k], sizeof(int) * p.lvl_root[k].size());
    add(p.o_lstart[k], sizeof(long long) * p.lvl_start[k].size());
  }
  size_t tables_end = 0;
  for (auto& r : reg) tables_end = std::max(tables_end, r.first + r.second);
  CHECK(tables_end <= p.table_bytes, "tables end %zu past table_bytes %zu", tables_end, p.table_bytes);
  if (host_io) {
    add(p.o_root_pos, sizeof(int32_t) * n * kSprites * 2);
    add(p.o_root_stack, (size_t)n * 4 * kFrameBytes);
    add(p.o_act, sizeof(int32_t) * n);
    add(p.o_q, sizeof(float) * (size_t)n * kMaxA);
  }
  for (int k = 1; k <= p.maxd; ++k) {
    add(p.o_pos[k], (size_t)p.lvl_count[k] * 16);
    add(p.o_frames[k], (size_t)p.lvl_count[k] * kFrameBytes);
    add(p.o_ret[k], (size_t)p.lvl_count[k] * 4);
    add(p.o_rew[k], (size_t)p.lvl_count[k]);
    if (p.keep_count[k]) add(p.o_keep[k], sizeof(int) * (size_t)p.keep_count[k]);
  }
  add(p.o_V, sizeof(float) * p.n_items);
  add(p.o_q0, sizeof(float) * (size_t)n * kMaxA);
  const size_t search_end = [&] { size_t e = 0; for (auto& r : reg) e = std::max(e, r.first + r.second); return e; }();
  CHECK(search_end <= p.search_bytes(), "search regions end at %zu, search_bytes %zu", search_end, p.search_bytes());
  add(p.o_desc, sizeof(ItemDesc) * std::max(p.chunk, p.tail_chunk));
  size_t ws = 0;
  if (!p.chunks.empty()) ws = p.fused ? fused_workspace_bytes(p.chunk, prec) : qnet_workspace_bytes(p.chunk, prec);
  if (p.tail_chunk > 0) ws = std::max(ws, qnet_workspace_bytes(p.tail_chunk, P_FP32));
  add(p.o_ws, ws);
  std::sort(reg.begin(), reg.end());
  for (size_t i = 0; i < reg.size(); ++i) {
    CHECK(reg[i].first % kAlign == 0, "region at %zu not aligned", reg[i].first);
    CHECK(reg[i].first + reg[i].second <= p.total, "region past total");
    if (i) CHECK(reg[i - 1].first + reg[i - 1].second <= reg[i].first, "regions overlap at %zu", reg[i].first);
  }
  CHECK(p.o_desc >= p.search_bytes() && p.o_desc <= p.total, "shared part last");
  (void)fused;
}

static void plans(uint64_t seed, int trials) {
  Rng g(seed);
  for (int t = 0; t < trials; ++t) {
    const int n = g.uni(1, 40);
    std::vector<int32_t> dv(n), av(n);
    long long leaves = 0;
    for (int r = 0; r < n; ++r) {
      do {
        av[r] = g.uni(1, kMaxA);
        dv[r] = g.uni(0, kMaxD);
      } while (ipow(av[r], dv[r]) > 20000 || (av[r] < 2 && dv[r] > 0 && g.uni(0, 1)));
      leaves += ipow(av[r], dv[r]);
    }
    bcts_correction corr{g.uni(0, 1), 1.0f, g.uni(0, 1)};
    for (int r = 0; r < n; ++r)
      if (corr.enabled && dv[r] >= 1 && av[r] < 2) av[r] = 2;
    const int prec = g.uni(0, 2);
    const bool fused = g.uni(0, 1), host_io = g.uni(0, 1), cf = g.uni(0, 1);
    const int beam = g.uni(0, 3) == 0 ? g.uni(1, 40) : 0;
    const long long chunk = g.uni(0, 3) == 0 ? g.uni(1, 64) : g.uni(1, 300000);
    const long long tail = g.uni(1, 9000);
    Plan p;
    make_plan(p, n, dv.data(), av.data(), 0.99f, corr, kMaxA, chunk, prec, host_io, fused, beam, cf, tail);
    check_plan(p, n, dv, av, corr, chunk, prec, host_io, fused, beam, cf, tail);
    // a cohort of single requests never needs more than the sum of their own request_bytes
    size_t sum = 0;
    for (int r = 0; r < n; ++r) sum += request_bytes(dv[r], av[r]);
    Plan q;
    make_plan(q, n, dv.data(), av.data(), 0.99f, corr, kMaxA, chunk, prec, true, fused, 0, cf, tail);
    CHECK(q.search_bytes() <= sum, "cohort of %d: %zu bytes > %zu summed request_bytes", n, q.search_bytes(), sum);
    (void)leaves;
  }
}

static void single_requests() {
  for (int A = 1; A <= kMaxA; ++A)
    for (int d = 0; d <= kMaxD; ++d) {
      if (ipow(A, d) > 2000000) continue;
      for (int cf = 0; cf < 2; ++cf)
        for (int prec = 0; prec < 3; ++prec) {
          bcts_correction corr{A >= 2 ? 1 : 0, 1.0f, 0};
          int32_t dd = d, aa = A;
          Plan p;
          make_plan(p, 1, &dd, &aa, 0.99f, corr, kMaxA, 16384, prec, true, prec != P_FP32, 0, cf != 0, 2048);
          CHECK(p.search_bytes() <= request_bytes(d, A), "request (d %d, A %d) needs %zu > request_bytes %zu", d, A,
                p.search_bytes(), request_bytes(d, A));
        }
    }
}

static void pool(uint64_t seed) {
  Rng g(seed);
  for (int t = 0; t < 50; ++t) {
    const size_t cap = (size_t)g.uni(1, 4000) * kAlign + (size_t)g.uni(0, 255);
    RangePool pool;
    pool.reset(cap);
    const size_t units = cap / kAlign;
    std::vector<int> owner(units, -1);
    std::vector<std::pair<size_t, size_t>> live;   // (off, bytes)
    for (int step = 0; step < 2000; ++step) {
      if (live.empty() || g.uni(0, 2) != 0) {
        const size_t bytes = (size_t)g.uni(1, (int)std::min<size_t>(cap, 300 * kAlign));
        size_t off = 0;
        // brute force: is there a free run of the needed units?
        const size_t need = align_up(bytes) / kAlign;
        size_t run = 0, first_fit = SIZE_MAX;
        for (size_t u = 0; u < units; ++u) {
          run = owner[u] < 0 ? run + 1 : 0;
          if (run == need) { first_fit = u + 1 - need; break; }
        }
        const bool ok = pool.alloc(bytes, &off);
        CHECK(ok == (first_fit != SIZE_MAX), "alloc of %zu bytes: %d, first fit %zu", bytes, ok, first_fit);
        if (!ok) continue;
        CHECK(off == first_fit * kAlign, "first fit at %zu, got %zu", first_fit * kAlign, off);
        for (size_t u = off / kAlign; u < off / kAlign + need; ++u) {
          CHECK(u < units && owner[u] < 0, "overlap at unit %zu", u);
          owner[u] = step;
        }
        live.emplace_back(off, bytes);
      } else {
        const size_t i = (size_t)g.uni(0, (int)live.size() - 1);
        const auto r = live[i];
        live.erase(live.begin() + (long)i);
        pool.release(r.first, r.second);
        for (size_t u = r.first / kAlign; u < (r.first + align_up(r.second)) / kAlign; ++u) owner[u] = -1;
      }
      size_t used = 0;
      for (int o : owner) used += o >= 0;
      CHECK(pool.in_use() == used * kAlign, "in_use %zu vs %zu", pool.in_use(), used * kAlign);
    }
    for (const auto& r : live) pool.release(r.first, r.second);
    CHECK(pool.in_use() == 0 && pool.free_ranges() == 1 && pool.largest_free() == units * kAlign,
          "pool does not coalesce back to one range");
  }
}

static void coefficients() {
  // Eq. 6 worked from the formula: B(d_e, d_o, A, d) = pen_e d_e - pen_o d_o
  struct Case { double de, dob; int A, d; double B; } cs[] = {
      {1.0, 0.5, 4, 2, 0.8996275157610213}, {1.0, 0.5, 18, 3, 1.565740213901015},
      {2.0, 1.0, 6, 1, 2.3235790074984273}, {1.0, 1.0, 4, 1, 1.1774100225154747}};
  for (const auto& c : cs) {
    double pe, po;
    eq6_coeffs(c.A, c.d, &pe, &po);
    const double B = pe * c.de - po * c.dob;
    CHECK(std::fabs(B - c.B) < 1e-12, "Eq. 6 B(%g, %g, %d, %d) = %.16g, want %.16g", c.de, c.dob, c.A, c.d, B, c.B);
  }
  // probit: known quantiles of the standard normal
  CHECK(std::fabs(probit_upper_tail(0.025) - 1.959963984540054) < 1e-9, "z(0.975)");
  CHECK(std::fabs(probit_upper_tail(0.5)) < 1e-9, "z(0.5)");
  CHECK(std::fabs(probit_upper_tail(1e-6) - 4.753424308822899) < 1e-8, "z(1 - 1e-6)");
  for (int A = 2; A <= kMaxA; ++A)
    for (int d = 1; d <= kMaxD; ++d) {
      double pe, po;
      gev_coeffs(A, d, &pe, &po);
      CHECK(std::isfinite(pe) && std::isfinite(po) && pe >= 0 && po >= 0, "GEV coefficients A %d d %d", A, d);
      // one leaf per root action (d = 1) has no bias (B_o = 0), and the max of
      // a single other leaf (A = 2, d = 1) none either (B_e = 0)
      if (d == 1) CHECK(po == 0.0, "B_o at depth 1");
      CHECK((pe == 0.0) == (A == 2 && d == 1), "B_e = 0 exactly at A = 2, d = 1 (A %d d %d)", A, d);
    }
}

static void discounts() {
  // exact cases: powers of 1/2 and 1
  for (int n = 0; n <= 5; ++n) {
    CHECK(discount_f32(0.5f, n) == std::ldexp(1.0f, -n), "0.5^%d", n);
    CHECK(discount_f32(1.0f, n) == 1.0f, "1^%d", n);
  }
  // g^2 has 48 significant bits, exact in double: one rounding to float
  Rng rg(7);
  for (int t = 0; t < 20000; ++t) {
    const float g = (float)((double)(rg.next() >> 11) * 0x1.0p-53);
    if (!(g > 0.f)) continue;
    CHECK(discount_f32(g, 1) == g, "g^1");
    CHECK(discount_f32(g, 2) == (float)((double)g * (double)g), "g^2 for g = %a", g);
    // higher powers: the nearest float to the long-double power (64-bit
    // mantissa), skipping values too close to a rounding boundary to decide
    for (int n = 3; n <= 5; ++n) {
      long double pw = 1.0L;
      for (int i = 0; i < n; ++i) pw *= (long double)g;
      const float f = (float)pw;
      const long double up = (long double)std::nextafter(f, 1.0f), dn = (long double)std::nextafter(f, 0.0f);
      const long double lo = ((long double)f + dn) / 2, hi = ((long double)f + up) / 2;
      if (std::fabs((double)((pw - lo) / pw)) < 1e-15 || std::fabs((double)((hi - pw) / pw)) < 1e-15) continue;
      CHECK(discount_f32(g, n) == f, "g^%d for g = %a", n, g);
    }
  }
  CHECK(discount_f32(0.99f, 2) == (float)(0.99f * (double)0.99f), "0.99^2");
}

int main() {
  discounts();
  coefficients();
  single_requests();
  plans(1, 400);
  plans(2, 400);
  pool(3);
  std::printf("plan_check: %d checks passed\n", g_checks);
  return 0;
}
