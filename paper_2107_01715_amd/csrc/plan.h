// Host-side planning of a batched search: node counts per level, eval
// segments and sibling groups, Q-network chunks, the byte layout of the work
// arena, the correction coefficients, and a first-fit range allocator for
// pooled device memory.  Pure C++ (no HIP): built into libbcts and, on its
// own, into the host tests (with the address and undefined-behaviour
// sanitizers).
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <map>
#include <utility>
#include <vector>

#include "../../include/bcts.h"
#include "layout.h"

namespace bcts {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Penalty coefficients of one (A, d): B = pen_e d_e - pen_o d_o.
//   eq6_coeffs: Eq. 6, pen_e = sqrt(ln A) sqrt(d) - 1/sqrt 8,
//               pen_o = sqrt(ln A) sqrt(d - 1) - 1/sqrt 8;
//   gev_coeffs: Lemma 3.2's exact gap with sigma = |delta| / sqrt 2.
void eq6_coeffs(int A, int d, double* pe, double* po);
void gev_coeffs(int A, int d, double* pe, double* po);
// z with Phi(z) = 1 - p for an upper tail p <= 1/2.
double probit_upper_tail(double p);

// The FP32 discount of a level-(n+1) reward: the FP32 value nearest to the
// exact n-th power of g (ties to even), for finite g > 0 and 0 <= n <= 5.
// A pruned search ranks nodes by FP32 returns formed with these discounts.
float discount_f32(float g, int n);

// Workspace of the layer-by-layer Q-network path for `chunk` stacks, and of
// the fused path (x3 in fc1's tiles, h).
size_t qnet_workspace_bytes(long long chunk, int prec);
size_t fused_x3_bytes(long long chunk, int prec);
size_t fused_workspace_bytes(long long chunk, int prec);

struct Plan {
  int n = 0, maxd = 0;
  std::vector<RootInfo> roots;
  std::vector<Seg> segs;
  long long n_items = 0;
  long long lvl_count[kMaxD + 1] = {0};
  std::vector<int> lvl_root[kMaxD + 1];
  std::vector<long long> lvl_start[kMaxD + 1];
  int beam = 0;                        // beam of the cut levels (0: exhaustive)
  long long keep_count[kMaxD + 1] = {0};   // keep-list entries of level k over all roots
  long long chunk = 0;                 // max items of a chunk
  bool fused = false;                  // conv stack fused per sibling group
  std::vector<FusedGroup> groups;      // sibling groups in item order (main items, then the tail's)
  // A chunk: groups [g0, g1), items [i0, i1); its largest group and the sum
  // over its groups of (6 + 2 x group size), the conv1 stages of the group
  // kernel per 128 pixel rows
  struct Chunk { int g0, g1; long long i0, i1; int max_group; long long group_stages; };
  std::vector<Chunk> chunks;           // whole groups of the main items, ~chunk_items items each
  // The correction's own Q-network inputs (the root and depth-1 evaluations
  // of corrected roots) can run in FP32 whatever the leaf precision: they
  // then occupy the item range [tail_item0, n_items), evaluated by the FP32
  // layer kernels in tail_chunks (whole groups, ~tail_chunk_items items each).
  // tail_item0 == n_items when every item runs at the search precision.
  long long tail_item0 = 0;
  std::vector<Chunk> tail_chunks;
  long long tail_chunk = 0;            // max items of a tail chunk
  size_t o_groups = 0;
  // arena offsets
  size_t o_root_pos = 0, o_root_stack = 0, o_roots = 0, o_segs = 0, o_V = 0, o_q0 = 0,
         o_desc = 0, o_ws = 0, o_act = 0, o_q = 0, total = 0;
  size_t o_pos[kMaxD + 1] = {0}, o_frames[kMaxD + 1] = {0}, o_ret[kMaxD + 1] = {0},
         o_rew[kMaxD + 1] = {0}, o_lroot[kMaxD + 1] = {0}, o_lstart[kMaxD + 1] = {0},
         o_keep[kMaxD + 1] = {0};
  size_t table_bytes = 0;   // bytes of host tables uploaded (roots .. lstart)
  // Everything before o_desc belongs to this search; the item descriptors
  // and the Q-network workspace (o_desc .. total) are needed only while one
  // of its Q-network chunks runs, so work ordered on one stream can share
  // them (the serving engine does).
  size_t search_bytes() const { return o_desc; }
  size_t shared_bytes() const { return total - o_desc; }
};

// Chunks of whole groups p.groups[g0, g1), up to `target` items each (one
// group alone if it is larger), appended to `out`; *most is raised to the
// largest chunk's items.
void make_chunks(const Plan& p, int g0, int g1, long long target, std::vector<Plan::Chunk>& out, long long* most);


// Build the plan: node counts, eval segments and the arena layout.
// `q_stride` is the row stride of out_q; `host_io` reserves room for the
// roots and results of a host-buffer search.  `corr_fp32` moves the root and
// depth-1 evaluations of corrected roots to the FP32 tail (chunks of
// `tail_chunk_items`) when `prec` is not FP32.
void make_plan(Plan& p, int n, const int32_t* depth, const int32_t* A, float gamma,
               const bcts_correction& corr, int q_stride, long long chunk_items, int prec,
               bool host_io, bool fused = false, int beam = 0, bool corr_fp32 = false,
               long long tail_chunk_items = 8192);

// Device bytes one served request of (depth, A) takes at least (its levels,
// tables and eval values), without the shared workspace.
size_t request_bytes(int d, int A);

// First-fit allocator over the offsets [0, capacity) of a memory pool, in
// units of kAlign bytes; adjacent free ranges merge on release.
class RangePool {
 public:
  void reset(size_t capacity);
  // false (and nothing taken) when no free range holds `bytes`
  bool alloc(size_t bytes, size_t* off);
  void release(size_t off, size_t bytes);
  size_t capacity() const { return cap_; }
  size_t in_use() const { return used_; }
  size_t largest_free() const;
  size_t free_ranges() const { return free_.size(); }

 private:
  std::map<size_t, size_t> free_;   // offset -> length
  size_t cap_ = 0, used_ = 0;
};

}  // namespace bcts
