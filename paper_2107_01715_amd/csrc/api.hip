// C ABI of libbcts: context, argument validation, the search planner and the
// launch sequence of a batched Batch-BFS search (Alg. 1 for many roots at
// once, followed by the correction of Eq. 3).
//
// A search over n roots runs, on one stream:
//   1. expand level k = 1..max depth      (one launch per level, all roots)
//   2. Q-network over every eval item     (chunks of items, 5 launches each)
//   3. backup + correction + argmax       (one launch, one wavefront per root)
// The plan (node counts A^k per root, eval segments, arena offsets) is made on
// the host; its tables are copied to the device once per search.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <list>
#include <mutex>
#include <string>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "../../include/bcts.h"
#include "bcts_internal.h"
#include "qnet_groups.h"
#include "plan.h"
#include "mlp_host.h"

using namespace bcts;

constexpr int kMlpMaxD = 16;            // deepest forward-model search

namespace {


double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct bcts_ctx {
  int device = 0;
  size_t budget = 0;
  hipStream_t stream = nullptr;
  std::string err;
  bool error_state = false;
  bool env_set = false, qnet_set = false;
  EnvTables env{};
  int prec = P_FP32;
  long long chunk_items = 65536;       // layer-by-layer path (FP32): ~6.6 GB of FP32 workspace
  long long fused_chunk_items = 262144; // fused path (BF16 / FP8)
  int fused_T = 3;                      // items per LDS round of the fused conv kernel
  bool fp8_k128 = true;                 // FP8 conv2 / conv3 on the K = 128 matrix instruction
  int conv1_groups = 1;                 // layer path, conv1 by sibling groups: 0 never, 1 when faster, 2 always
  bool fc2_folded = true;               // fused path: fc2 in fc1's epilogue (else fc1 writes h)
  bool fused = true;
  bool corr_fp32 = true;                // root / depth-1 evals of corrected roots in FP32
  int beam = 0;                         // pruned search: nodes kept per root action at cut levels (0: none)
  // weights
  void* wmem = nullptr;
  size_t wbytes = 0;
  QnetDev q{};
  float wabs[5] = {0};
  bool fp8_calibrated = false;
  // arena
  char* arena = nullptr;
  size_t arena_bytes = 0;
  // pinned staging for host I/O
  char* pinned = nullptr;
  size_t pinned_bytes = 0;
  // two pinned staging buffers for the plan tables, used in turn: a search
  // fills one while the copy of the previous search's tables from the other
  // may still be queued; tpin_ev[b] marks the end of buffer b's last copy
  char* tpin[2] = {nullptr, nullptr};
  size_t tpin_bytes[2] = {0, 0};
  hipEvent_t tpin_ev[2] = {nullptr, nullptr};
  bool tpin_busy[2] = {false, false};
  int tpin_next = 0;
  // cross-stream order of the arena: the stream of the last search enqueued
  // on it and an event recorded after that search's work (see order_arena)
  hipEvent_t arena_ev = nullptr;
  hipStream_t arena_stream = nullptr;
  bool arena_pending = false;
  // the no-allocation entry point: the device's static scratch (its device
  // address, looked up at bcts_create) and a host staging buffer for its
  // tables, reused once its last copy has finished (na_copy_ev); na_ev marks
  // the end of the last search enqueued on the scratch, on stream na_stream
  char* scratch = nullptr;
  std::string scratch_err;
  std::vector<char> na_tables;
  hipEvent_t na_ev = nullptr, na_copy_ev = nullptr;
  hipStream_t na_stream = nullptr;
  bool na_pending = false, na_copy_pending = false;
  // timing: events of the last timed search (see collect_timing)
  bool timing = false;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  std::vector<hipEvent_t> tev;      // [start, level 1..maxd, chunk x 6, qnet end, end]
  int t_maxd = 0, t_chunks = 0, t_conv1_groups = 0;
  bool t_fused = false, t_tail = false;
  long long t_items = 0, t_nodes = 0;
  double t_ms[24] = {0};
  // serving
  struct ServeEngine* serve = nullptr;
  // launches still to fail on purpose (bcts_debug_fail_launches)
  int inject_fail = 0;
  // captured search graphs alive (bcts_graph_create): they read the
  // weights, so the calls that replace them refuse while any exists
  int live_graphs = 0;
  // learned forward-model world (device weights, and a host copy for the
  // host levels of a search that starts on the CPU)
  void* mlp_mem = nullptr;
  MlpDev mlp{};
  bool mlp_set = false;
  MlpHost mlp_h{};
  int mlp_crossover = 0;               // levels a host-buffer search expands on the CPU
  int mlp_host = 0;                     // host-buffer searches wholly on the CPU: 0 never, 1 always, 2 small trees
};

namespace {

bcts_status fail(bcts_ctx* c, bcts_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) {
    c->err = buf;
    if (st == BCTS_E_HIP) c->error_state = true;
  }
  return st;
}

#define HIPCHECK(ctx, expr)                                                               \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(ctx, BCTS_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));       \
  } while (0)

bcts_status check_usable(bcts_ctx* c) {
  if (!c) return BCTS_E_INVAL;
  if (c->error_state) return BCTS_E_STATE;
  c->err.clear();
  return BCTS_OK;
}

bcts_status ensure_pinned(bcts_ctx* c, size_t bytes) {
  if (c->pinned_bytes >= bytes) return BCTS_OK;
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  if (c->pinned) HIPCHECK(c, hipHostFree(c->pinned));
  c->pinned = nullptr;
  c->pinned_bytes = 0;
  size_t nb = std::max(bytes, (size_t)1 << 20);
  HIPCHECK(c, hipHostMalloc((void**)&c->pinned, nb, hipHostMallocDefault));
  c->pinned_bytes = nb;
  return BCTS_OK;
}

// Work on the arena is ordered on the stream it is enqueued on.  A call on a
// different stream than the previous search first waits (on the device) for
// the event recorded after that search, so it cannot overwrite tables,
// levels or activations the previous search still reads; the arena is only
// freed once that event has completed.
bcts_status order_arena(bcts_ctx* c, hipStream_t s) {
  if (c->arena_pending && c->arena_stream != s) HIPCHECK(c, hipStreamWaitEvent(s, c->arena_ev, 0));
  return BCTS_OK;
}
bcts_status arena_enqueued(bcts_ctx* c, hipStream_t s) {
  if (!c->arena_ev) HIPCHECK(c, hipEventCreateWithFlags(&c->arena_ev, hipEventDisableTiming));
  HIPCHECK(c, hipEventRecord(c->arena_ev, s));
  c->arena_stream = s;
  c->arena_pending = true;
  return BCTS_OK;
}
bcts_status arena_idle(bcts_ctx* c) {
  if (c->arena_pending) HIPCHECK(c, hipEventSynchronize(c->arena_ev));
  c->arena_pending = false;
  return BCTS_OK;
}

bcts_status ensure_arena(bcts_ctx* c, size_t bytes) {
  if (c->arena_bytes >= bytes) return BCTS_OK;
  {
    const bcts_status st = arena_idle(c);
    if (st != BCTS_OK) return st;
  }
  if (bytes + c->wbytes > c->budget)
    return fail(c, BCTS_E_NOMEM, "search needs %zu bytes of device memory; budget is %zu", bytes + c->wbytes,
                c->budget);
  // grow geometrically (bounded by the budget) to avoid re-allocation churn
  size_t want = std::min(std::max(bytes, c->arena_bytes * 3 / 2), c->budget - c->wbytes);
  if (want < bytes) want = bytes;
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  if (c->arena) HIPCHECK(c, hipFree(c->arena));
  c->arena = nullptr;
  c->arena_bytes = 0;
  hipError_t e = hipMalloc((void**)&c->arena, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, BCTS_E_NOMEM, "hipMalloc(%zu) failed: %s", want, hipGetErrorString(e));
  }
  c->arena_bytes = want;
  return BCTS_OK;
}

bcts_status validate_shape(bcts_ctx* c, int A, int d, const bcts_correction& corr) {
  if (A < 1 || A > kMaxA) return fail(c, BCTS_E_INVAL, "A=%d outside [1,18]", A);
  if (d < 0 || d > kMaxD) return fail(c, BCTS_E_INVAL, "depth=%d outside [0,6]", d);
  if (corr.enabled && d >= 1 && A < 2)
    return fail(c, BCTS_E_INVAL, "the correction needs A >= 2 (there is no other action)");
  return BCTS_OK;
}

bcts_status validate_common(bcts_ctx* c, int n, float gamma, const bcts_correction& corr) {
  if (n <= 0) return fail(c, BCTS_E_INVAL, "n_roots=%d must be positive", n);
  if (!(gamma > 0.f && gamma <= 1.f)) return fail(c, BCTS_E_INVAL, "gamma=%g outside (0,1]", gamma);
  if (corr.enabled && !std::isfinite(corr.scale))
    return fail(c, BCTS_E_INVAL, "correction scale is not finite");
  if (corr.enabled && corr.mode != BCTS_CORR_EQ6 && corr.mode != BCTS_CORR_EXACT_GEV)
    return fail(c, BCTS_E_INVAL, "unknown correction mode %d", corr.mode);
  if (!c->env_set) return fail(c, BCTS_E_STATE, "no environment set (bcts_set_env)");
  if (!c->qnet_set) return fail(c, BCTS_E_STATE, "no Q-network set (bcts_set_qnet)");
  return BCTS_OK;
}

bcts_status validate_pos(bcts_ctx* c, int n, const int32_t* pos) {
  for (long long i = 0; i < (long long)n * kSprites * 2; ++i)
    if (pos[i] < 0 || pos[i] >= kFrame)
      return fail(c, BCTS_E_INVAL, "root %lld: position %d outside [0,84)", i / (kSprites * 2), pos[i]);
  return BCTS_OK;
}

// Plan a search with the context's Q-network path settings.
void plan_search(bcts_ctx* c, Plan& p, int n, const int32_t* depth, const int32_t* A, float gamma,
                 const bcts_correction& corr, int q_stride, bool host_io) {
  const bool fz = c->fused && c->prec != P_FP32;
  make_plan(p, n, depth, A, gamma, corr, q_stride, fz ? c->fused_chunk_items : c->chunk_items, c->prec, host_io, fz,
            c->beam, c->corr_fp32, c->chunk_items);
}

// Copy the plan's tables to `arena` through the pinned staging buffer `h`
// (at least p.table_bytes; the caller makes sure no earlier copy still reads it).
bcts_status upload_tables_at(bcts_ctx* c, const Plan& p, char* arena, char* h, hipStream_t s) {
  std::memcpy(h + p.o_roots, p.roots.data(), sizeof(RootInfo) * p.n);
  std::memcpy(h + p.o_segs, p.segs.data(), sizeof(Seg) * p.segs.size());
  std::memcpy(h + p.o_groups, p.groups.data(), sizeof(FusedGroup) * p.groups.size());
  for (int k = 1; k <= p.maxd; ++k) {
    std::memcpy(h + p.o_lroot[k], p.lvl_root[k].data(), sizeof(int) * p.lvl_root[k].size());
    std::memcpy(h + p.o_lstart[k], p.lvl_start[k].data(), sizeof(long long) * p.lvl_start[k].size());
  }
  HIPCHECK(c, hipMemcpyAsync(arena, h, p.table_bytes, hipMemcpyHostToDevice, s));
  return BCTS_OK;
}

// The tables go through the staging buffer not used by the previous search,
// after waiting for that buffer's own last copy only: the host plans and
// stages a search while the previous one still runs.  The device copy is
// ordered on `s` after the previous search's kernels, which read the tables.
bcts_status upload_tables(bcts_ctx* c, const Plan& p, hipStream_t s) {
  {
    const bcts_status st = order_arena(c, s);
    if (st != BCTS_OK) return st;
  }
  const int b = c->tpin_next;
  if (c->tpin_busy[b]) {
    HIPCHECK(c, hipEventSynchronize(c->tpin_ev[b]));
    c->tpin_busy[b] = false;
  }
  if (c->tpin_bytes[b] < p.table_bytes) {
    if (c->tpin[b]) HIPCHECK(c, hipHostFree(c->tpin[b]));
    c->tpin[b] = nullptr;
    c->tpin_bytes[b] = 0;
    const size_t nb = std::max(p.table_bytes, (size_t)1 << 20);
    HIPCHECK(c, hipHostMalloc((void**)&c->tpin[b], nb, hipHostMallocDefault));
    c->tpin_bytes[b] = nb;
  }
  if (!c->tpin_ev[b]) HIPCHECK(c, hipEventCreateWithFlags(&c->tpin_ev[b], hipEventDisableTiming));
  const bcts_status st = upload_tables_at(c, p, c->arena, c->tpin[b], s);
  if (st != BCTS_OK) return st;
  HIPCHECK(c, hipEventRecord(c->tpin_ev[b], s));
  c->tpin_busy[b] = true;
  c->tpin_next = b ^ 1;
  return BCTS_OK;
}

// Enqueue the kernels of a planned search.  Root inputs and outputs are
// device pointers.
bcts_status ensure_events(bcts_ctx* c, size_t n) {
  while (c->tev.size() < n) {
    hipEvent_t e;
    HIPCHECK(c, hipEventCreate(&e));
    c->tev.push_back(e);
  }
  return BCTS_OK;
}

// ---- the launch sequence of a planned search, stage by stage -------------
// A stage is a bounded unit of one search's device work: one level of the
// expansion, one Q-network chunk, the FP32 correction evaluations, or the
// backup.  `A` is the base of the search's arena (the plan's offsets), `desc`
// and `ws` the item descriptors and Q-network workspace the Q-network stages
// use (the arena's own, or a region several searches on one stream share).
// Every stage first passes launch_gate, which lets a test make the next
// launches fail from the host.
bcts_status launch_gate(bcts_ctx* c) {
  if (c->inject_fail > 0) {
    --c->inject_fail;
    return fail(c, BCTS_E_HIP, "injected launch failure (bcts_debug_fail_launches)");
  }
  return BCTS_OK;
}

FrameBases frame_bases(const Plan& p, char* A, const uint8_t* d_stacks) {
  FrameBases fb{};
  fb.level_frames[0] = d_stacks;
  for (int k = 1; k <= p.maxd; ++k) {
    fb.level_frames[k] = reinterpret_cast<const uint8_t*>(A + p.o_frames[k]);
    fb.keep[k] = p.keep_count[k] > 0 ? reinterpret_cast<const int*>(A + p.o_keep[k]) : nullptr;
  }
  return fb;
}

// Level k of the expansion (and its beam cut).
bcts_status enqueue_level(bcts_ctx* c, const Plan& p, char* A, int k, const int32_t* d_pos, float gamma,
                          hipStream_t s) {
  bcts_status st = launch_gate(c);
  if (st != BCTS_OK) return st;
  const RootInfo* roots = reinterpret_cast<const RootInfo*>(A + p.o_roots);
  const float g = discount_f32(gamma, k - 1);    // the FP32 discount a pruned search ranks by
  LevelRoots lr{reinterpret_cast<const int*>(A + p.o_lroot[k]), reinterpret_cast<const long long*>(A + p.o_lstart[k]),
                (int)p.lvl_root[k].size()};
  launch_expand(k, p.lvl_count[k], lr, roots, d_pos,
                k > 1 ? reinterpret_cast<const uint8_t*>(A + p.o_pos[k - 1]) : nullptr,
                k > 1 ? reinterpret_cast<const float*>(A + p.o_ret[k - 1]) : nullptr,
                k > 1 && p.keep_count[k - 1] > 0 ? reinterpret_cast<const int*>(A + p.o_keep[k - 1]) : nullptr,
                c->env, g, reinterpret_cast<uint8_t*>(A + p.o_pos[k]), reinterpret_cast<uint8_t*>(A + p.o_frames[k]),
                reinterpret_cast<float*>(A + p.o_ret[k]), reinterpret_cast<uint8_t*>(A + p.o_rew[k]), s);
  if (p.keep_count[k] > 0)
    launch_prune(k, (int)p.lvl_root[k].size(), lr, roots, reinterpret_cast<const float*>(A + p.o_ret[k]),
                 reinterpret_cast<int*>(A + p.o_keep[k]), p.beam, s);
  return BCTS_OK;
}

// conv1 of a layer-path chunk by sibling groups (true) or stack by stack.
// Workgroups of 128 pixel rows, about kSlots resident at once: the group
// kernel runs 6 + 2 x (group size) stages per workgroup, the per-stack
// kernel 8; the time of a launch is taken as the larger of its total stages
// over the slots and one workgroup's stages.  A lone small request is then
// latency-bound and runs per stack; a chunk of many groups runs by groups.
bool conv1_by_groups(const bcts_ctx* c, const Plan::Chunk& ch) {
  if (c->conv1_groups != 1) return c->conv1_groups == 2;
  constexpr double kSlots = 256.0 * 5.0;            // CUs x resident workgroups of the FP32 kernels
  constexpr double kTilesPerStack = 400.0 / 128.0;  // workgroups per stack (or per group)
  const double per_stack = std::max(8.0 * kTilesPerStack * (double)(ch.i1 - ch.i0) / kSlots, 8.0);
  const double grouped = std::max(kTilesPerStack * (double)ch.group_stages / kSlots, 6.0 + 2.0 * ch.max_group);
  return grouped < per_stack;
}

// Q-network chunk ci of the plan.  With `cev` (6 events) its launches are
// bracketed.
bcts_status enqueue_qnet_chunk(bcts_ctx* c, const Plan& p, char* A, ItemDesc* desc, char* ws, const FrameBases& fb,
                               int ci, hipStream_t s, hipEvent_t* cev) {
  bcts_status st = launch_gate(c);
  if (st != BCTS_OK) return st;
  const RootInfo* roots = reinterpret_cast<const RootInfo*>(A + p.o_roots);
  float* V = reinterpret_cast<float*>(A + p.o_V);
  float* q0 = reinterpret_cast<float*>(A + p.o_q0);
  const FusedGroup* groups = reinterpret_cast<const FusedGroup*>(A + p.o_groups);
  const Plan::Chunk& ch = p.chunks[ci];
  const long long cnt = ch.i1 - ch.i0;
  launch_item_desc(ch.i0, cnt, reinterpret_cast<const Seg*>(A + p.o_segs), (int)p.segs.size(), roots, fb, desc, s);
  if (!p.fused) {
    const ChunkGroups cg{groups + ch.g0, conv1_by_groups(c, ch) ? ch.g1 - ch.g0 : 0, ch.i0};
    launch_qnet_groups(c->prec, c->q, desc, cnt, cg, ws, V + ch.i0, q0, s, cev);
    return BCTS_OK;
  }
  const QnetDev& q = c->q;
  FusedConvArgs fa{};
  fa.groups = groups + ch.g0;
  fa.item_base = ch.i0;
  fa.desc = desc;
  const bool f8 = c->prec == P_FP8;
  for (int l = 0; l < 3; ++l) {
    // conv1 in GEMM layout, conv2 / conv3 fragment-major
    fa.w[l] = l == 0 ? (f8 ? (const void*)q.w8[0] : (const void*)q.wb[0])
                     : (f8 ? (c->fp8_k128 ? q.wf8k[l] : q.wf8[l]) : q.wfb[l]);
    fa.bias[l] = q.b[l];
    fa.acc_scale[l] = f8 ? 1.f / (q.ascale[l] * q.wscale[l]) : 1.f;
    fa.out_s8[l] = f8 ? q.ascale[l + 1] : 1.f;
  }
  fa.acc_scale[0] /= 255.f;
  fa.pix_s8 = f8 ? q.ascale[0] : 1.f;
  char* x3 = ws;
  char* h = x3 + fused_x3_bytes(p.chunk, c->prec);
  fa.x3 = x3;
  if (cev) HIPCHECK(c, hipEventRecord(cev[0], s));
  launch_conv_fused(c->prec, c->fused_T, fa, ch.g1 - ch.g0, s, c->fp8_k128);
  if (cev) {
    HIPCHECK(c, hipEventRecord(cev[1], s));
    HIPCHECK(c, hipEventRecord(cev[2], s));
    HIPCHECK(c, hipEventRecord(cev[3], s));
  }
  launch_qnet_fc(c->prec, q, desc, cnt, x3, h, V + ch.i0, q0, s, cev ? cev[4] : nullptr, c->fc2_folded);
  if (cev) HIPCHECK(c, hipEventRecord(cev[5], s));
  return BCTS_OK;
}

// The correction's root and depth-1 evaluations in FP32 (layer kernels).
bcts_status enqueue_tail(bcts_ctx* c, const Plan& p, char* A, ItemDesc* desc, char* ws, const FrameBases& fb,
                         hipStream_t s) {
  if (p.tail_chunks.empty()) return BCTS_OK;
  bcts_status st = launch_gate(c);
  if (st != BCTS_OK) return st;
  const RootInfo* roots = reinterpret_cast<const RootInfo*>(A + p.o_roots);
  float* V = reinterpret_cast<float*>(A + p.o_V);
  float* q0 = reinterpret_cast<float*>(A + p.o_q0);
  const FusedGroup* groups = reinterpret_cast<const FusedGroup*>(A + p.o_groups);
  for (const auto& tc : p.tail_chunks) {
    const long long cnt = tc.i1 - tc.i0;
    launch_item_desc(tc.i0, cnt, reinterpret_cast<const Seg*>(A + p.o_segs), (int)p.segs.size(), roots, fb, desc, s);
    const ChunkGroups cg{groups + tc.g0, conv1_by_groups(c, tc) ? tc.g1 - tc.g0 : 0, tc.i0};
    launch_qnet_groups(P_FP32, c->q, desc, cnt, cg, ws, V + tc.i0, q0, s, nullptr);
  }
  return BCTS_OK;
}

// Backup, correction and root action into d_act / d_q.
bcts_status enqueue_backup(bcts_ctx* c, const Plan& p, char* A, float gamma, float corr_scale, int32_t* d_act,
                           float* d_q, hipStream_t s) {
  bcts_status st = launch_gate(c);
  if (st != BCTS_OK) return st;
  LevelRet lr{};
  for (int k = 1; k <= p.maxd; ++k) lr.ret[k] = reinterpret_cast<const float*>(A + p.o_ret[k]);
  launch_backup_correct(p.n, reinterpret_cast<const RootInfo*>(A + p.o_roots), reinterpret_cast<float*>(A + p.o_V),
                        reinterpret_cast<float*>(A + p.o_q0), lr, gamma, corr_scale, d_act, d_q, s);
  return BCTS_OK;
}

// Q-network over every eval item of the plan, chunk by chunk, then the FP32
// correction evaluations.  With `ev` (6 events per chunk, then 2 around the
// FP32 evaluations) the launches are bracketed.
bcts_status enqueue_qnet_stage(bcts_ctx* c, const Plan& p, char* A, const FrameBases& fb, hipStream_t s,
                               hipEvent_t* ev) {
  ItemDesc* desc = reinterpret_cast<ItemDesc*>(A + p.o_desc);
  char* ws = A + p.o_ws;
  const int nchunks = (int)p.chunks.size();
  for (int ci = 0; ci < nchunks; ++ci) {
    const bcts_status st = enqueue_qnet_chunk(c, p, A, desc, ws, fb, ci, s, ev ? ev + 6 * ci : nullptr);
    if (st != BCTS_OK) return st;
  }
  if (ev && !p.tail_chunks.empty()) HIPCHECK(c, hipEventRecord(ev[6 * nchunks], s));
  const bcts_status st = enqueue_tail(c, p, A, desc, ws, fb, s);
  if (st != BCTS_OK) return st;
  if (ev && !p.tail_chunks.empty()) HIPCHECK(c, hipEventRecord(ev[6 * nchunks + 1], s));
  return BCTS_OK;
}

// Enqueue the whole search (every stage, in order).  Root inputs and
// outputs are device pointers.
bcts_status enqueue_search_at(bcts_ctx* c, const Plan& p, char* A, const int32_t* d_pos,
                              const uint8_t* d_stacks, float gamma, float corr_scale, int32_t* d_act,
                              float* d_q, hipStream_t s, bool timed) {
  const int nchunks = (int)p.chunks.size();
  hipEvent_t* ev = nullptr;
  if (timed) {
    bcts_status st = ensure_events(c, (size_t)(5 + p.maxd + 6 * nchunks));
    if (st != BCTS_OK) return st;
    ev = c->tev.data();
    c->t_maxd = p.maxd;
    c->t_chunks = nchunks;
    c->t_fused = p.fused;
    c->t_items = p.n_items;
    c->t_tail = !p.tail_chunks.empty();
    c->t_conv1_groups = 0;
    if (!p.fused)
      for (const auto& ch : p.chunks) c->t_conv1_groups += conv1_by_groups(c, ch) ? 1 : 0;
    c->t_nodes = 0;
    for (int k = 1; k <= p.maxd; ++k) c->t_nodes += p.lvl_count[k];
    HIPCHECK(c, hipEventRecord(ev[0], s));
  }
  bcts_status st;
  for (int k = 1; k <= p.maxd; ++k) {
    if ((st = enqueue_level(c, p, A, k, d_pos, gamma, s)) != BCTS_OK) return st;
    if (timed) HIPCHECK(c, hipEventRecord(ev[k], s));
  }
  const FrameBases fb = frame_bases(p, A, d_stacks);
  if ((st = enqueue_qnet_stage(c, p, A, fb, s, timed ? ev + 1 + p.maxd : nullptr)) != BCTS_OK) return st;
  if (timed) HIPCHECK(c, hipEventRecord(ev[3 + p.maxd + 6 * nchunks], s));
  if ((st = enqueue_backup(c, p, A, gamma, corr_scale, d_act, d_q, s)) != BCTS_OK) return st;
  if (timed) HIPCHECK(c, hipEventRecord(ev[4 + p.maxd + 6 * nchunks], s));
  HIPCHECK(c, hipGetLastError());
  return BCTS_OK;
}

bcts_status enqueue_search(bcts_ctx* c, const Plan& p, const int32_t* d_pos, const uint8_t* d_stacks,
                           float gamma, float corr_scale, int32_t* d_act, float* d_q, hipStream_t s,
                           bool timed) {
  return enqueue_search_at(c, p, c->arena, d_pos, d_stacks, gamma, corr_scale, d_act, d_q, s, timed);
}

// Per-stage and per-kernel durations of the last timed search:
// [0] expansion, [1] Q-network, [2] backup + correction, [3] total (ms);
// [4..8] conv1, conv2, conv3, fc1, fc2 summed over chunks (ms); [9] chunks;
// [10..15] expansion of levels 1..6 (ms); [16] eval items; [17] new nodes;
// [18] fused kernel ran; [19] FP32 correction evaluations (ms); [20] chunks
// of the layer path whose conv1 ran by sibling groups.
// Events: [0] start, [k] after level k, then 6 per chunk, 2 around the FP32
// correction evaluations, the Q-network end and the search end.
bcts_status collect_timing(bcts_ctx* c) {
  const int D = c->t_maxd, C = c->t_chunks;
  hipEvent_t* ev = c->tev.data();
  const int tail0 = 1 + D + 6 * C, q_end = tail0 + 2, end = q_end + 1;
  HIPCHECK(c, hipEventSynchronize(ev[end]));
  auto el = [&](int a, int b) -> double {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ev[a], ev[b]) != hipSuccess) return -1.0;
    return ms;
  };
  for (double& v : c->t_ms) v = 0.0;
  c->t_ms[0] = el(0, D);
  c->t_ms[1] = el(D, q_end);
  c->t_ms[2] = el(q_end, end);
  c->t_ms[3] = el(0, end);
  for (int ci = 0; ci < C; ++ci)
    for (int l = 0; l < 5; ++l) c->t_ms[4 + l] += el(1 + D + 6 * ci + l, 1 + D + 6 * ci + l + 1);
  c->t_ms[9] = C;
  for (int k = 1; k <= D; ++k) c->t_ms[9 + k] = el(k - 1, k);
  c->t_ms[16] = (double)c->t_items;
  c->t_ms[17] = (double)c->t_nodes;
  c->t_ms[18] = c->t_fused ? 1.0 : 0.0;
  c->t_ms[19] = c->t_tail ? el(tail0, tail0 + 1) : 0.0;
  c->t_ms[20] = c->t_conv1_groups;
  return BCTS_OK;
}

// Host-buffer search: stage inputs, run, copy results back.
bcts_status search_host(bcts_ctx* c, int n, const int32_t* pos, const uint8_t* stacks, const int32_t* depth,
                        const int32_t* Av, float gamma, const bcts_correction& corr, int32_t* out_action,
                        float* out_q, int q_stride) {
  Plan p;
  plan_search(c, p, n, depth, Av, gamma, corr, q_stride, true);
  bcts_status st = ensure_arena(c, p.total);
  if (st != BCTS_OK) return st;
  hipStream_t s = c->stream;
  st = upload_tables(c, p, s);
  if (st != BCTS_OK) return st;
  const size_t in_bytes = sizeof(int32_t) * n * kSprites * 2 + (size_t)n * 4 * kFrameBytes;
  const size_t out_bytes = sizeof(int32_t) * n + sizeof(float) * (size_t)n * q_stride;
  st = ensure_pinned(c, std::max(p.table_bytes, std::max(in_bytes, out_bytes)));
  if (st != BCTS_OK) return st;
  HIPCHECK(c, hipStreamSynchronize(s));
  std::memcpy(c->pinned, pos, sizeof(int32_t) * n * kSprites * 2);
  HIPCHECK(c, hipMemcpyAsync(c->arena + p.o_root_pos, c->pinned, sizeof(int32_t) * n * kSprites * 2,
                             hipMemcpyHostToDevice, s));
  // stacks can be large: copy directly (synchronous for pageable memory)
  HIPCHECK(c, hipMemcpyAsync(c->arena + p.o_root_stack, stacks, (size_t)n * 4 * kFrameBytes,
                             hipMemcpyHostToDevice, s));
  int32_t* d_act = reinterpret_cast<int32_t*>(c->arena + p.o_act);
  float* d_q = reinterpret_cast<float*>(c->arena + p.o_q);
  st = enqueue_search(c, p, reinterpret_cast<const int32_t*>(c->arena + p.o_root_pos),
                      reinterpret_cast<const uint8_t*>(c->arena + p.o_root_stack), gamma,
                      corr.enabled ? corr.scale : 0.f, d_act, d_q, s, c->timing);
  if (st != BCTS_OK) return st;
  HIPCHECK(c, hipMemcpyAsync(out_action, d_act, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
  HIPCHECK(c, hipMemcpyAsync(out_q, d_q, sizeof(float) * (size_t)n * q_stride, hipMemcpyDeviceToHost, s));
  HIPCHECK(c, hipStreamSynchronize(s));
  c->arena_pending = false;
  if (c->timing) return collect_timing(c);
  return BCTS_OK;
}

}  // namespace


// ===========================================================================
// Serving: iteration-level continuous batching with pooled HBM admission.
//
// Requests queue on bcts_submit.  The engine runs in steps, all on its own
// stream.  Before a step it admits queued requests, in arrival order, as a
// new cohort (the requests admitted together, planned as one batch) while
// the memory pool and the pinned staging pool hold its plan; then the step
// advances every admitted cohort by one stage of its search -- its upload
// and level 1, each further level, each Q-network chunk, the FP32 correction
// evaluations, the backup with the copy of its results to the host.  A light
// cohort (few nodes and items) runs all its stages in one step.  A request
// that arrives while a large search runs therefore joins at the next stage
// boundary and completes after a few steps, not after that search.
// Every cohort's device memory is one range of a single pool; the range
// returns to the pool when the step holding the cohort's last stage has
// finished on the device.  The Q-network stages of all cohorts share one
// descriptor and workspace region: they run on one stream, one at a time.
// Up to `max_steps` steps are in flight; the host plans and stages the next
// step while the device runs the previous one.
// ===========================================================================
struct ServeReq {
  uint64_t ticket;
  int A, d;
  float gamma;
  bcts_correction corr;
  int32_t pos[kSprites * 2];
  std::vector<uint8_t> stack;
};

struct ServeResult {
  int action;
  int A;
  float q[kMaxA];
  double t_done;
};

struct Cohort {
  std::vector<uint64_t> tickets;
  std::vector<int> A;
  float gamma = 1.f;
  bcts_correction corr{};
  Plan p;
  size_t dev_off = 0, pin_off = 0, pin_bytes = 0;
  size_t h_pos = 0, h_stack = 0, h_act = 0, h_q = 0;   // offsets inside its pinned range
  int n_stages = 0, next = 0;     // stages: levels 1..maxd, chunks, FP32 tail (if any), backup
  bool light = false;             // all stages in one step
  uint64_t last_step = 0;         // step holding its last stage (valid once next == n_stages)
};

struct ServeEngine {
  bcts_ctx* c;
  int max_batch = 512, max_steps = 2;
  long long layer_chunk = 2048;              // stacks per Q-network chunk (layer path; fused: 8x)
  static constexpr size_t kPoolCap = (size_t)16 << 30;     // device pool cap (bytes)
  static constexpr size_t kPinnedBytes = (size_t)96 << 20; // pinned staging pool
  static constexpr long long kCohortLeaves = 1 << 19;      // leaves admitted into one cohort, at most
  static constexpr long long kLightWork = 32768;           // nodes + items of a light cohort
  bool ready = false;
  struct Settings {
    int prec, fused, T, corr_fp32, beam;
    long long fchunk, lchunk;
    bool operator==(const Settings& o) const {
      return prec == o.prec && fused == o.fused && T == o.T && corr_fp32 == o.corr_fp32 && beam == o.beam &&
             fchunk == o.fchunk && lchunk == o.lchunk;
    }
  } cfg{};
  uint64_t cohorts_done = 0, requests_done = 0;
  hipStream_t stream = nullptr;
  char* dev = nullptr;          // [shared desc + workspace | pool]
  size_t dev_bytes = 0, shared_bytes = 0;
  RangePool pool, pin_pool;
  char* pinned = nullptr;
  std::deque<ServeReq> queue;
  std::list<Cohort> active;
  struct Step { hipEvent_t ev; uint64_t id; };
  std::deque<Step> inflight;
  std::vector<hipEvent_t> spare_events;
  uint64_t step_id = 0, done_step = 0;
  std::unordered_map<uint64_t, ServeResult> results;
  std::unordered_set<uint64_t> live;
  uint64_t next_ticket = 1;

  explicit ServeEngine(bcts_ctx* ctx) : c(ctx) {}
  ~ServeEngine() { release(); }

  bool fused() const { return c->fused && c->prec != P_FP32; }
  long long chunk_items() const { return fused() ? 8 * layer_chunk : layer_chunk; }
  Settings current() const {
    return Settings{c->prec, c->fused ? 1 : 0, c->fused_T, c->corr_fp32 ? 1 : 0, c->beam, chunk_items(),
                    layer_chunk};
  }
  bool busy() const { return !queue.empty() || !active.empty(); }
  size_t pool_capacity() const { return ready ? pool.capacity() : 0; }

  // descriptors + workspace of the largest Q-network stage of any cohort
  size_t shared_need() const {
    const long long ch = chunk_items(), tail = layer_chunk;
    size_t ws = fused() ? fused_workspace_bytes(ch, c->prec) : qnet_workspace_bytes(ch, c->prec);
    ws = std::max(ws, qnet_workspace_bytes(tail, P_FP32));
    return align_up(sizeof(ItemDesc) * (size_t)std::max(ch, tail)) + align_up(ws);
  }

  void release() {
    if (stream) (void)hipStreamSynchronize(stream);
    for (auto& st : inflight) (void)hipEventDestroy(st.ev);
    inflight.clear();
    for (hipEvent_t e : spare_events) (void)hipEventDestroy(e);
    spare_events.clear();
    active.clear();
    if (dev) (void)hipFree(dev);
    if (pinned) (void)hipHostFree(pinned);
    if (stream) (void)hipStreamDestroy(stream);
    dev = nullptr;
    pinned = nullptr;
    stream = nullptr;
    dev_bytes = shared_bytes = 0;
    ready = false;
  }

  void drop_all() {
    release();
    queue.clear();
    results.clear();
    live.clear();
  }

  // Allocate the pools for the context's current settings; an idle engine
  // whose settings changed (precision, fusion, chunking, beam) is rebuilt.
  bcts_status init() {
    const Settings now = current();
    if (ready && now == cfg) return BCTS_OK;
    if (ready && busy()) return fail(c, BCTS_E_STATE, "serving settings changed while requests are in flight");
    release();
    cfg = now;
    const size_t used = c->wbytes + c->arena_bytes;
    const size_t avail = c->budget > used ? c->budget - used : 0;
    shared_bytes = shared_need();
    if (avail <= shared_bytes + kAlign)
      return fail(c, BCTS_E_NOMEM, "serving needs %zu bytes of workspace; the budget leaves %zu", shared_bytes, avail);
    dev_bytes = std::min(avail, shared_bytes + kPoolCap) / kAlign * kAlign;
    HIPCHECK(c, hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
    hipError_t e = hipMalloc((void**)&dev, dev_bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      dev = nullptr;
      return fail(c, BCTS_E_NOMEM, "hipMalloc(%zu) for the serving pool failed: %s", dev_bytes, hipGetErrorString(e));
    }
    HIPCHECK(c, hipHostMalloc((void**)&pinned, kPinnedBytes, hipHostMallocDefault));
    pool.reset(dev_bytes - shared_bytes);
    pin_pool.reset(kPinnedBytes);
    ready = true;
    return BCTS_OK;
  }

  hipEvent_t take_event() {
    if (!spare_events.empty()) {
      hipEvent_t e = spare_events.back();
      spare_events.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
  }

  // Finished steps, then the cohorts whose last stage they held.
  bcts_status retire() {
    while (!inflight.empty()) {
      const hipError_t e = hipEventQuery(inflight.front().ev);
      if (e == hipErrorNotReady) break;
      if (e != hipSuccess) return fail(c, BCTS_E_HIP, "serving step failed: %s", hipGetErrorString(e));
      done_step = inflight.front().id;
      spare_events.push_back(inflight.front().ev);
      inflight.pop_front();
    }
    const double t = now_s();
    for (auto it = active.begin(); it != active.end();) {
      Cohort& k = *it;
      if (k.next < k.n_stages || k.last_step > done_step) { ++it; continue; }
      const int32_t* act = reinterpret_cast<const int32_t*>(pinned + k.pin_off + k.h_act);
      const float* q = reinterpret_cast<const float*>(pinned + k.pin_off + k.h_q);
      for (size_t i = 0; i < k.tickets.size(); ++i) {
        ServeResult r;
        r.action = act[i];
        r.A = k.A[i];
        for (int a = 0; a < kMaxA; ++a) r.q[a] = q[i * kMaxA + a];
        r.t_done = t;
        if (live.count(k.tickets[i])) results[k.tickets[i]] = r;
      }
      pool.release(k.dev_off, k.p.search_bytes());
      pin_pool.release(k.pin_off, k.pin_bytes);
      ++cohorts_done;
      requests_done += k.tickets.size();
      it = active.erase(it);
    }
    return BCTS_OK;
  }

  // Admit the longest FIFO prefix of compatible requests that fits a
  // cohort; returns false when the front request cannot be admitted now.
  bool admit_one() {
    if (queue.empty()) return false;
    const ServeReq& f = queue.front();
    int n = 0;
    long long leaves = 0;
    for (const auto& r : queue) {
      long long lv = 1;
      for (int k = 0; k < r.d; ++k) lv *= r.A;
      if (n >= max_batch || r.gamma != f.gamma || r.corr.enabled != f.corr.enabled ||
          r.corr.scale != f.corr.scale || r.corr.mode != f.corr.mode || (n > 0 && leaves + lv > kCohortLeaves))
        break;
      leaves += lv;
      ++n;
    }
    std::vector<int32_t> dep(n), Av(n);
    for (int i = 0; i < n; ++i) { dep[i] = queue[i].d; Av[i] = queue[i].A; }
    for (;;) {
      Cohort k;
      make_plan(k.p, n, dep.data(), Av.data(), f.gamma, f.corr, kMaxA, chunk_items(), c->prec, true, fused(),
                c->beam, c->corr_fp32, layer_chunk);
      k.h_pos = align_up(k.p.table_bytes);
      k.h_stack = k.h_pos + align_up(sizeof(int32_t) * n * kSprites * 2);
      k.h_act = k.h_stack + align_up((size_t)n * 4 * kFrameBytes);
      k.h_q = k.h_act + align_up(sizeof(int32_t) * n);
      k.pin_bytes = k.h_q + align_up(sizeof(float) * (size_t)n * kMaxA);
      bool ok = pool.alloc(k.p.search_bytes(), &k.dev_off);
      if (ok && !pin_pool.alloc(k.pin_bytes, &k.pin_off)) {
        pool.release(k.dev_off, k.p.search_bytes());
        ok = false;
      }
      if (!ok) {
        if (n == 1) return false;     // wait for memory (arrival order is kept)
        n = (n + 1) / 2;              // a smaller prefix may fit now
        continue;
      }
      // stage the tables and inputs in the cohort's pinned range
      char* h = pinned + k.pin_off;
      const Plan& p = k.p;
      std::memcpy(h + p.o_roots, p.roots.data(), sizeof(RootInfo) * p.n);
      std::memcpy(h + p.o_segs, p.segs.data(), sizeof(Seg) * p.segs.size());
      std::memcpy(h + p.o_groups, p.groups.data(), sizeof(FusedGroup) * p.groups.size());
      for (int lv = 1; lv <= p.maxd; ++lv) {
        std::memcpy(h + p.o_lroot[lv], p.lvl_root[lv].data(), sizeof(int) * p.lvl_root[lv].size());
        std::memcpy(h + p.o_lstart[lv], p.lvl_start[lv].data(), sizeof(long long) * p.lvl_start[lv].size());
      }
      int32_t* hp = reinterpret_cast<int32_t*>(h + k.h_pos);
      uint8_t* hs = reinterpret_cast<uint8_t*>(h + k.h_stack);
      k.tickets.resize(n);
      k.A.resize(n);
      for (int i = 0; i < n; ++i) {
        const ServeReq& r = queue[i];
        std::memcpy(hp + i * kSprites * 2, r.pos, sizeof r.pos);
        std::memcpy(hs + (size_t)i * 4 * kFrameBytes, r.stack.data(), (size_t)4 * kFrameBytes);
        k.tickets[i] = r.ticket;
        k.A[i] = r.A;
      }
      k.gamma = f.gamma;
      k.corr = f.corr;
      k.n_stages = p.maxd + (int)p.chunks.size() + (p.tail_chunks.empty() ? 0 : 1) + 1;
      long long work = p.n_items;
      for (int lv = 1; lv <= p.maxd; ++lv) work += p.lvl_count[lv];
      k.light = work <= kLightWork;
      for (int i = 0; i < n; ++i) queue.pop_front();
      active.push_back(std::move(k));
      return true;
    }
  }

  // Stage `i` of cohort k on the engine stream (stage 0 also uploads).
  bcts_status enqueue_stage(Cohort& k, int i) {
    const Plan& p = k.p;
    char* A = dev + shared_bytes + k.dev_off;
    char* h = pinned + k.pin_off;
    ItemDesc* desc = reinterpret_cast<ItemDesc*>(dev);
    char* ws = dev + align_up(sizeof(ItemDesc) * (size_t)std::max(chunk_items(), layer_chunk));
    const int32_t* d_pos = reinterpret_cast<const int32_t*>(A + p.o_root_pos);
    const uint8_t* d_stacks = reinterpret_cast<const uint8_t*>(A + p.o_root_stack);
    const int n = p.n;
    if (i == 0) {
      HIPCHECK(c, hipMemcpyAsync(A, h, p.table_bytes, hipMemcpyHostToDevice, stream));
      HIPCHECK(c, hipMemcpyAsync(A + p.o_root_pos, h + k.h_pos, sizeof(int32_t) * n * kSprites * 2,
                                 hipMemcpyHostToDevice, stream));
      HIPCHECK(c, hipMemcpyAsync(A + p.o_root_stack, h + k.h_stack, (size_t)n * 4 * kFrameBytes,
                                 hipMemcpyHostToDevice, stream));
    }
    const int nl = p.maxd, nc = (int)p.chunks.size(), nt = p.tail_chunks.empty() ? 0 : 1;
    if (i < nl) return enqueue_level(c, p, A, i + 1, d_pos, k.gamma, stream);
    const FrameBases fb = frame_bases(p, A, d_stacks);
    if (i < nl + nc) return enqueue_qnet_chunk(c, p, A, desc, ws, fb, i - nl, stream, nullptr);
    if (i < nl + nc + nt) return enqueue_tail(c, p, A, desc, ws, fb, stream);
    int32_t* d_act = reinterpret_cast<int32_t*>(A + p.o_act);
    float* d_q = reinterpret_cast<float*>(A + p.o_q);
    bcts_status st = enqueue_backup(c, p, A, k.gamma, k.corr.enabled ? k.corr.scale : 0.f, d_act, d_q, stream);
    if (st != BCTS_OK) return st;
    HIPCHECK(c, hipMemcpyAsync(h + k.h_act, d_act, sizeof(int32_t) * n, hipMemcpyDeviceToHost, stream));
    HIPCHECK(c, hipMemcpyAsync(h + k.h_q, d_q, sizeof(float) * (size_t)n * kMaxA, hipMemcpyDeviceToHost, stream));
    return BCTS_OK;
  }

  // One step: admissions, then one stage of every cohort (all of a light
  // one).  Returns whether anything was enqueued.
  bcts_status step(bool* did) {
    *did = false;
    while (admit_one()) {
    }
    const uint64_t id = step_id + 1;
    bool any = false;
    for (Cohort& k : active) {
      if (k.next >= k.n_stages) continue;
      const int upto = k.light ? k.n_stages : k.next + 1;
      for (; k.next < upto; ++k.next) {
        const bcts_status st = enqueue_stage(k, k.next);
        if (st != BCTS_OK) return st;
      }
      if (k.next == k.n_stages) k.last_step = id;
      any = true;
    }
    if (!any) return BCTS_OK;
    HIPCHECK(c, hipGetLastError());
    hipEvent_t ev = take_event();
    if (!ev) return fail(c, BCTS_E_HIP, "hipEventCreate failed");
    HIPCHECK(c, hipEventRecord(ev, stream));
    inflight.push_back(Step{ev, id});
    step_id = id;
    *did = true;
    return BCTS_OK;
  }

  bcts_status progress(int* pending) {
    bcts_status st = init();
    if (st != BCTS_OK) return st;
    if ((st = retire()) != BCTS_OK) return st;
    while ((int)inflight.size() < max_steps) {
      bool did = false;
      if ((st = step(&did)) != BCTS_OK) return st;
      if (!did) break;
    }
    if (pending) {
      int n = (int)queue.size();
      for (const auto& k : active) n += (int)k.tickets.size();
      *pending = n;
    }
    return BCTS_OK;
  }
};

// Serving work that reads the context's model, tables and settings: queued
// requests and admitted cohorts (finished results waiting for bcts_poll do
// not count).  The calls that change that state refuse while it exists.
static bcts_status refuse_if_serving(bcts_ctx* c, const char* what) {
  if (c->live_graphs > 0)
    return fail(c, BCTS_E_STATE, "%s: %d captured search graph(s) still exist", what, c->live_graphs);
  if (!c->serve) return BCTS_OK;
  bcts_status st = c->serve->retire();
  if (st != BCTS_OK) return st;
  if (c->serve->busy()) return fail(c, BCTS_E_STATE, "%s: serving requests are queued or in flight", what);
  return BCTS_OK;
}

// ---------------------------------------------------------------------------
// Static scratch of bcts_search_batch_device_noalloc: device memory the
// library never allocates at run time.  Host code uses the array's name only
// to look up its device address (once per device, at bcts_create); kernels
// receive that address, as they receive the arena in the other entry points.
// Each device holds its own copy until the process ends; every context on a
// device shares it.
constexpr size_t kScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

constexpr int kScratchDevs = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kScratchDevs] = {};

// The device address of `scratch` on the current device (c->device).
void scratch_setup(bcts_ctx* c) {
  if (c->device >= kScratchDevs) {
    c->scratch_err = "device index beyond the static scratch table";
    return;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[c->device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      c->scratch_err = std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e);
      return;
    }
    g_scratch_ptr[c->device] = static_cast<char*>(ptr);
  }
  c->scratch = g_scratch_ptr[c->device];
}

}  // namespace

// ===========================================================================
extern "C" {

bcts_status bcts_create(int hip_device, size_t hbm_budget_bytes, bcts_ctx** out) {
  if (!out) return BCTS_E_INVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev) {
    (void)hipGetLastError();
    return BCTS_E_HIP;
  }
  if (hipSetDevice(hip_device) != hipSuccess) return BCTS_E_HIP;
  bcts_ctx* c = new bcts_ctx();
  c->device = hip_device;
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) { delete c; return BCTS_E_HIP; }
  c->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.8 * (double)fr);
  bool ok = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) == hipSuccess;
  for (int i = 0; i < 4 && ok; ++i) ok = hipEventCreate(&c->ev[i]) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&c->na_ev, hipEventDisableTiming) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&c->na_copy_ev, hipEventDisableTiming) == hipSuccess;
  if (!ok) {                          // release what was created
    (void)hipGetLastError();
    bcts_destroy(c);
    return BCTS_E_HIP;
  }
  scratch_setup(c);                   // device address of the static scratch (device current)
  *out = c;
  return BCTS_OK;
}

void bcts_destroy(bcts_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  if (c->arena_pending) (void)hipEventSynchronize(c->arena_ev);
  if (c->na_pending) (void)hipEventSynchronize(c->na_ev);
  if (c->na_copy_pending) (void)hipEventSynchronize(c->na_copy_ev);
  delete c->serve;
  if (c->arena) (void)hipFree(c->arena);
  if (c->wmem) (void)hipFree(c->wmem);
  if (c->mlp_mem) (void)hipFree(c->mlp_mem);
  if (c->pinned) (void)hipHostFree(c->pinned);
  for (int b = 0; b < 2; ++b) {
    if (c->tpin_ev[b]) (void)hipEventSynchronize(c->tpin_ev[b]);
    if (c->tpin_ev[b]) (void)hipEventDestroy(c->tpin_ev[b]);
    if (c->tpin[b]) (void)hipHostFree(c->tpin[b]);
  }
  for (int i = 0; i < 4; ++i)
    if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
  if (c->arena_ev) (void)hipEventDestroy(c->arena_ev);
  if (c->na_ev) (void)hipEventDestroy(c->na_ev);
  if (c->na_copy_ev) (void)hipEventDestroy(c->na_copy_ev);
  for (hipEvent_t e : c->tev) (void)hipEventDestroy(e);
  if (c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

const char* bcts_last_error(const bcts_ctx* c) { return c ? c->err.c_str() : "null context"; }

bcts_status bcts_reset(bcts_ctx* c) {
  if (!c) return BCTS_E_INVAL;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  if (c->arena_pending) (void)hipEventSynchronize(c->arena_ev);
  c->arena_pending = false;
  if (c->na_pending) (void)hipEventSynchronize(c->na_ev);
  c->na_pending = false;
  if (c->na_copy_pending) (void)hipEventSynchronize(c->na_copy_ev);
  c->na_copy_pending = false;
  (void)hipGetLastError();
  if (c->serve) c->serve->drop_all();
  if (c->arena) (void)hipFree(c->arena);
  c->arena = nullptr;
  c->arena_bytes = 0;
  c->error_state = false;
  c->err.clear();
  return BCTS_OK;
}

bcts_status bcts_set_env(bcts_ctx* c, const bcts_env_params* env) {
  bcts_status st = check_usable(c);
  if (st != BCTS_OK) return st;
  if ((st = refuse_if_serving(c, "bcts_set_env")) != BCTS_OK) return st;
  if (!env) return fail(c, BCTS_E_INVAL, "env is NULL");
  for (int a = 0; a < kMaxA; ++a)
    for (int k = 0; k < 2; ++k)
      if (env->delta[a][k] < -3 || env->delta[a][k] > 3)
        return fail(c, BCTS_E_INVAL, "delta[%d] outside [-3,3]", a);
  for (int i = 0; i < kSprites - 1; ++i)
    for (int k = 0; k < 2; ++k)
      if (env->vel[i][k] < -2 || env->vel[i][k] > 2)
        return fail(c, BCTS_E_INVAL, "vel[%d] outside [-2,2]", i);
  std::memcpy(c->env.delta, env->delta, sizeof c->env.delta);
  std::memcpy(c->env.vel, env->vel, sizeof c->env.vel);
  c->env_set = true;
  return BCTS_OK;
}

bcts_status bcts_set_qnet(bcts_ctx* c, const float* blob, size_t n_floats) {
  bcts_status st = check_usable(c);
  if (st != BCTS_OK) return st;
  if ((st = refuse_if_serving(c, "bcts_set_qnet")) != BCTS_OK) return st;
  if (!blob) return fail(c, BCTS_E_INVAL, "blob is NULL");
  if (n_floats != (size_t)BCTS_QNET_NUMEL)
    return fail(c, BCTS_E_INVAL, "blob has %zu floats, expected %d", n_floats, BCTS_QNET_NUMEL);
  for (size_t i = 0; i < n_floats; ++i)
    if (!std::isfinite(blob[i])) return fail(c, BCTS_E_INVAL, "blob[%zu] is not finite", i);
  HIPCHECK(c, hipSetDevice(c->device));
  // re-layout to W[N][K] with the K orders of the implicit GEMMs
  static const int NK[5][2] = {{32, 256}, {64, 512}, {64, 576}, {512, 3136}, {32, 512}};
  std::vector<float> W[5], B[5];
  const float* p = blob;
  const float* c1w = p; p += 32 * 256;  const float* c1b = p; p += 32;
  const float* c2w = p; p += 64 * 512;  const float* c2b = p; p += 64;
  const float* c3w = p; p += 64 * 576;  const float* c3b = p; p += 64;
  const float* f1w = p; p += 512 * 3136; const float* f1b = p; p += 512;
  const float* f2w = p; p += 18 * 512;  const float* f2b = p; p += 18;
  for (int l = 0; l < 5; ++l) { W[l].assign((size_t)NK[l][0] * NK[l][1], 0.f); B[l].assign(NK[l][0], 0.f); }
  std::memcpy(W[0].data(), c1w, sizeof(float) * 32 * 256);            // (c, kh, kw) as OIHW
  for (int o = 0; o < 64; ++o)
    for (int ci = 0; ci < 32; ++ci)
      for (int kh = 0; kh < 4; ++kh)
        for (int kw = 0; kw < 4; ++kw)
          W[1][(size_t)o * 512 + (kh * 4 + kw) * 32 + ci] = c2w[((o * 32 + ci) * 4 + kh) * 4 + kw];
  for (int o = 0; o < 64; ++o)
    for (int ci = 0; ci < 64; ++ci)
      for (int kh = 0; kh < 3; ++kh)
        for (int kw = 0; kw < 3; ++kw)
          W[2][(size_t)o * 576 + (kh * 3 + kw) * 64 + ci] = c3w[((o * 64 + ci) * 3 + kh) * 3 + kw];
  for (int o = 0; o < 512; ++o)
    for (int ci = 0; ci < 64; ++ci)
      for (int hw = 0; hw < 49; ++hw)
        W[3][(size_t)o * 3136 + hw * 64 + ci] = f1w[(size_t)o * 3136 + ci * 49 + hw];
  std::memcpy(W[4].data(), f2w, sizeof(float) * 18 * 512);              // rows 18..31 stay 0
  std::memcpy(B[0].data(), c1b, sizeof(float) * 32);
  std::memcpy(B[1].data(), c2b, sizeof(float) * 64);
  std::memcpy(B[2].data(), c3b, sizeof(float) * 64);
  std::memcpy(B[3].data(), f1b, sizeof(float) * 512);
  std::memcpy(B[4].data(), f2b, sizeof(float) * 18);

  // fp32 w, bf16 w, fp8 w, bias, and for conv2 / conv3 fragment-major (fc1: stage-major tiled)
  // bf16 and fp8 copies
  size_t off[5][7], o = 0;
  for (int l = 0; l < 5; ++l) {
    const size_t n = W[l].size();
    off[l][0] = o; o += align_up(n * 4);
    off[l][1] = o; o += align_up(n * 2);
    off[l][2] = o; o += align_up(n);
    off[l][3] = o; o += align_up(B[l].size() * 4);
    const size_t fc1_tiles = (size_t)(NK[3][0] / kFc1Rows);
    off[l][4] = o; o += (l == 1 || l == 2) ? align_up(n * 2) : l == 3 ? align_up(fc1_tiles * fc1_tile_bytes(2)) : 0;
    off[l][5] = o; o += (l == 1 || l == 2) ? align_up(n) : l == 3 ? align_up(fc1_tiles * fc1_tile_bytes(1)) : 0;
    off[l][6] = o; o += (l == 1 || l == 2) ? align_up(n) : 0;        // FP8 for the K = 128 instruction
  }
  if (c->wmem) {
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    HIPCHECK(c, hipFree(c->wmem));
    c->wmem = nullptr;
  }
  HIPCHECK(c, hipMalloc(&c->wmem, o));
  c->wbytes = o;
  char* base = static_cast<char*>(c->wmem);
  for (int l = 0; l < 5; ++l) {
    HIPCHECK(c, hipMemcpy(base + off[l][0], W[l].data(), W[l].size() * 4, hipMemcpyHostToDevice));
    HIPCHECK(c, hipMemcpy(base + off[l][3], B[l].data(), B[l].size() * 4, hipMemcpyHostToDevice));
    c->q.w[l] = reinterpret_cast<const float*>(base + off[l][0]);
    c->q.wb[l] = reinterpret_cast<const uint16_t*>(base + off[l][1]);
    c->q.w8[l] = reinterpret_cast<const uint8_t*>(base + off[l][2]);
    c->q.b[l] = reinterpret_cast<const float*>(base + off[l][3]);
    float m = 0.f;
    for (float v : W[l]) m = std::max(m, std::fabs(v));
    c->wabs[l] = m;
    c->q.wscale[l] = m > 0.f ? 448.f / m : 1.f;
    launch_convert_bf16(c->q.w[l], const_cast<uint16_t*>(c->q.wb[l]), (long long)W[l].size(), c->stream);
    launch_convert_fp8(c->q.w[l], const_cast<uint8_t*>(c->q.w8[l]), (long long)W[l].size(), c->q.wscale[l],
                       c->stream);
    c->q.wfb[l] = c->q.wf8[l] = c->q.wf8k[l] = nullptr;
    if (l == 1 || l == 2) {
      c->q.wfb[l] = base + off[l][4];
      c->q.wf8[l] = base + off[l][5];
      c->q.wf8k[l] = base + off[l][6];
      launch_fragment_major(c->q.wb[l], const_cast<void*>(c->q.wfb[l]), NK[l][0], NK[l][1], 2, true, c->stream);
      launch_fragment_major(c->q.w8[l], const_cast<void*>(c->q.wf8[l]), NK[l][0], NK[l][1], 1, true, c->stream);
      launch_fragment_major_k128(c->q.w8[l], const_cast<void*>(c->q.wf8k[l]), NK[l][0], NK[l][1], c->stream);
    } else if (l == 3) {
      c->q.wfb[l] = base + off[l][4];
      c->q.wf8[l] = base + off[l][5];
      launch_fc1_weight_tiles(c->q.wb[l], const_cast<void*>(c->q.wfb[l]), NK[l][0], NK[l][1], 2, c->stream);
      launch_fc1_weight_tiles(c->q.w8[l], const_cast<void*>(c->q.wf8[l]), NK[l][0], NK[l][1], 1, c->stream);
    }
  }
  // activation scales until calibrated: pixels 1:1 (255 -> 256 in e4m3), others unit
  c->q.ascale[0] = 1.f;
  for (int l = 1; l < 5; ++l) c->q.ascale[l] = 1.f;
  c->fp8_calibrated = false;
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  c->qnet_set = true;
  return BCTS_OK;
}

bcts_status bcts_set_precision(bcts_ctx* c, bcts_precision prec) {
  bcts_status st = check_usable(c);
  if (st != BCTS_OK) return st;
  if ((st = refuse_if_serving(c, "bcts_set_precision")) != BCTS_OK) return st;
  if (prec != BCTS_FP32 && prec != BCTS_BF16 && prec != BCTS_FP8)
    return fail(c, BCTS_E_INVAL, "unknown precision %d", (int)prec);
  c->prec = (int)prec;
  return BCTS_OK;
}

bcts_status bcts_get_fp8_scales(bcts_ctx* c, float* out5) {
  if (!c || !out5) return BCTS_E_INVAL;
  for (int l = 0; l < 5; ++l) out5[l] = c->q.ascale[l];
  return BCTS_OK;
}

bcts_status bcts_set_fp8_scales(bcts_ctx* c, const float* in5) {
  bcts_status st = check_usable(c);
  if (st != BCTS_OK) return st;
  if ((st = refuse_if_serving(c, "bcts_set_fp8_scales")) != BCTS_OK) return st;
  if (!in5) return fail(c, BCTS_E_INVAL, "scales are NULL");
  for (int l = 0; l < 5; ++l)
    if (!(in5[l] > 0.f) || !std::isfinite(in5[l])) return fail(c, BCTS_E_INVAL, "scale %d not positive", l);
  for (int l = 0; l < 5; ++l) c->q.ascale[l] = in5[l];
  c->fp8_calibrated = true;
  return BCTS_OK;
}

bcts_status bcts_calibrate_fp8(bcts_ctx* c, int32_t n, const uint8_t* stacks) {
  bcts_status st = check_usable(c);
  if (st != BCTS_OK) return st;
  if ((st = refuse_if_serving(c, "bcts_calibrate_fp8")) != BCTS_OK) return st;
  if (n <= 0 || !stacks) return fail(c, BCTS_E_INVAL, "need n > 0 calibration stacks");
  if (!c->qnet_set) return fail(c, BCTS_E_STATE, "no Q-network set");
  HIPCHECK(c, hipSetDevice(c->device));
  std::vector<int32_t> dep(n, 0), Av(n, kMaxA);
  bcts_correction off{0, 0.f, 0};
  Plan p;
  make_plan(p, n, dep.data(), Av.data(), 1.f, off, kMaxA, n, P_FP32, true);
  const size_t maxb = p.total + 64;
  st = ensure_arena(c, maxb);
  if (st != BCTS_OK) return st;
  hipStream_t s = c->stream;
  st = upload_tables(c, p, s);
  if (st != BCTS_OK) return st;
  HIPCHECK(c, hipMemcpyAsync(c->arena + p.o_root_stack, stacks, (size_t)n * 4 * kFrameBytes,
                             hipMemcpyHostToDevice, s));
  FrameBases fb{};
  fb.level_frames[0] = reinterpret_cast<const uint8_t*>(c->arena + p.o_root_stack);
  ItemDesc* desc = reinterpret_cast<ItemDesc*>(c->arena + p.o_desc);
  launch_item_desc(0, n, reinterpret_cast<const Seg*>(c->arena + p.o_segs), (int)p.segs.size(),
                   reinterpret_cast<const RootInfo*>(c->arena + p.o_roots), fb, desc, s);
  float* ws = reinterpret_cast<float*>(c->arena + p.o_ws);
  launch_qnet(P_FP32, c->q, desc, n, ws, reinterpret_cast<float*>(c->arena + p.o_V),
              reinterpret_cast<float*>(c->arena + p.o_q0), s);
  // absmax of each layer's FP32 input: x1, x2, x3, h
  float* mx = reinterpret_cast<float*>(c->arena + p.total);
  HIPCHECK(c, hipMemsetAsync(mx, 0, 16, s));
  const long long sz[4] = {12800LL * n, 5184LL * n, 3136LL * n, 512LL * n};
  const float* src = ws;
  for (int l = 0; l < 4; ++l) {
    launch_absmax(src, sz[l], mx + l, s);
    src += sz[l];
  }
  float h[4];
  HIPCHECK(c, hipMemcpyAsync(h, mx, 16, hipMemcpyDeviceToHost, s));
  HIPCHECK(c, hipStreamSynchronize(s));
  c->q.ascale[0] = 1.f;
  for (int l = 0; l < 4; ++l) c->q.ascale[l + 1] = h[l] > 0.f ? 448.f / h[l] : 1.f;
  c->fp8_calibrated = true;
  return BCTS_OK;
}

bcts_status bcts_search(bcts_ctx* c, int32_t n, const int32_t* pos, const uint8_t* stacks, int32_t depth,
                        int32_t A, float gamma, bcts_correction corr, int32_t* out_action, float* out_q) {
  bcts_status st = check_usable(c);
  if (st != BCTS_OK) return st;
  if ((st = validate_common(c, n, gamma, corr)) != BCTS_OK) return st;
  if ((st = validate_shape(c, A, depth, corr)) != BCTS_OK) return st;
  if (!pos || !stacks || !out_action || !out_q) return fail(c, BCTS_E_INVAL, "NULL buffer");
  if ((st = validate_pos(c, n, pos)) != BCTS_OK) return st;
  HIPCHECK(c, hipSetDevice(c->device));
  std::vector<int32_t> dv(n, depth), av(n, A);
  return search_host(c, n, pos, stacks, dv.data(), av.data(), gamma, corr, out_action, out_q, A);
}

bcts_status bcts_search_batch(bcts_ctx* c, int32_t n, const int32_t* pos, const uint8_t* stacks,
                              const int32_t* depth, const int32_t* A, float gamma, bcts_correction corr,
                              int32_t* out_action, float* out_q) {
  bcts_status st = check_usable(c);
  if (st != BCTS_OK) return st;
  if ((st = validate_common(c, n, gamma, corr)) != BCTS_OK) return st;
  if (!pos || !stacks || !out_action || !out_q || !depth || !A) return fail(c, BCTS_E_INVAL, "NULL buffer");
  for (int r = 0; r < n; ++r)
    if ((st = validate_shape(c, A[r], depth[r], corr)) != BCTS_OK) return st;
  if ((st = validate_pos(c, n, pos)) != BCTS_OK) return st;
  HIPCHECK(c, hipSetDevice(c->device));
  return search_host(c, n, pos, stacks, depth, A, gamma, corr, out_action, out_q, kMaxA);
}

bcts_status bcts_search_batch_device(bcts_ctx* c, int32_t n, const int32_t* d_pos, const uint8_t* d_stacks,
                                     const int32_t* depth, const int32_t* A, float gamma, bcts_correction corr,
                                     int32_t* d_act, float* d_q, void* hip_stream) {
  bcts_status st = check_usable(c);
  if (st != BCTS_OK) return st;
  if ((st = validate_common(c, n, gamma, corr)) != BCTS_OK) return st;
  if (!d_pos || !d_stacks || !d_act || !d_q || !depth || !A) return fail(c, BCTS_E_INVAL, "NULL buffer");
  for (int r = 0; r < n; ++r)
    if ((st = validate_shape(c, A[r], depth[r], corr)) != BCTS_OK) return st;
  HIPCHECK(c, hipSetDevice(c->device));
  hipStream_t s = hip_stream ? reinterpret_cast<hipStream_t>(hip_stream) : c->stream;
  Plan p;
  plan_search(c, p, n, depth, A, gamma, corr, kMaxA, false);
  if ((st = ensure_arena(c, p.total)) != BCTS_OK) return st;
  if ((st = upload_tables(c, p, s)) != BCTS_OK) return st;
  st = enqueue_search(c, p, d_pos, d_stacks, gamma, corr.enabled ? corr.scale : 0.f, d_act, d_q, s, c->timing);
  if (st != BCTS_OK) return st;
  if ((st = arena_enqueued(c, s)) != BCTS_OK) return st;
  if (c->timing) return collect_timing(c);
  return BCTS_OK;
}

bcts_status bcts_search_batch_device_noalloc(bcts_ctx* c, int32_t n, const int32_t* d_pos,
                                             const uint8_t* d_stacks, const int32_t* depth, const int32_t* A,
                                             float gamma, bcts_correction corr, int32_t* d_act, float* d_q,
                                             void* hip_stream) {
  bcts_status st = check_usable(c);
  if (st != BCTS_OK) return st;
  if ((st = validate_common(c, n, gamma, corr)) != BCTS_OK) return st;
  if (!d_pos || !d_stacks || !d_act || !d_q || !depth || !A) return fail(c, BCTS_E_INVAL, "NULL buffer");
  for (int r = 0; r < n; ++r)
    if ((st = validate_shape(c, A[r], depth[r], corr)) != BCTS_OK) return st;
  if (!c->scratch) return fail(c, BCTS_E_HIP, "static scratch unavailable: %s", c->scratch_err.c_str());
  HIPCHECK(c, hipSetDevice(c->device));
  hipStream_t s = hip_stream ? reinterpret_cast<hipStream_t>(hip_stream) : c->stream;
  // The context's chunking, halved until the plan fits the scratch (results
  // do not depend on the chunking).
  const bool fz = c->fused && c->prec != P_FP32;
  long long chunk = fz ? c->fused_chunk_items : c->chunk_items, tail = c->chunk_items;
  Plan p;
  for (;;) {
    make_plan(p, n, depth, A, gamma, corr, kMaxA, chunk, c->prec, false, fz, c->beam, c->corr_fp32, tail);
    if (p.total <= kScratchBytes || (chunk <= 256 && tail <= 256)) break;
    chunk = std::max(256LL, chunk / 2);
    tail = std::max(256LL, tail / 2);
  }
  if (p.total > kScratchBytes)
    return fail(c, BCTS_E_NOMEM,
                "search needs %zu bytes of device memory; the static scratch of the no-allocation entry point "
                "holds %zu",
                p.total, kScratchBytes);
  // the host staging buffer is reused once its previous copy has finished
  if (c->na_copy_pending) {
    HIPCHECK(c, hipEventSynchronize(c->na_copy_ev));
    c->na_copy_pending = false;
  }
  if (c->na_tables.size() < p.table_bytes) c->na_tables.resize(p.table_bytes);
  // a search enqueued on the scratch from another stream finishes first
  if (c->na_pending && c->na_stream != s) HIPCHECK(c, hipStreamWaitEvent(s, c->na_ev, 0));
  if ((st = upload_tables_at(c, p, c->scratch, c->na_tables.data(), s)) != BCTS_OK) return st;
  HIPCHECK(c, hipEventRecord(c->na_copy_ev, s));
  c->na_copy_pending = true;
  st = enqueue_search_at(c, p, c->scratch, d_pos, d_stacks, gamma, corr.enabled ? corr.scale : 0.f, d_act, d_q, s,
                         false);
  if (st != BCTS_OK) return st;
  HIPCHECK(c, hipEventRecord(c->na_ev, s));
  c->na_stream = s;
  c->na_pending = true;
  return BCTS_OK;
}

}  // extern "C"

// A captured search: its own arena (so later calls may grow or free the
// context's), the plan's tables uploaded once, and the instantiated graph
// of the launch sequence on fixed input and output pointers.
struct bcts_graph {
  bcts_ctx* c = nullptr;
  char* arena = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  long long leaves = 0;
};

extern "C" {

bcts_status bcts_graph_create(bcts_ctx* c, int32_t n, const int32_t* d_pos, const uint8_t* d_stacks,
                              const int32_t* depth, const int32_t* A, float gamma, bcts_correction corr,
                              int32_t* d_act, float* d_q, void* hip_stream, bcts_graph** out) {
  bcts_status st = check_usable(c);
  if (st != BCTS_OK) return st;
  if (!out) return fail(c, BCTS_E_INVAL, "NULL graph handle");
  *out = nullptr;
  if ((st = validate_common(c, n, gamma, corr)) != BCTS_OK) return st;
  if (!d_pos || !d_stacks || !d_act || !d_q || !depth || !A) return fail(c, BCTS_E_INVAL, "NULL buffer");
  for (int r = 0; r < n; ++r)
    if ((st = validate_shape(c, A[r], depth[r], corr)) != BCTS_OK) return st;
  HIPCHECK(c, hipSetDevice(c->device));
  hipStream_t s = hip_stream ? reinterpret_cast<hipStream_t>(hip_stream) : c->stream;
  Plan p;
  plan_search(c, p, n, depth, A, gamma, corr, kMaxA, false);
  const size_t used = c->wbytes + c->arena_bytes;
  if (p.total + used > c->budget)
    return fail(c, BCTS_E_NOMEM, "graph needs %zu bytes of device memory; the budget leaves %zu", p.total,
                c->budget > used ? c->budget - used : 0);
  bcts_graph* g = new bcts_graph();
  g->c = c;
  for (int r = 0; r < n; ++r) {
    long long lv = 1;
    for (int k = 0; k < depth[r]; ++k) lv *= A[r];
    g->leaves += lv;
  }
  auto undo = [&](bcts_status e) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->arena) (void)hipFree(g->arena);
    delete g;
    return e;
  };
  if (hipMalloc((void**)&g->arena, p.total) != hipSuccess) {
    (void)hipGetLastError();
    g->arena = nullptr;
    return undo(fail(c, BCTS_E_NOMEM, "hipMalloc(%zu) for the graph's arena failed", p.total));
  }
  // tables: staged through host memory, copied before any replay can run
  std::vector<char> h(p.table_bytes);
  if ((st = upload_tables_at(c, p, g->arena, h.data(), s)) != BCTS_OK) return undo(st);
  if (hipStreamSynchronize(s) != hipSuccess) return undo(fail(c, BCTS_E_HIP, "table upload failed"));
  hipStream_t cap;
  if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess)
    return undo(fail(c, BCTS_E_HIP, "hipStreamCreate failed"));
  hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    st = enqueue_search_at(c, p, g->arena, d_pos, d_stacks, gamma, corr.enabled ? corr.scale : 0.f, d_act, d_q, cap,
                           false);
    const hipError_t e2 = hipStreamEndCapture(cap, &g->graph);
    if (e == hipSuccess) e = e2;
  }
  if (e == hipSuccess && st == BCTS_OK) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  (void)hipStreamDestroy(cap);
  if (st != BCTS_OK) return undo(st);
  if (e != hipSuccess) return undo(fail(c, BCTS_E_HIP, "graph capture failed: %s", hipGetErrorString(e)));
  ++c->live_graphs;
  *out = g;
  return BCTS_OK;
}

bcts_status bcts_graph_launch(bcts_graph* g, int32_t replays, void* hip_stream) {
  if (!g) return BCTS_E_INVAL;
  bcts_ctx* c = g->c;
  bcts_status st = check_usable(c);
  if (st != BCTS_OK) return st;
  if (replays < 1) return fail(c, BCTS_E_INVAL, "replays must be >= 1");
  if ((st = launch_gate(c)) != BCTS_OK) return st;
  HIPCHECK(c, hipSetDevice(c->device));
  hipStream_t s = hip_stream ? reinterpret_cast<hipStream_t>(hip_stream) : c->stream;
  for (int i = 0; i < replays; ++i) HIPCHECK(c, hipGraphLaunch(g->exec, s));
  return BCTS_OK;
}

void bcts_graph_destroy(bcts_graph* g) {
  if (!g) return;
  (void)hipSetDevice(g->c->device);
  (void)hipDeviceSynchronize();           // replays on any stream have finished
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->arena) (void)hipFree(g->arena);
  --g->c->live_graphs;
  delete g;
}

bcts_status bcts_search_batch_graph(bcts_ctx* c, int32_t n, const int32_t* d_pos, const uint8_t* d_stacks,
                                    const int32_t* depth, const int32_t* A, float gamma, bcts_correction corr,
                                    int32_t* d_act, float* d_q, int32_t replays, void* hip_stream) {
  bcts_status st = check_usable(c);
  if (st != BCTS_OK) return st;
  if (replays < 1) return fail(c, BCTS_E_INVAL, "replays must be >= 1");
  bcts_graph* g = nullptr;
  if ((st = bcts_graph_create(c, n, d_pos, d_stacks, depth, A, gamma, corr, d_act, d_q, hip_stream, &g)) != BCTS_OK)
    return st;
  hipStream_t s = hip_stream ? reinterpret_cast<hipStream_t>(hip_stream) : c->stream;
  hipError_t e = hipSuccess;
  if (c->timing) e = hipEventRecord(c->ev[0], s);
  if (e == hipSuccess) st = bcts_graph_launch(g, replays, hip_stream);
  if (st == BCTS_OK && c->timing && e == hipSuccess) e = hipEventRecord(c->ev[3], s);
  if (st == BCTS_OK && e == hipSuccess) e = hipStreamSynchronize(s);
  bcts_graph_destroy(g);
  if (st != BCTS_OK) return st;
  if (e != hipSuccess) return fail(c, BCTS_E_HIP, "graph replay failed: %s", hipGetErrorString(e));
  if (c->timing) {
    float ms = 0.f;
    HIPCHECK(c, hipEventElapsedTime(&ms, c->ev[0], c->ev[3]));
    for (double& v : c->t_ms) v = 0.0;
    c->t_ms[3] = ms / replays;
  }
  return BCTS_OK;
}

bcts_status bcts_debug_expand(bcts_ctx* c, const int32_t* pos, const uint8_t* stack, int32_t depth, int32_t A,
                              int32_t* out_pos, uint8_t* out_frames, int32_t* out_reward) {
  bcts_status st = check_usable(c);
  if (st != BCTS_OK) return st;
  bcts_correction off{0, 0.f, 0};
  if ((st = validate_common(c, 1, 0.5f, off)) != BCTS_OK) return st;
  if ((st = validate_shape(c, A, depth, off)) != BCTS_OK) return st;
  if (depth < 1) return fail(c, BCTS_E_INVAL, "debug expansion needs depth >= 1");
  if (!pos || !stack || !out_pos || !out_frames || !out_reward) return fail(c, BCTS_E_INVAL, "NULL buffer");
  if ((st = validate_pos(c, 1, pos)) != BCTS_OK) return st;
  HIPCHECK(c, hipSetDevice(c->device));
  Plan p;
  make_plan(p, 1, &depth, &A, 1.f, off, A, c->chunk_items, c->prec, true);
  if ((st = ensure_arena(c, p.total)) != BCTS_OK) return st;
  hipStream_t s = c->stream;
  if ((st = upload_tables(c, p, s)) != BCTS_OK) return st;
  HIPCHECK(c, hipMemcpyAsync(c->arena + p.o_root_pos, pos, sizeof(int32_t) * 16, hipMemcpyHostToDevice, s));
  char* Ar = c->arena;
  const RootInfo* roots = reinterpret_cast<const RootInfo*>(Ar + p.o_roots);
  for (int k = 1; k <= depth; ++k) {
    LevelRoots lr{reinterpret_cast<const int*>(Ar + p.o_lroot[k]),
                  reinterpret_cast<const long long*>(Ar + p.o_lstart[k]), (int)p.lvl_root[k].size()};
    launch_expand(k, p.lvl_count[k], lr, roots, reinterpret_cast<const int32_t*>(Ar + p.o_root_pos),
                  k > 1 ? reinterpret_cast<const uint8_t*>(Ar + p.o_pos[k - 1]) : nullptr,
                  k > 1 ? reinterpret_cast<const float*>(Ar + p.o_ret[k - 1]) : nullptr, nullptr, c->env, 1.f,
                  reinterpret_cast<uint8_t*>(Ar + p.o_pos[k]), reinterpret_cast<uint8_t*>(Ar + p.o_frames[k]),
                  reinterpret_cast<float*>(Ar + p.o_ret[k]), reinterpret_cast<uint8_t*>(Ar + p.o_rew[k]), s);
  }
  HIPCHECK(c, hipGetLastError());
  HIPCHECK(c, hipStreamSynchronize(s));
  long long at = 0;
  for (int k = 1; k <= depth; ++k) {
    const long long nk = p.lvl_count[k];
    std::vector<uint8_t> pb((size_t)nk * 16), rb((size_t)nk);
    HIPCHECK(c, hipMemcpy(pb.data(), Ar + p.o_pos[k], pb.size(), hipMemcpyDeviceToHost));
    HIPCHECK(c, hipMemcpy(rb.data(), Ar + p.o_rew[k], rb.size(), hipMemcpyDeviceToHost));
    HIPCHECK(c, hipMemcpy(out_frames + at * kFrameBytes, Ar + p.o_frames[k], (size_t)nk * kFrameBytes,
                          hipMemcpyDeviceToHost));
    for (long long i = 0; i < nk; ++i) {
      for (int q = 0; q < 16; ++q) out_pos[(at + i) * 16 + q] = pb[i * 16 + q];
      out_reward[at + i] = rb[i];
    }
    at += nk;
  }
  (void)stack;
  return BCTS_OK;
}

bcts_status bcts_debug_expand_batch(bcts_ctx* c, int32_t n, const int32_t* pos, const uint8_t* stacks,
                                    const int32_t* depth, const int32_t* A, float gamma, int64_t* level_nodes,
                                    int64_t* keep_entries, int64_t* root_levels, int32_t* out_pos,
                                    uint8_t* out_frames, int32_t* out_reward, float* out_ret, int32_t* out_keep) {
  bcts_status st = check_usable(c);
  if (st != BCTS_OK) return st;
  bcts_correction off{0, 0.f, 0};
  if ((st = validate_common(c, n, gamma, off)) != BCTS_OK) return st;
  if (!pos || !stacks || !depth || !A || !level_nodes || !keep_entries || !root_levels)
    return fail(c, BCTS_E_INVAL, "NULL buffer");
  for (int r = 0; r < n; ++r)
    if ((st = validate_shape(c, A[r], depth[r], off)) != BCTS_OK) return st;
  if ((st = validate_pos(c, n, pos)) != BCTS_OK) return st;
  Plan p;
  make_plan(p, n, depth, A, gamma, off, kMaxA, c->chunk_items, P_FP32, true, false, c->beam, false, c->chunk_items);
  for (int k = 0; k <= kMaxD; ++k) {
    level_nodes[k] = k >= 1 && k <= p.maxd ? p.lvl_count[k] : 0;
    keep_entries[k] = k >= 1 && k <= p.maxd ? p.keep_count[k] : 0;
  }
  for (int r = 0; r < n; ++r)
    for (int k = 0; k <= kMaxD; ++k) {
      int64_t* e = root_levels + ((size_t)r * (kMaxD + 1) + k) * 3;
      const bool in = k >= 1 && k <= p.roots[r].d;
      e[0] = in ? p.roots[r].base[k] : -1;
      e[1] = in ? p.roots[r].lcnt[k] : 0;
      e[2] = in ? p.roots[r].kbase[k] : -1;
    }
  if (!out_pos) return BCTS_OK;                  // sizes only
  if (!out_frames || !out_reward || !out_ret || !out_keep) return fail(c, BCTS_E_INVAL, "NULL buffer");
  HIPCHECK(c, hipSetDevice(c->device));
  if ((st = ensure_arena(c, p.total)) != BCTS_OK) return st;
  hipStream_t s = c->stream;
  if ((st = upload_tables(c, p, s)) != BCTS_OK) return st;
  HIPCHECK(c, hipMemcpyAsync(c->arena + p.o_root_pos, pos, sizeof(int32_t) * n * kSprites * 2, hipMemcpyHostToDevice,
                             s));
  for (int k = 1; k <= p.maxd; ++k)
    if ((st = enqueue_level(c, p, c->arena, k, reinterpret_cast<const int32_t*>(c->arena + p.o_root_pos), gamma, s)) !=
        BCTS_OK)
      return st;
  HIPCHECK(c, hipGetLastError());
  HIPCHECK(c, hipStreamSynchronize(s));
  long long at = 0, kat = 0;
  char* Ar = c->arena;
  for (int k = 1; k <= p.maxd; ++k) {
    const long long nk = p.lvl_count[k];
    std::vector<uint8_t> pb((size_t)nk * 16), rb((size_t)nk);
    HIPCHECK(c, hipMemcpy(pb.data(), Ar + p.o_pos[k], pb.size(), hipMemcpyDeviceToHost));
    HIPCHECK(c, hipMemcpy(rb.data(), Ar + p.o_rew[k], rb.size(), hipMemcpyDeviceToHost));
    HIPCHECK(c, hipMemcpy(out_ret + at, Ar + p.o_ret[k], sizeof(float) * (size_t)nk, hipMemcpyDeviceToHost));
    HIPCHECK(c, hipMemcpy(out_frames + at * kFrameBytes, Ar + p.o_frames[k], (size_t)nk * kFrameBytes,
                          hipMemcpyDeviceToHost));
    if (p.keep_count[k] > 0)
      HIPCHECK(c, hipMemcpy(out_keep + kat, Ar + p.o_keep[k], sizeof(int) * (size_t)p.keep_count[k],
                            hipMemcpyDeviceToHost));
    for (long long i = 0; i < nk; ++i) {
      for (int q = 0; q < 16; ++q) out_pos[(at + i) * 16 + q] = pb[i * 16 + q];
      out_reward[at + i] = rb[i];
    }
    at += nk;
    kat += p.keep_count[k];
  }
  (void)stacks;
  return BCTS_OK;
}

}  // extern "C"

namespace {
// Q-network on n host stacks; with group > 1 consecutive stacks form sibling
// groups of that size (the last one may be shorter) for the fused kernel,
// which then computes their shared channels 0..2 once per group.
bcts_status debug_qnet_impl(bcts_ctx* c, int32_t n, const uint8_t* stacks, int32_t A, int32_t group,
                            float* out_q) {
  bcts_status st = check_usable(c);
  if (st != BCTS_OK) return st;
  if (n <= 0 || !stacks || !out_q) return fail(c, BCTS_E_INVAL, "bad arguments");
  if (A < 1 || A > kMaxA) return fail(c, BCTS_E_INVAL, "A=%d outside [1,18]", A);
  if (group < 1 || group > kMaxA) return fail(c, BCTS_E_INVAL, "group=%d outside [1,18]", group);
  for (long long i = 0; i < n; ++i) {
    const long long first = i / group * group;
    if (i != first &&
        std::memcmp(stacks + (size_t)i * 4 * kFrameBytes, stacks + (size_t)first * 4 * kFrameBytes,
                    (size_t)3 * kFrameBytes) != 0)
      return fail(c, BCTS_E_INVAL, "stack %lld does not share channels 0..2 with its group's first stack", i);
  }
  if (!c->qnet_set) return fail(c, BCTS_E_STATE, "no Q-network set");
  HIPCHECK(c, hipSetDevice(c->device));
  std::vector<int32_t> dep(n, 0), Av(n, A);
  bcts_correction off{0, 0.f, 0};
  Plan p;
  plan_search(c, p, n, dep.data(), Av.data(), 1.f, off, kMaxA, true);
  if (group > 1) {
    // regroup the one-item root groups into sibling groups, chunks of whole groups
    p.groups.clear();
    for (long long i = 0; i < n; i += group) p.groups.push_back(FusedGroup{i, (int)std::min<long long>(group, n - i), 0});
    p.chunks.clear();
    long long most = 1;
    make_chunks(p, 0, (int)p.groups.size(), p.fused ? c->fused_chunk_items : c->chunk_items, p.chunks, &most);
    if (most > p.chunk)       // the workspace was laid out for chunks of p.chunk items
      return fail(c, BCTS_E_INVAL, "group of %d exceeds the chunk size of %lld stacks", group, p.chunk);
  }
  if ((st = ensure_arena(c, p.total)) != BCTS_OK) return st;
  hipStream_t s = c->stream;
  if ((st = upload_tables(c, p, s)) != BCTS_OK) return st;
  HIPCHECK(c, hipMemcpyAsync(c->arena + p.o_root_stack, stacks, (size_t)n * 4 * kFrameBytes,
                             hipMemcpyHostToDevice, s));
  FrameBases fb{};
  fb.level_frames[0] = reinterpret_cast<const uint8_t*>(c->arena + p.o_root_stack);
  float* q0 = reinterpret_cast<float*>(c->arena + p.o_q0);
  if ((st = enqueue_qnet_stage(c, p, c->arena, fb, s, nullptr)) != BCTS_OK) return st;
  HIPCHECK(c, hipGetLastError());
  std::vector<float> h((size_t)n * kMaxA);
  HIPCHECK(c, hipMemcpyAsync(h.data(), q0, h.size() * 4, hipMemcpyDeviceToHost, s));
  HIPCHECK(c, hipStreamSynchronize(s));
  for (int i = 0; i < n; ++i)
    for (int a = 0; a < A; ++a) out_q[(size_t)i * A + a] = h[(size_t)i * kMaxA + a];
  return BCTS_OK;
}
}  // namespace

extern "C" {

bcts_status bcts_debug_qnet(bcts_ctx* c, int32_t n, const uint8_t* stacks, int32_t A, float* out_q) {
  return debug_qnet_impl(c, n, stacks, A, 1, out_q);
}

bcts_status bcts_debug_qnet_siblings(bcts_ctx* c, int32_t n, const uint8_t* stacks, int32_t A, int32_t group,
                                     float* out_q) {
  return debug_qnet_impl(c, n, stacks, A, group, out_q);
}

size_t bcts_request_bytes(int32_t depth, int32_t A) {
  if (A < 1 || A > kMaxA || depth < 0 || depth > kMaxD) return 0;
  return request_bytes(depth, A);
}

bcts_status bcts_serve_config(bcts_ctx* c, int32_t max_batch, int32_t max_inflight) {
  bcts_status st = check_usable(c);
  if (st != BCTS_OK) return st;
  if (max_batch < 1 || max_inflight < 1 || max_inflight > 8)
    return fail(c, BCTS_E_INVAL, "max_batch >= 1 and 1 <= max_inflight <= 8");
  if (c->serve && (c->serve->busy() || !c->serve->live.empty()))
    return fail(c, BCTS_E_STATE, "serving is active");
  HIPCHECK(c, hipSetDevice(c->device));
  delete c->serve;
  c->serve = new ServeEngine(c);
  c->serve->max_batch = max_batch;
  c->serve->max_steps = max_inflight;
  return BCTS_OK;
}

bcts_status bcts_submit(bcts_ctx* c, const int32_t* pos, const uint8_t* stack, int32_t depth, int32_t A,
                        float gamma, bcts_correction corr, uint64_t* ticket) {
  bcts_status st = check_usable(c);
  if (st != BCTS_OK) return st;
  if ((st = validate_common(c, 1, gamma, corr)) != BCTS_OK) return st;
  if ((st = validate_shape(c, A, depth, corr)) != BCTS_OK) return st;
  if (!pos || !stack || !ticket) return fail(c, BCTS_E_INVAL, "NULL buffer");
  if ((st = validate_pos(c, 1, pos)) != BCTS_OK) return st;
  HIPCHECK(c, hipSetDevice(c->device));
  if (!c->serve) c->serve = new ServeEngine(c);
  ServeEngine& e = *c->serve;
  if ((st = e.init()) != BCTS_OK) return st;
  const size_t need = request_bytes(depth, A);
  if (need > e.pool_capacity())
    return fail(c, BCTS_E_NOMEM, "request (depth %d, A %d) needs %zu bytes; the serving pool holds %zu", depth, A,
                need, e.pool_capacity());
  ServeReq r;
  r.ticket = e.next_ticket++;
  r.A = A;
  r.d = depth;
  r.gamma = gamma;
  r.corr = corr;
  std::memcpy(r.pos, pos, sizeof r.pos);
  r.stack.assign(stack, stack + (size_t)4 * kFrameBytes);
  e.live.insert(r.ticket);
  *ticket = r.ticket;
  e.queue.push_back(std::move(r));
  return e.progress(nullptr);
}

bcts_status bcts_serve_stats(bcts_ctx* c, int64_t* out8) {
  if (!c || !out8) return BCTS_E_INVAL;
  for (int i = 0; i < 8; ++i) out8[i] = 0;
  const ServeEngine* e = c->serve;
  if (!e) return BCTS_OK;
  int64_t admitted = 0, staged = 0;
  for (const auto& k : e->active) {
    admitted += (int64_t)k.tickets.size();
    staged += k.next < k.n_stages ? 1 : 0;
  }
  out8[0] = (int64_t)e->queue.size();
  out8[1] = admitted;
  out8[2] = (int64_t)e->active.size();
  out8[3] = staged;
  out8[4] = (int64_t)e->inflight.size();
  out8[5] = (int64_t)(e->ready ? e->pool.in_use() : 0);
  out8[6] = (int64_t)e->pool_capacity();
  out8[7] = (int64_t)e->cohorts_done;
  return BCTS_OK;
}

bcts_status bcts_debug_fail_launches(bcts_ctx* c, int32_t count) {
  if (!c || count < 0) return BCTS_E_INVAL;
  c->inject_fail = count;
  return BCTS_OK;
}

bcts_status bcts_progress(bcts_ctx* c, int32_t* pending) {
  bcts_status st = check_usable(c);
  if (st != BCTS_OK) return st;
  if (!c->serve) {
    if (pending) *pending = 0;
    return BCTS_OK;
  }
  HIPCHECK(c, hipSetDevice(c->device));
  return c->serve->progress(pending);
}

bcts_status bcts_poll(bcts_ctx* c, uint64_t ticket, int32_t* action, float* q, double* t_done) {
  bcts_status st = check_usable(c);
  if (st != BCTS_OK) return st;
  if (!c->serve || !c->serve->live.count(ticket)) return fail(c, BCTS_E_STATE, "unknown ticket %llu",
                                                             (unsigned long long)ticket);
  HIPCHECK(c, hipSetDevice(c->device));
  if ((st = c->serve->progress(nullptr)) != BCTS_OK) return st;
  auto it = c->serve->results.find(ticket);
  if (it == c->serve->results.end()) return BCTS_E_BUSY;
  if (action) *action = it->second.action;
  if (q)
    for (int a = 0; a < it->second.A; ++a) q[a] = it->second.q[a];
  if (t_done) *t_done = it->second.t_done;
  c->serve->results.erase(it);
  c->serve->live.erase(ticket);
  return BCTS_OK;
}

bcts_status bcts_set_tuning(bcts_ctx* c, int32_t key, int64_t value) {
  bcts_status st = check_usable(c);
  if (st != BCTS_OK) return st;
  if ((st = refuse_if_serving(c, "bcts_set_tuning")) != BCTS_OK) return st;
  switch (key) {
    case BCTS_TUNE_FUSED:
      c->fused = value != 0;
      return BCTS_OK;
    case BCTS_TUNE_FUSED_ROUND:
      if (value < 1 || value > 4) return fail(c, BCTS_E_INVAL, "fused round must be 1..4");
      c->fused_T = (int)value;
      return BCTS_OK;
    case BCTS_TUNE_FUSED_CHUNK:
      if (value < 1 || value > (1LL << 26)) return fail(c, BCTS_E_INVAL, "fused chunk out of range");
      c->fused_chunk_items = value;
      return BCTS_OK;
    case BCTS_TUNE_LAYER_CHUNK:
      if (value < 1 || value > (1LL << 22)) return fail(c, BCTS_E_INVAL, "layer chunk out of range");
      c->chunk_items = value;
      return BCTS_OK;
    case BCTS_TUNE_FP8_K128:
      c->fp8_k128 = value != 0;
      return BCTS_OK;
    case BCTS_TUNE_MLP_CROSSOVER:
      if (value < 0 || value > kMlpMaxD) return fail(c, BCTS_E_INVAL, "cross-over depth %lld outside [0,%d]",
                                                     (long long)value, kMlpMaxD);
      c->mlp_crossover = (int)value;
      return BCTS_OK;
    case BCTS_TUNE_CORR_FP32:
      c->corr_fp32 = value != 0;
      return BCTS_OK;
    case BCTS_TUNE_FC2_FOLDED:
      c->fc2_folded = value != 0;
      return BCTS_OK;
    case BCTS_TUNE_MLP_HOST:
      if (value < 0 || value > 2) return fail(c, BCTS_E_INVAL, "host search mode must be 0, 1 or 2");
      c->mlp_host = (int)value;
      return BCTS_OK;
    case BCTS_TUNE_CONV1_GROUPS:
      if (value < 0 || value > 2) return fail(c, BCTS_E_INVAL, "conv1 grouping must be 0, 1 or 2");
      c->conv1_groups = (int)value;
      return BCTS_OK;
    default:
      return fail(c, BCTS_E_INVAL, "unknown tuning key %d", key);
  }
}

bcts_status bcts_get_tuning(bcts_ctx* c, int32_t key, int64_t* value) {
  if (!c || !value) return BCTS_E_INVAL;
  switch (key) {
    case BCTS_TUNE_FUSED: *value = c->fused ? 1 : 0; return BCTS_OK;
    case BCTS_TUNE_FUSED_ROUND: *value = c->fused_T; return BCTS_OK;
    case BCTS_TUNE_FUSED_CHUNK: *value = c->fused_chunk_items; return BCTS_OK;
    case BCTS_TUNE_LAYER_CHUNK: *value = c->chunk_items; return BCTS_OK;
    case BCTS_TUNE_CORR_FP32: *value = c->corr_fp32 ? 1 : 0; return BCTS_OK;
    case BCTS_TUNE_MLP_CROSSOVER: *value = c->mlp_crossover; return BCTS_OK;
    case BCTS_TUNE_FP8_K128: *value = c->fp8_k128 ? 1 : 0; return BCTS_OK;
    case BCTS_TUNE_CONV1_GROUPS: *value = c->conv1_groups; return BCTS_OK;
    case BCTS_TUNE_MLP_HOST: *value = c->mlp_host; return BCTS_OK;
    case BCTS_TUNE_FC2_FOLDED: *value = c->fc2_folded ? 1 : 0; return BCTS_OK;
    default: return fail(c, BCTS_E_INVAL, "unknown tuning key %d", key);
  }
}

bcts_status bcts_autotune(bcts_ctx* c, int32_t n, const int32_t* d_pos, const uint8_t* d_stacks,
                          const int32_t* depth, const int32_t* A, float gamma, bcts_correction corr,
                          void* d_scratch_action, void* d_scratch_q, int32_t reps, void* hip_stream,
                          int64_t* out_best) {
  bcts_status st = check_usable(c);
  if (st != BCTS_OK) return st;
  if ((st = refuse_if_serving(c, "bcts_autotune")) != BCTS_OK) return st;
  if (reps < 1 || !out_best) return fail(c, BCTS_E_INVAL, "reps >= 1 and out_best required");
  // candidates: fused on/off (FP32 is never fused), the FP8 matrix
  // instruction (K = 128 or 32), round T, fused chunk size
  const int Ts[5] = {1, 2, 3, 4, 5};
  const long long chunks[2] = {262144, 1048576};
  const bool was_fused = c->fused, was_timing = c->timing, was_k128 = c->fp8_k128;
  const int was_T = c->fused_T;
  const long long was_chunk = c->fused_chunk_items;
  double best_ms = 1e30;
  int64_t best[5] = {was_fused, was_T, was_chunk, 0, was_k128};
  hipStream_t s = hip_stream ? reinterpret_cast<hipStream_t>(hip_stream) : c->stream;
  hipEvent_t e0, e1;
  HIPCHECK(c, hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(c, BCTS_E_HIP, "hipEventCreate failed");
  }
  c->timing = false;
  for (int fz = (c->prec == P_FP32 ? 0 : 1); fz >= 0 && st == BCTS_OK; --fz) {
   for (int k8 = (fz && c->prec == P_FP8) ? 1 : 0; k8 >= 0 && st == BCTS_OK; --k8) {
    for (int ti = 0; ti < (fz ? 5 : 1) && st == BCTS_OK; ++ti) {
      // rounds the kernel has: BF16 1..3 (4 is over the LDS of one CU), FP8
      // with K = 32 1..4, with K = 128 3 (its weights take 68 KB of LDS)
      if (fz && c->prec == P_BF16 && Ts[ti] > 3) continue;
      if (fz && c->prec == P_FP8 && !k8 && Ts[ti] > 4) continue;
      if (fz && k8 && Ts[ti] != 3) continue;
      for (int ci = 0; ci < (fz ? 2 : 1) && st == BCTS_OK; ++ci) {
        c->fused = fz != 0;
        c->fp8_k128 = k8 != 0;
        c->fused_T = Ts[ti];
        c->fused_chunk_items = chunks[ci];
        st = bcts_search_batch_device(c, n, d_pos, d_stacks, depth, A, gamma, corr,
                                      reinterpret_cast<int32_t*>(d_scratch_action),
                                      reinterpret_cast<float*>(d_scratch_q), s);   // warm-up, allocation
        if (st == BCTS_E_NOMEM) { st = BCTS_OK; c->err.clear(); continue; }
        if (st != BCTS_OK) break;
        if (hipEventRecord(e0, s) != hipSuccess) { st = fail(c, BCTS_E_HIP, "event record failed"); break; }
        for (int r = 0; r < reps && st == BCTS_OK; ++r)
          st = bcts_search_batch_device(c, n, d_pos, d_stacks, depth, A, gamma, corr,
                                        reinterpret_cast<int32_t*>(d_scratch_action),
                                        reinterpret_cast<float*>(d_scratch_q), s);
        if (st != BCTS_OK) break;
        float ms = 0.f;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
          st = fail(c, BCTS_E_HIP, "event timing failed");
          break;
        }
        ms /= reps;
        if (ms < best_ms) {
          best_ms = ms;
          best[0] = fz;
          best[1] = Ts[ti];
          best[2] = chunks[ci];
          best[4] = k8;
        }
      }
    }
   }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->timing = was_timing;
  if (st != BCTS_OK) {
    c->fused = was_fused;
    c->fused_T = was_T;
    c->fused_chunk_items = was_chunk;
    c->fp8_k128 = was_k128;
    return st;
  }
  c->fused = best[0] != 0;
  c->fused_T = (int)best[1];
  c->fused_chunk_items = best[2];
  c->fp8_k128 = best[4] != 0;
  out_best[0] = best[0];
  out_best[1] = best[1];
  out_best[2] = best[2];
  out_best[3] = (int64_t)(best_ms * 1000.0);   // microseconds per search
  out_best[4] = best[4];
  return BCTS_OK;
}

bcts_status bcts_set_beam(bcts_ctx* c, int32_t beam) {
  bcts_status st = check_usable(c);
  if (st != BCTS_OK) return st;
  if ((st = refuse_if_serving(c, "bcts_set_beam")) != BCTS_OK) return st;
  if (beam < 0 || beam > kMaxBeam) return fail(c, BCTS_E_INVAL, "beam=%d outside [0,%d]", beam, kMaxBeam);
  c->beam = beam;
  return BCTS_OK;
}

bcts_status bcts_set_timing(bcts_ctx* c, int32_t enabled) {
  if (!c) return BCTS_E_INVAL;
  c->timing = enabled != 0;
  return BCTS_OK;
}

bcts_status bcts_get_timing(bcts_ctx* c, double* out24) {
  if (!c || !out24) return BCTS_E_INVAL;
  for (int i = 0; i < 24; ++i) out24[i] = c->t_ms[i];
  return BCTS_OK;
}

// ---- learned forward-model world (Sec. 4.1) --------------------------------

namespace {

size_t mlp_numel(int A) {
  return (size_t)100 * (100 + A) + 100 + 100 * 100 + 100 + 100 * 100 + 100 + 101 * 100 + 101 + (size_t)A * 100 + A;
}

// arena layout of one forward-model search (byte offsets)
struct MlpPlan {
  size_t states[kMlpMaxD + 1] = {0}, ret[kMlpMaxD + 1] = {0};   // levels 1..d-1 (ret also at level 1)
  size_t v1 = 0, leaf = 0, qd = 0, in_states = 0, out_act = 0, out_q = 0, total = 0;
};

bcts_status mlp_plan(bcts_ctx* c, int n, int d, bool host_io, MlpPlan& p) {
  const int A = c->mlp.A;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o += align_up(bytes); return at; };
  long long cnt = n;
  for (int k = 1; k <= d; ++k) {
    if (cnt > (1LL << 40) / A) return fail(c, BCTS_E_INVAL, "tree too large: %d roots, A=%d, depth %d", n, A, d);
    cnt *= A;
    if (k < d) p.states[k] = take(sizeof(float) * 100 * (size_t)cnt);
    if (k < d || k == 1) p.ret[k] = take(sizeof(float) * (size_t)cnt);
  }
  if (d >= 1) {
    p.v1 = take(sizeof(float) * (size_t)n * A);
    p.leaf = take(sizeof(float) * (size_t)cnt);
    p.qd = take(sizeof(float) * (size_t)n * A);
  }
  if (host_io) {
    p.in_states = take(sizeof(float) * 100 * (size_t)n);
    p.out_act = take(sizeof(int32_t) * (size_t)n);
    p.out_q = take(sizeof(float) * (size_t)n * A);
  }
  p.total = o;
  return BCTS_OK;
}

bcts_status mlp_validate(bcts_ctx* c, int n, int d, float gamma, const bcts_correction& corr) {
  if (n <= 0) return fail(c, BCTS_E_INVAL, "n_roots=%d must be positive", n);
  if (d < 0 || d > kMlpMaxD) return fail(c, BCTS_E_INVAL, "depth=%d outside [0,%d]", d, kMlpMaxD);
  if (!(gamma > 0.f && gamma <= 1.f)) return fail(c, BCTS_E_INVAL, "gamma=%g outside (0,1]", gamma);
  if (corr.enabled && !std::isfinite(corr.scale)) return fail(c, BCTS_E_INVAL, "correction scale is not finite");
  if (corr.enabled && corr.mode != BCTS_CORR_EQ6 && corr.mode != BCTS_CORR_EXACT_GEV)
    return fail(c, BCTS_E_INVAL, "unknown correction mode %d", corr.mode);
  if (!c->mlp_set) return fail(c, BCTS_E_STATE, "no forward model set (bcts_set_mlp)");
  return BCTS_OK;
}

// Enqueue one forward-model search on stream s: level by level, children of
// level k from the states of level k - 1; the leaf level writes
// return + gamma^d max Q, reduced per (root, root action); then the root
// values and the correction.
void mlp_enqueue(bcts_ctx* c, const MlpPlan& p, int n, int d, const float* states, float gamma,
                 const bcts_correction& corr, int32_t* act, float* q, hipStream_t s, int k0 = 0) {
  const int A = c->mlp.A;
  char* base = c->arena;
  auto F = [&](size_t off) { return reinterpret_cast<float*>(base + off); };
  const bool corr_on = corr.enabled && d >= 1;
  const float gamma_d = (float)std::pow((double)gamma, d);
  long long cnt = n;
  for (int k = 1; k <= d; ++k) {
    cnt *= A;
    if (k <= k0) continue;             // expanded on the host
    const float* ps = k == 1 ? states : F(p.states[k - 1]);
    const float* pret = k == 1 ? nullptr : F(p.ret[k - 1]);
    float* os = k < d ? F(p.states[k]) : nullptr;
    float* oret = (k < d || k == 1) ? F(p.ret[k]) : nullptr;
    float* ov = (k == 1 && corr_on) ? F(p.v1) : nullptr;
    float* oleaf = k == d ? F(p.leaf) : nullptr;
    launch_mlp_level(c->mlp, cnt, ps, pret, (float)std::pow((double)gamma, k - 1), os, oret, ov, oleaf, gamma_d, s);
  }
  if (d >= 1) launch_mlp_blockmax((long long)n * A, cnt / ((long long)n * A), F(p.leaf), F(p.qd), s);
  double pe = 0.0, po = 0.0;
  if (corr_on) {
    if (corr.mode == BCTS_CORR_EXACT_GEV) gev_coeffs(A, d, &pe, &po);
    else eq6_coeffs(A, d, &pe, &po);
  }
  launch_mlp_root(c->mlp, n, d, states, d >= 1 ? F(p.ret[1]) : nullptr, corr_on ? F(p.v1) : nullptr,
                  d >= 1 ? F(p.qd) : nullptr, gamma, gamma_d, (float)pe, (float)po, corr_on ? 1 : 0,
                  corr.enabled ? corr.scale : 0.f, act, q, s);
}
}  // namespace

bcts_status bcts_set_mlp(bcts_ctx* c, int32_t A, const float* blob, size_t n_floats) {
  bcts_status st = check_usable(c);
  if (st != BCTS_OK) return st;
  if (A < 2 || A > kMaxA) return fail(c, BCTS_E_INVAL, "A=%d outside [2,18]", A);
  if (!blob) return fail(c, BCTS_E_INVAL, "blob is NULL");
  if (n_floats != mlp_numel(A))
    return fail(c, BCTS_E_INVAL, "blob has %zu floats, expected %zu for A=%d", n_floats, mlp_numel(A), A);
  for (size_t i = 0; i < n_floats; ++i)
    if (!std::isfinite(blob[i])) return fail(c, BCTS_E_INVAL, "blob[%zu] is not finite", i);
  HIPCHECK(c, hipSetDevice(c->device));
  // device order: w1s [100][100], w1a [A][100], b1, w2, b2, w3, b3, wo [101][100], bo, wq [A][100], bq
  const float* l1w = blob;
  const float* rest = blob + (size_t)100 * (100 + A);   // l1.b onwards, already in device order after w1a
  std::vector<float> h;
  h.reserve(n_floats);
  for (int o = 0; o < 100; ++o)
    for (int k = 0; k < 100; ++k) h.push_back(l1w[(size_t)o * (100 + A) + k]);
  for (int a = 0; a < A; ++a)
    for (int o = 0; o < 100; ++o) h.push_back(l1w[(size_t)o * (100 + A) + 100 + a]);
  h.insert(h.end(), rest, blob + n_floats);
  if (c->mlp_mem) {
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    HIPCHECK(c, hipFree(c->mlp_mem));
    c->mlp_mem = nullptr;
    c->mlp_set = false;
  }
  HIPCHECK(c, hipMalloc(&c->mlp_mem, sizeof(float) * h.size()));
  HIPCHECK(c, hipMemcpy(c->mlp_mem, h.data(), sizeof(float) * h.size(), hipMemcpyHostToDevice));
  mlp_host_prepare(c->mlp_h, A, h.data());
  auto carve = [&](const float* d0, auto& m) {
    size_t o = 0;
    auto next = [&](size_t k) { const float* p = d0 + o; o += k; return p; };
    m.A = A;
    m.w1s = next(100 * 100);
    m.w1a = next((size_t)A * 100);
    m.b1 = next(100);
    m.w2 = next(100 * 100);
    m.b2 = next(100);
    m.w3 = next(100 * 100);
    m.b3 = next(100);
    m.wo = next(101 * 100);
    m.bo = next(101);
    m.wq = next((size_t)A * 100);
    m.bq = next(A);
  };
  MlpDev m;
  carve(static_cast<const float*>(c->mlp_mem), m);
  c->mlp = m;
  c->mlp_set = true;
  return BCTS_OK;
}

bcts_status bcts_mlp_search_device(bcts_ctx* c, int32_t n_roots, const float* d_states, int32_t depth, float gamma,
                                   bcts_correction corr, int32_t* d_out_action, float* d_out_q, void* hip_stream) {
  bcts_status st = check_usable(c);
  if (st != BCTS_OK) return st;
  if ((st = mlp_validate(c, n_roots, depth, gamma, corr)) != BCTS_OK) return st;
  if (!d_states || !d_out_action || !d_out_q) return fail(c, BCTS_E_INVAL, "NULL pointer");
  HIPCHECK(c, hipSetDevice(c->device));
  MlpPlan p;
  if ((st = mlp_plan(c, n_roots, depth, false, p)) != BCTS_OK) return st;
  if ((st = ensure_arena(c, p.total)) != BCTS_OK) return st;
  hipStream_t s = hip_stream ? static_cast<hipStream_t>(hip_stream) : c->stream;
  if ((st = order_arena(c, s)) != BCTS_OK) return st;
  mlp_enqueue(c, p, n_roots, depth, d_states, gamma, corr, d_out_action, d_out_q, s);
  HIPCHECK(c, hipGetLastError());
  return arena_enqueued(c, s);
}

bcts_status bcts_mlp_search(bcts_ctx* c, int32_t n_roots, const float* states, int32_t depth, float gamma,
                            bcts_correction corr, int32_t* out_action, float* out_q) {
  bcts_status st = check_usable(c);
  if (st != BCTS_OK) return st;
  if ((st = mlp_validate(c, n_roots, depth, gamma, corr)) != BCTS_OK) return st;
  if (!states || !out_action || !out_q) return fail(c, BCTS_E_INVAL, "NULL pointer");
  for (long long i = 0; i < (long long)n_roots * 100; ++i)
    if (!std::isfinite(states[i])) return fail(c, BCTS_E_INVAL, "state value %lld is not finite", i);
  // Mode 2 takes the host for small trees: one host node (a child's model
  // step and head) costs about 1.4 us on one core, a host-buffer search on
  // the GPU about 45 us plus 12.5 us per level (PCIe both ways, a launch per
  // level), so the host is the faster device below 32 + 9 d nodes per root.
  long long nodes = 0;
  for (long long k = 1, cnt = 1; k <= depth; ++k) nodes += (cnt *= c->mlp.A);
  if (c->mlp_host == 1 || (c->mlp_host == 2 && nodes <= 32 + 9LL * depth)) {
    // the CPU BFS: every level, the leaves, the backup and the correction on
    // the host, in the device kernels' arithmetic
    double pe = 0.0, po = 0.0;
    if (corr.enabled && depth >= 1) {
      if (corr.mode == BCTS_CORR_EXACT_GEV) gev_coeffs(c->mlp.A, depth, &pe, &po);
      else eq6_coeffs(c->mlp.A, depth, &pe, &po);
    }
    mlp_host_search(c->mlp_h, n_roots, states, depth, gamma, corr.enabled != 0, (float)pe, (float)po,
                    corr.enabled ? corr.scale : 0.f, out_action, out_q);
    return BCTS_OK;
  }
  HIPCHECK(c, hipSetDevice(c->device));
  MlpPlan p;
  if ((st = mlp_plan(c, n_roots, depth, true, p)) != BCTS_OK) return st;
  if ((st = ensure_arena(c, p.total)) != BCTS_OK) return st;
  if ((st = order_arena(c, c->stream)) != BCTS_OK) return st;
  const int A = c->mlp.A;
  HIPCHECK(c, hipMemcpyAsync(c->arena + p.in_states, states, sizeof(float) * 100 * (size_t)n_roots,
                             hipMemcpyHostToDevice, c->stream));
  // CPU-to-GPU cross-over: levels 1..k0 on the host (never the leaves, which
  // the Q-head scores on the device), their last level's states and returns
  // -- and level 1's returns and head values, which the correction reads --
  // then go to the device, which continues at level k0 + 1
  const int k0 = std::min(c->mlp_crossover, depth - 1);
  if (k0 > 0) {
    const bool corr_on = corr.enabled && depth >= 1;
    long long cnt_k0 = n_roots;
    for (int k = 1; k <= k0; ++k) cnt_k0 *= A;
    const size_t s_bytes = sizeof(float) * 100 * (size_t)cnt_k0, r_bytes = sizeof(float) * (size_t)cnt_k0;
    const size_t l1 = (size_t)n_roots * A;
    const size_t need = align_up(s_bytes) + align_up(r_bytes) + 2 * align_up(sizeof(float) * l1);
    if ((st = ensure_pinned(c, need)) != BCTS_OK) return st;
    HIPCHECK(c, hipStreamSynchronize(c->stream));      // the pinned buffer is free
    float* hs = reinterpret_cast<float*>(c->pinned);
    float* hr = reinterpret_cast<float*>(c->pinned + align_up(s_bytes));
    float* hr1 = reinterpret_cast<float*>(c->pinned + align_up(s_bytes) + align_up(r_bytes));
    float* hv1 = hr1 + align_up(sizeof(float) * l1) / sizeof(float);
    std::vector<float> ps(states, states + (size_t)n_roots * 100), pr, ns, nr;
    long long cnt = n_roots;
    for (int k = 1; k <= k0; ++k) {
      cnt *= A;
      const bool last = k == k0;
      ns.resize(last ? 0 : (size_t)cnt * 100);
      nr.resize(last ? 0 : (size_t)cnt);
      mlp_host_level(c->mlp_h, cnt, ps.data(), k == 1 ? nullptr : pr.data(),
                     (float)std::pow((double)gamma, (double)(k - 1)), last ? hs : ns.data(),
                     last ? hr : nr.data(), (k == 1 && corr_on) ? hv1 : nullptr);
      if (k == 1) std::memcpy(hr1, last ? hr : nr.data(), sizeof(float) * l1);
      ps.swap(ns);
      pr.swap(nr);
    }
    auto D = [&](size_t off) { return c->arena + off; };
    HIPCHECK(c, hipMemcpyAsync(D(p.states[k0]), hs, s_bytes, hipMemcpyHostToDevice, c->stream));
    HIPCHECK(c, hipMemcpyAsync(D(p.ret[k0]), hr, r_bytes, hipMemcpyHostToDevice, c->stream));
    if (k0 > 1) HIPCHECK(c, hipMemcpyAsync(D(p.ret[1]), hr1, sizeof(float) * l1, hipMemcpyHostToDevice, c->stream));
    if (corr_on) HIPCHECK(c, hipMemcpyAsync(D(p.v1), hv1, sizeof(float) * l1, hipMemcpyHostToDevice, c->stream));
  }
  int32_t* d_act = reinterpret_cast<int32_t*>(c->arena + p.out_act);
  float* d_q = reinterpret_cast<float*>(c->arena + p.out_q);
  mlp_enqueue(c, p, n_roots, depth, reinterpret_cast<const float*>(c->arena + p.in_states), gamma, corr, d_act, d_q,
              c->stream, k0);
  HIPCHECK(c, hipGetLastError());
  HIPCHECK(c, hipMemcpyAsync(out_action, d_act, sizeof(int32_t) * (size_t)n_roots, hipMemcpyDeviceToHost, c->stream));
  HIPCHECK(c, hipMemcpyAsync(out_q, d_q, sizeof(float) * (size_t)n_roots * A, hipMemcpyDeviceToHost, c->stream));
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  c->arena_pending = false;
  return BCTS_OK;
}

}  // extern "C"
