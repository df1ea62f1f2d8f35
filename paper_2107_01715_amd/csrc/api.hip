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
#include <mutex>
#include <string>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "../../include/bcts.h"
#include "bcts_internal.h"
#include "plan.h"

using namespace bcts;

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
  long long chunk_items = 8192;        // layer-by-layer path (FP32)
  long long fused_chunk_items = 262144; // fused path (BF16 / FP8)
  int fused_T = 3;                      // items per LDS round of the fused conv kernel
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
  int t_maxd = 0, t_chunks = 0;
  bool t_fused = false, t_tail = false;
  long long t_items = 0, t_nodes = 0;
  double t_ms[24] = {0};
  // serving
  struct ServeEngine* serve = nullptr;
  // learned forward-model world
  void* mlp_mem = nullptr;
  MlpDev mlp{};
  bool mlp_set = false;
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

// Q-network over every eval item of the plan, chunk by chunk.  With `ev`
// (6 events per chunk) the launches of each chunk are bracketed.
bcts_status enqueue_qnet_stage(bcts_ctx* c, const Plan& p, char* A, const FrameBases& fb, hipStream_t s,
                               hipEvent_t* ev) {
  const RootInfo* roots = reinterpret_cast<const RootInfo*>(A + p.o_roots);
  ItemDesc* desc = reinterpret_cast<ItemDesc*>(A + p.o_desc);
  float* V = reinterpret_cast<float*>(A + p.o_V);
  float* q0 = reinterpret_cast<float*>(A + p.o_q0);
  const int nchunks = (int)p.chunks.size();
  const FusedGroup* groups = reinterpret_cast<const FusedGroup*>(A + p.o_groups);
  for (int ci = 0; ci < nchunks; ++ci) {
    const Plan::Chunk& ch = p.chunks[ci];
    const long long cnt = ch.i1 - ch.i0;
    hipEvent_t* cev = ev ? ev + 6 * ci : nullptr;
    launch_item_desc(ch.i0, cnt, reinterpret_cast<const Seg*>(A + p.o_segs), (int)p.segs.size(), roots, fb, desc, s);
    if (!p.fused) {
      launch_qnet(c->prec, c->q, desc, cnt, A + p.o_ws, V + ch.i0, q0, s, cev);
      continue;
    }
    const QnetDev& q = c->q;
    FusedConvArgs fa{};
    fa.groups = groups + ch.g0;
    fa.item_base = ch.i0;
    fa.desc = desc;
    const bool f8 = c->prec == P_FP8;
    for (int l = 0; l < 3; ++l) {
      // conv1 in GEMM layout, conv2 / conv3 fragment-major
      fa.w[l] = l == 0 ? (f8 ? (const void*)q.w8[0] : (const void*)q.wb[0]) : (f8 ? q.wf8[l] : q.wfb[l]);
      fa.bias[l] = q.b[l];
      fa.acc_scale[l] = f8 ? 1.f / (q.ascale[l] * q.wscale[l]) : 1.f;
      fa.out_s8[l] = f8 ? q.ascale[l + 1] : 1.f;
    }
    fa.acc_scale[0] /= 255.f;
    fa.pix_s8 = f8 ? q.ascale[0] : 1.f;
    char* x3 = A + p.o_ws;
    char* h = x3 + fused_x3_bytes(p.chunk, c->prec);
    fa.x3 = x3;
    if (cev) HIPCHECK(c, hipEventRecord(cev[0], s));
    launch_conv_fused(c->prec, c->fused_T, fa, ch.g1 - ch.g0, s);
    if (cev) {
      HIPCHECK(c, hipEventRecord(cev[1], s));
      HIPCHECK(c, hipEventRecord(cev[2], s));
      HIPCHECK(c, hipEventRecord(cev[3], s));
    }
    launch_qnet_fc(c->prec, q, desc, cnt, x3, h, V + ch.i0, q0, s, cev ? cev[4] : nullptr);
    if (cev) HIPCHECK(c, hipEventRecord(cev[5], s));
  }
  // the correction's root and depth-1 evaluations in FP32 (layer kernels)
  if (ev && !p.tail_chunks.empty()) HIPCHECK(c, hipEventRecord(ev[6 * nchunks], s));
  for (const auto& tc : p.tail_chunks) {
    const long long cnt = tc.second - tc.first;
    launch_item_desc(tc.first, cnt, reinterpret_cast<const Seg*>(A + p.o_segs), (int)p.segs.size(), roots, fb, desc,
                     s);
    launch_qnet(P_FP32, c->q, desc, cnt, A + p.o_ws, V + tc.first, q0, s, nullptr);
  }
  if (ev && !p.tail_chunks.empty()) HIPCHECK(c, hipEventRecord(ev[6 * nchunks + 1], s));
  return BCTS_OK;
}

bcts_status enqueue_search_at(bcts_ctx* c, const Plan& p, char* A, const int32_t* d_pos,
                              const uint8_t* d_stacks, float gamma, float corr_scale, int32_t* d_act,
                              float* d_q, hipStream_t s, bool timed) {
  const RootInfo* roots = reinterpret_cast<const RootInfo*>(A + p.o_roots);
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
    c->t_nodes = 0;
    for (int k = 1; k <= p.maxd; ++k) c->t_nodes += p.lvl_count[k];
    HIPCHECK(c, hipEventRecord(ev[0], s));
  }
  double g = 1.0;
  for (int k = 1; k <= p.maxd; ++k) {
    LevelRoots lr{reinterpret_cast<const int*>(A + p.o_lroot[k]),
                  reinterpret_cast<const long long*>(A + p.o_lstart[k]), (int)p.lvl_root[k].size()};
    launch_expand(k, p.lvl_count[k], lr, roots, d_pos,
                  k > 1 ? reinterpret_cast<const uint8_t*>(A + p.o_pos[k - 1]) : nullptr,
                  k > 1 ? reinterpret_cast<const float*>(A + p.o_ret[k - 1]) : nullptr,
                  k > 1 && p.keep_count[k - 1] > 0 ? reinterpret_cast<const int*>(A + p.o_keep[k - 1]) : nullptr,
                  c->env, (float)g,
                  reinterpret_cast<uint8_t*>(A + p.o_pos[k]), reinterpret_cast<uint8_t*>(A + p.o_frames[k]),
                  reinterpret_cast<float*>(A + p.o_ret[k]), reinterpret_cast<uint8_t*>(A + p.o_rew[k]), s);
    if (p.keep_count[k] > 0)
      launch_prune(k, (int)p.lvl_root[k].size(), lr, roots, reinterpret_cast<const float*>(A + p.o_ret[k]),
                   reinterpret_cast<int*>(A + p.o_keep[k]), p.beam, s);
    if (timed) HIPCHECK(c, hipEventRecord(ev[k], s));
    g *= gamma;
  }
  FrameBases fb{};
  fb.level_frames[0] = d_stacks;
  for (int k = 1; k <= p.maxd; ++k) {
    fb.level_frames[k] = reinterpret_cast<const uint8_t*>(A + p.o_frames[k]);
    fb.keep[k] = p.keep_count[k] > 0 ? reinterpret_cast<const int*>(A + p.o_keep[k]) : nullptr;
  }
  float* V = reinterpret_cast<float*>(A + p.o_V);
  float* q0 = reinterpret_cast<float*>(A + p.o_q0);
  {
    bcts_status st = enqueue_qnet_stage(c, p, A, fb, s, timed ? ev + 1 + p.maxd : nullptr);
    if (st != BCTS_OK) return st;
  }
  if (timed) HIPCHECK(c, hipEventRecord(ev[3 + p.maxd + 6 * nchunks], s));
  LevelRet lr{};
  for (int k = 1; k <= p.maxd; ++k) lr.ret[k] = reinterpret_cast<const float*>(A + p.o_ret[k]);
  launch_backup_correct(p.n, roots, V, q0, lr, gamma, corr_scale, d_act, d_q, s);
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
// [18] fused kernel ran; [19] FP32 correction evaluations (ms).
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
// Serving: continuous batching with HBM-budget admission.
//
// Requests are queued on submit (inputs copied).  Up to `max_inflight`
// batches run at once, each on its own stream with its own device arena and
// pinned staging; a batch is the longest FIFO prefix of the queue that shares
// (gamma, correction), fits the slot's memory and has at most `max_batch`
// requests.  Whenever a batch completes its slot is refilled, so requests that
// arrive while others are on the GPU join the next free slot and run
// concurrently with the batches still in flight.
// ===========================================================================
struct ServeReq {
  uint64_t ticket;
  int A, d;
  float gamma;
  bcts_correction corr;
  int32_t pos[kSprites * 2];
  std::vector<uint8_t> stack;
  size_t bytes;
};

struct ServeResult {
  int action;
  int A;
  float q[kMaxA];
  double t_done;
};

struct ServeSlot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  char* arena = nullptr;
  size_t arena_bytes = 0;
  char* pinned = nullptr;
  size_t pinned_bytes = 0;
  bool busy = false;
  std::vector<uint64_t> tickets;
  std::vector<int> A;
  size_t h_act = 0, h_q = 0;   // output offsets in pinned
};

struct ServeEngine {
  bcts_ctx* c;
  int max_batch = 512, max_inflight = 2;
  long long chunk = 2048;
  size_t slot_cap = 0;
  std::deque<ServeReq> queue;
  std::vector<ServeSlot> slots;
  std::unordered_map<uint64_t, ServeResult> results;
  std::unordered_set<uint64_t> live;
  uint64_t next_ticket = 1;

  explicit ServeEngine(bcts_ctx* ctx) : c(ctx) {}
  ~ServeEngine() { release(); }

  long long chunk_items() const { return (c->fused && c->prec != P_FP32) ? 8 * chunk : chunk; }
  size_t fixed_bytes() const {
    const long long ch = chunk_items() + kMaxA;
    size_t ws = (c->fused && c->prec != P_FP32) ? fused_workspace_bytes(ch, c->prec)
                                                 : qnet_workspace_bytes(ch, c->prec);
    if (c->corr_fp32 && c->prec != P_FP32) ws = std::max(ws, qnet_workspace_bytes(chunk, P_FP32));
    return ws + sizeof(ItemDesc) * ch + 8 * kAlign;
  }

  void release() {
    for (auto& sl : slots) {
      if (sl.stream) (void)hipStreamSynchronize(sl.stream);
      if (sl.arena) (void)hipFree(sl.arena);
      if (sl.pinned) (void)hipHostFree(sl.pinned);
      if (sl.done) (void)hipEventDestroy(sl.done);
      if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    slots.clear();
  }

  void drop_all() {
    release();
    queue.clear();
    results.clear();
    live.clear();
  }

  bcts_status init() {
    if (!slots.empty()) return BCTS_OK;
    const size_t used = c->wbytes + c->arena_bytes;
    const size_t avail = c->budget > used ? c->budget - used : 0;
    slot_cap = avail / (size_t)max_inflight;
    if (slot_cap <= fixed_bytes())
      return fail(c, BCTS_E_NOMEM, "serving budget too small (%zu bytes per slot)", slot_cap);
    slots.resize(max_inflight);
    for (auto& sl : slots) {
      HIPCHECK(c, hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking));
      HIPCHECK(c, hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
    }
    return BCTS_OK;
  }

  bcts_status retire() {
    for (auto& sl : slots) {
      if (!sl.busy) continue;
      hipError_t e = hipEventQuery(sl.done);
      if (e == hipErrorNotReady) continue;
      if (e != hipSuccess) return fail(c, BCTS_E_HIP, "serving batch failed: %s", hipGetErrorString(e));
      const double t = now_s();
      const int32_t* act = reinterpret_cast<const int32_t*>(sl.pinned + sl.h_act);
      const float* q = reinterpret_cast<const float*>(sl.pinned + sl.h_q);
      for (size_t i = 0; i < sl.tickets.size(); ++i) {
        ServeResult r;
        r.action = act[i];
        r.A = sl.A[i];
        for (int a = 0; a < kMaxA; ++a) r.q[a] = q[i * kMaxA + a];
        r.t_done = t;
        if (live.count(sl.tickets[i])) results[sl.tickets[i]] = r;
      }
      sl.busy = false;
    }
    return BCTS_OK;
  }

  bcts_status launch(ServeSlot& sl) {
    // FIFO prefix sharing (gamma, correction) within the slot's memory
    const size_t cap = slot_cap - fixed_bytes();
    const ServeReq& f = queue.front();
    size_t sum = 0;
    int n = 0;
    for (const auto& r : queue) {
      if (n >= max_batch || r.gamma != f.gamma || r.corr.enabled != f.corr.enabled ||
          r.corr.scale != f.corr.scale || r.corr.mode != f.corr.mode || sum + r.bytes > cap)
        break;
      sum += r.bytes;
      ++n;
    }
    if (n == 0) return BCTS_OK;
    std::vector<int32_t> dep(n), Av(n);
    for (int i = 0; i < n; ++i) { dep[i] = queue[i].d; Av[i] = queue[i].A; }
    Plan p;
    const bool fz = c->fused && c->prec != P_FP32;
    make_plan(p, n, dep.data(), Av.data(), f.gamma, f.corr, kMaxA, chunk_items(), c->prec, true, fz, c->beam,
              c->corr_fp32, chunk);
    while (p.total > slot_cap && n > 1) {   // alignment slack: shrink the batch
      --n;
      make_plan(p, n, dep.data(), Av.data(), f.gamma, f.corr, kMaxA, chunk_items(), c->prec, true, fz, c->beam,
                c->corr_fp32, chunk);
    }
    if (p.total > slot_cap) return fail(c, BCTS_E_NOMEM, "request does not fit a serving slot");
    if (sl.arena_bytes < slot_cap) {
      if (sl.arena) HIPCHECK(c, hipFree(sl.arena));
      sl.arena = nullptr;
      sl.arena_bytes = 0;
      HIPCHECK(c, hipMalloc((void**)&sl.arena, slot_cap));
      sl.arena_bytes = slot_cap;
    }
    const size_t in_pos = align_up(p.table_bytes), in_stack = in_pos + align_up(sizeof(int32_t) * n * 16);
    sl.h_act = in_stack + align_up((size_t)n * 4 * kFrameBytes);
    sl.h_q = sl.h_act + align_up(sizeof(int32_t) * n);
    const size_t need = sl.h_q + align_up(sizeof(float) * (size_t)n * kMaxA);
    if (sl.pinned_bytes < need) {
      if (sl.pinned) HIPCHECK(c, hipHostFree(sl.pinned));
      sl.pinned = nullptr;
      sl.pinned_bytes = 0;
      const size_t nb = std::max(need * 2, (size_t)1 << 20);
      HIPCHECK(c, hipHostMalloc((void**)&sl.pinned, nb, hipHostMallocDefault));
      sl.pinned_bytes = nb;
    }
    bcts_status st = upload_tables_at(c, p, sl.arena, sl.pinned, sl.stream);
    if (st != BCTS_OK) return st;
    int32_t* hp = reinterpret_cast<int32_t*>(sl.pinned + in_pos);
    uint8_t* hs = reinterpret_cast<uint8_t*>(sl.pinned + in_stack);
    sl.tickets.resize(n);
    sl.A.resize(n);
    for (int i = 0; i < n; ++i) {
      const ServeReq& r = queue[i];
      std::memcpy(hp + i * 16, r.pos, sizeof r.pos);
      std::memcpy(hs + (size_t)i * 4 * kFrameBytes, r.stack.data(), (size_t)4 * kFrameBytes);
      sl.tickets[i] = r.ticket;
      sl.A[i] = r.A;
    }
    HIPCHECK(c, hipMemcpyAsync(sl.arena + p.o_root_pos, hp, sizeof(int32_t) * n * 16, hipMemcpyHostToDevice,
                               sl.stream));
    HIPCHECK(c, hipMemcpyAsync(sl.arena + p.o_root_stack, hs, (size_t)n * 4 * kFrameBytes,
                               hipMemcpyHostToDevice, sl.stream));
    int32_t* d_act = reinterpret_cast<int32_t*>(sl.arena + p.o_act);
    float* d_q = reinterpret_cast<float*>(sl.arena + p.o_q);
    st = enqueue_search_at(c, p, sl.arena, reinterpret_cast<const int32_t*>(sl.arena + p.o_root_pos),
                           reinterpret_cast<const uint8_t*>(sl.arena + p.o_root_stack), f.gamma,
                           f.corr.enabled ? f.corr.scale : 0.f, d_act, d_q, sl.stream, false);
    if (st != BCTS_OK) return st;
    HIPCHECK(c, hipMemcpyAsync(sl.pinned + sl.h_act, d_act, sizeof(int32_t) * n, hipMemcpyDeviceToHost,
                               sl.stream));
    HIPCHECK(c, hipMemcpyAsync(sl.pinned + sl.h_q, d_q, sizeof(float) * (size_t)n * kMaxA,
                               hipMemcpyDeviceToHost, sl.stream));
    HIPCHECK(c, hipEventRecord(sl.done, sl.stream));
    sl.busy = true;
    for (int i = 0; i < n; ++i) queue.pop_front();
    return BCTS_OK;
  }

  bcts_status progress(int* pending) {
    bcts_status st = init();
    if (st != BCTS_OK) return st;
    if ((st = retire()) != BCTS_OK) return st;
    for (auto& sl : slots) {
      if (queue.empty()) break;
      if (sl.busy) continue;
      if ((st = launch(sl)) != BCTS_OK) return st;
    }
    if (pending) {
      int busy = 0;
      for (auto& sl : slots) busy += sl.busy ? (int)sl.tickets.size() : 0;
      *pending = (int)queue.size() + busy;
    }
    return BCTS_OK;
  }
};

// Serving work that reads the context's model, tables and settings: queued
// requests and batches in flight (finished results waiting for bcts_poll do
// not count).  The calls that change that state refuse while it exists.
static bcts_status refuse_if_serving(bcts_ctx* c, const char* what) {
  if (!c->serve) return BCTS_OK;
  bcts_status st = c->serve->retire();
  if (st != BCTS_OK) return st;
  bool busy = !c->serve->queue.empty();
  for (const auto& sl : c->serve->slots) busy = busy || sl.busy;
  if (busy) return fail(c, BCTS_E_STATE, "%s: serving requests are queued or in flight", what);
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
  size_t off[5][6], o = 0;
  for (int l = 0; l < 5; ++l) {
    const size_t n = W[l].size();
    off[l][0] = o; o += align_up(n * 4);
    off[l][1] = o; o += align_up(n * 2);
    off[l][2] = o; o += align_up(n);
    off[l][3] = o; o += align_up(B[l].size() * 4);
    const size_t fc1_tiles = (size_t)(NK[3][0] / kFc1Rows);
    off[l][4] = o; o += (l == 1 || l == 2) ? align_up(n * 2) : l == 3 ? align_up(fc1_tiles * fc1_tile_bytes(2)) : 0;
    off[l][5] = o; o += (l == 1 || l == 2) ? align_up(n) : l == 3 ? align_up(fc1_tiles * fc1_tile_bytes(1)) : 0;
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
    c->q.wfb[l] = c->q.wf8[l] = nullptr;
    if (l == 1 || l == 2) {
      c->q.wfb[l] = base + off[l][4];
      c->q.wf8[l] = base + off[l][5];
      launch_fragment_major(c->q.wb[l], const_cast<void*>(c->q.wfb[l]), NK[l][0], NK[l][1], 2, true, c->stream);
      launch_fragment_major(c->q.w8[l], const_cast<void*>(c->q.wf8[l]), NK[l][0], NK[l][1], 1, true, c->stream);
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

bcts_status bcts_search_batch_graph(bcts_ctx* c, int32_t n, const int32_t* d_pos, const uint8_t* d_stacks,
                                    const int32_t* depth, const int32_t* A, float gamma, bcts_correction corr,
                                    int32_t* d_act, float* d_q, int32_t replays, void* hip_stream) {
  bcts_status st = check_usable(c);
  if (st != BCTS_OK) return st;
  if ((st = validate_common(c, n, gamma, corr)) != BCTS_OK) return st;
  if (!d_pos || !d_stacks || !d_act || !d_q || !depth || !A) return fail(c, BCTS_E_INVAL, "NULL buffer");
  if (replays < 1) return fail(c, BCTS_E_INVAL, "replays must be >= 1");
  for (int r = 0; r < n; ++r)
    if ((st = validate_shape(c, A[r], depth[r], corr)) != BCTS_OK) return st;
  HIPCHECK(c, hipSetDevice(c->device));
  hipStream_t s = hip_stream ? reinterpret_cast<hipStream_t>(hip_stream) : c->stream;
  Plan p;
  plan_search(c, p, n, depth, A, gamma, corr, kMaxA, false);
  if ((st = ensure_arena(c, p.total)) != BCTS_OK) return st;
  if ((st = upload_tables(c, p, s)) != BCTS_OK) return st;
  HIPCHECK(c, hipStreamSynchronize(s));
  c->arena_pending = false;
  hipStream_t cap;
  HIPCHECK(c, hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    st = enqueue_search(c, p, d_pos, d_stacks, gamma, corr.enabled ? corr.scale : 0.f, d_act, d_q, cap, false);
    hipError_t e2 = hipStreamEndCapture(cap, &graph);
    if (st == BCTS_OK && e2 != hipSuccess) e = e2;
  }
  if (e == hipSuccess && st == BCTS_OK) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e == hipSuccess && st == BCTS_OK) {
    if (c->timing) e = hipEventRecord(c->ev[0], s);
    for (int i = 0; i < replays && e == hipSuccess; ++i) e = hipGraphLaunch(exec, s);
    if (c->timing && e == hipSuccess) e = hipEventRecord(c->ev[3], s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  }
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  (void)hipStreamDestroy(cap);
  if (st != BCTS_OK) return st;
  if (e != hipSuccess) return fail(c, BCTS_E_HIP, "graph capture/replay failed: %s", hipGetErrorString(e));
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
  if (group > 1 && p.fused) {
    // regroup the one-item root groups into sibling groups, chunks of whole groups
    p.groups.clear();
    for (long long i = 0; i < n; i += group) p.groups.push_back(FusedGroup{i, (int)std::min<long long>(group, n - i), 0});
    const long long target = std::max(1LL, c->fused_chunk_items);
    p.chunks.clear();
    int g = 0;
    while (g < (int)p.groups.size()) {
      Plan::Chunk ch;
      ch.g0 = g;
      ch.i0 = p.groups[g].item0;
      long long items = 0;
      while (g < (int)p.groups.size() && (items == 0 || items + p.groups[g].count <= target)) {
        items += p.groups[g].count;
        ++g;
      }
      ch.g1 = g;
      ch.i1 = ch.i0 + items;
      p.chunks.push_back(ch);
    }
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
  if (c->serve && (!c->serve->queue.empty() || !c->serve->live.empty()))
    return fail(c, BCTS_E_STATE, "serving is active");
  delete c->serve;
  c->serve = new ServeEngine(c);
  c->serve->max_batch = max_batch;
  c->serve->max_inflight = max_inflight;
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
  ServeReq r;
  r.bytes = request_bytes(depth, A);
  if (r.bytes > e.slot_cap - e.fixed_bytes())
    return fail(c, BCTS_E_NOMEM, "request (depth %d, A %d) needs %zu bytes; a serving slot holds %zu", depth, A,
                r.bytes, e.slot_cap - e.fixed_bytes());
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
    case BCTS_TUNE_CORR_FP32:
      c->corr_fp32 = value != 0;
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
  // candidates: fused on/off (FP32 is never fused), round T, fused chunk size
  const int Ts[4] = {1, 2, 3, 4};
  const long long chunks[2] = {262144, 1048576};
  const bool was_fused = c->fused, was_timing = c->timing;
  const int was_T = c->fused_T;
  const long long was_chunk = c->fused_chunk_items;
  double best_ms = 1e30;
  int64_t best[4] = {was_fused, was_T, was_chunk, 0};
  hipStream_t s = hip_stream ? reinterpret_cast<hipStream_t>(hip_stream) : c->stream;
  hipEvent_t e0, e1;
  HIPCHECK(c, hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(c, BCTS_E_HIP, "hipEventCreate failed");
  }
  c->timing = false;
  for (int fz = (c->prec == P_FP32 ? 0 : 1); fz >= 0 && st == BCTS_OK; --fz) {
    for (int ti = 0; ti < (fz ? 4 : 1) && st == BCTS_OK; ++ti) {
      if (fz && c->prec == P_BF16 && Ts[ti] == 4) continue;   // over the LDS of one CU
      for (int ci = 0; ci < (fz ? 2 : 1) && st == BCTS_OK; ++ci) {
        c->fused = fz != 0;
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
    return st;
  }
  c->fused = best[0] != 0;
  c->fused_T = (int)best[1];
  c->fused_chunk_items = best[2];
  out_best[0] = best[0];
  out_best[1] = best[1];
  out_best[2] = best[2];
  out_best[3] = (int64_t)(best_ms * 1000.0);   // microseconds per search
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
constexpr int kMlpMaxD = 16;

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
                 const bcts_correction& corr, int32_t* act, float* q, hipStream_t s) {
  const int A = c->mlp.A;
  char* base = c->arena;
  auto F = [&](size_t off) { return reinterpret_cast<float*>(base + off); };
  const bool corr_on = corr.enabled && d >= 1;
  const float gamma_d = (float)std::pow((double)gamma, d);
  long long cnt = n;
  for (int k = 1; k <= d; ++k) {
    cnt *= A;
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
  const float* d0 = static_cast<const float*>(c->mlp_mem);
  size_t o = 0;
  auto next = [&](size_t k) { const float* p = d0 + o; o += k; return p; };
  MlpDev m;
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
  HIPCHECK(c, hipSetDevice(c->device));
  MlpPlan p;
  if ((st = mlp_plan(c, n_roots, depth, true, p)) != BCTS_OK) return st;
  if ((st = ensure_arena(c, p.total)) != BCTS_OK) return st;
  if ((st = order_arena(c, c->stream)) != BCTS_OK) return st;
  const int A = c->mlp.A;
  HIPCHECK(c, hipMemcpyAsync(c->arena + p.in_states, states, sizeof(float) * 100 * (size_t)n_roots,
                             hipMemcpyHostToDevice, c->stream));
  int32_t* d_act = reinterpret_cast<int32_t*>(c->arena + p.out_act);
  float* d_q = reinterpret_cast<float*>(c->arena + p.out_q);
  mlp_enqueue(c, p, n_roots, depth, reinterpret_cast<const float*>(c->arena + p.in_states), gamma, corr, d_act, d_q,
              c->stream);
  HIPCHECK(c, hipGetLastError());
  HIPCHECK(c, hipMemcpyAsync(out_action, d_act, sizeof(int32_t) * (size_t)n_roots, hipMemcpyDeviceToHost, c->stream));
  HIPCHECK(c, hipMemcpyAsync(out_q, d_q, sizeof(float) * (size_t)n_roots * A, hipMemcpyDeviceToHost, c->stream));
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  c->arena_pending = false;
  return BCTS_OK;
}

}  // extern "C"
