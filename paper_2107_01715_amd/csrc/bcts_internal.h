// Internal declarations shared by the translation units of libbcts.
// Device data layout (all per search batch, in the context's HBM arena):
//
//   root_pos    int32 [n][8][2]            root positions (x, y)
//   root_stack  uint8 [n][4][7056]         root frame stacks, channel 0 oldest
//   level k = 1..maxd (nodes of every root with depth >= k, root-major,
//   inside a root in the index order of Alg. 1: child a of node j is j*A + a)
//     pos_k     uint8 [N_k][16]            (x0, y0, x1, y1, ...) after the move
//     frame_k   uint8 [N_k][7056]          the frame rendered at that node
//     ret_k     float [N_k]                sum_{t<k} gamma^t r_t along the path
//     rew_k     uint8 [N_k]                the reward of the step into the node
//   eval items (the nodes whose stack goes through the Q-network), grouped in
//   segments of one (root, level): leaves, depth-1 nodes, roots
//     V         float [n_items]            max_{a<A} Q(s, a)
//     q0        float [n][18]              Q(s_0, .) of root evaluations
//
// A node's 4-frame stack is never materialised: channel c of a level-m node
// is the frame of its ancestor at level m-3+c (the root's stack for levels
// <= 0).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "layout.h"

namespace bcts {

// One level's participating roots, sorted by first node.
struct LevelRoots {
  const int* root;             // [cnt]
  const long long* start;      // [cnt] first node index of that root at this level
  int cnt;
};

// Where frames live: level k >= 1 at level_frames[k] (node-major, 7056 B
// each); level_frames[0] is the root stack array [n][4][7056].
struct FrameBases {
  const uint8_t* level_frames[kMaxD + 1];
  const int* keep[kMaxD + 1];  // keep lists of cut levels (root-local node indices)
};

// Parent of root-local node j at level k >= 2: node j / A of level k - 1
// counted among that level's kept nodes (the keep list maps it back to a
// root-local index when the level was cut).
__device__ __forceinline__ long long parent_local(const RootInfo& ri, const int* const* keep, int k, long long j) {
  const long long i = j / ri.A;
  return ri.kbase[k - 1] >= 0 ? (long long)keep[k - 1][ri.kbase[k - 1] + i] : i;
}

// Arguments of the fused conv1->conv2->conv3 kernel (BF16 / FP8).
struct FusedConvArgs {
  const FusedGroup* groups;    // groups of this chunk
  int n_groups;                // groups in the chunk (the kernel loops over them)
  long long item_base;         // plan-global index of desc[0]
  const ItemDesc* desc;        // chunk-relative item descriptors
  const void* w[3];            // conv weights in operand type: conv1 [N][K], conv2/conv3 fragment-major
  const float* bias[3];
  float acc_scale[3];          // accumulator scale (1/255 on conv1; fp8 operand scales)
  float out_s8[3];             // fp8: input scale of the next layer
  float pix_s8;                // fp8: pixel scale
  void* x3;                    // out: [chunk items][49][64] channels-last, in fc1's stage-major tiles
};
// k8: FP8 conv2 / conv3 on the K = 128 instruction (weights in wf8k).
void launch_conv_fused(int prec, int T, const FusedConvArgs& a, int n_groups, hipStream_t s, bool k8 = false);

// Device weights in GEMM layout W[N][K] for every precision.  K orders:
// conv1 (c, kh, kw); conv2, conv3 (kh, kw, c); fc1 (h, w, c); fc2 (k).
struct QnetDev {
  const float* w[5];           // fp32
  const uint16_t* wb[5];       // bf16 bits
  const uint8_t* w8[5];        // e4m3 bytes (weights scaled by wscale)
  const float* b[5];           // biases, fp32
  float wscale[5];             // fp8 weight scale: w8 = e4m3(w * wscale)
  float ascale[5];             // fp8 input scale of each layer: x8 = e4m3(x * ascale)
  // conv2 / conv3 (index 1, 2) in fragment-major order for the fused kernel:
  // unit (cf, s, lane) = the 8 operand elements W[16cf + lane%16][32s + 8(lane/16) ..]
  // (rows paired, see launch_fragment_major);
  // fc1 (index 3) in stage-major tiles for fc1_kernel
  const void* wfb[5];          // bf16
  const void* wf8[5];          // e4m3
  const void* wf8k[5];         // e4m3, conv2 / conv3 for the K = 128 instruction (launch_fragment_major_k128)
};

// Learned forward-model world: weights on the device, FP32, [out][in] rows of
// 100 inputs.  l1's state part and its one-hot action columns are split so
// that an action adds one column: w1a[a][o] = l1.w[o][100 + a].
struct MlpDev {
  int A;
  const float *w1s, *w1a, *b1, *w2, *b2, *w3, *b3, *wo, *bo, *wq, *bq;
};
void launch_mlp_level(const MlpDev& m, long long n, const float* ps, const float* pret, float gpow, float* os,
                      float* oret, float* ov, float* oleaf, float gamma_d, hipStream_t s);
void launch_mlp_blockmax(long long n_blocks, long long block, const float* leaf, float* qd, hipStream_t s);
void launch_mlp_root(const MlpDev& m, int n, int d, const float* states, const float* ret1, const float* v1,
                     const float* qd, float gamma, float gamma_d, float pen_e, float pen_o, int corr, float scale,
                     int32_t* act, float* q, hipStream_t s);

// Copies W[N][K] (element size eb bytes) into fragment-major order; with
// pair8 (conv2, conv3: N = 64) the rows of channel fragments 2h, 2h + 1 are
// interleaved in groups of 4 so each lane group's results are 8 consecutive
// channels.
void launch_fragment_major(const void* src, void* dst, int N, int K, int eb, bool pair8, hipStream_t s);
// The FP8 copy for the K = 128 instruction: per channel fragment, 32 bytes
// (K 128s + 32(lane/16) .. +31) per lane and step, then 8-byte units for the
// K % 128 remainder; rows paired as above.
void launch_fragment_major_k128(const void* src, void* dst, int N, int K, hipStream_t s);

// Copies fc1's W[N][K] (N a multiple of 256, eb bytes per element) into
// stage-major tiles.
void launch_fc1_weight_tiles(const void* src, void* dst, int N, int K, int eb, hipStream_t s);

// fc1 as a 256 x 256-tiled MFMA GEMM (BF16 / FP8): h = ReLU(acc_scale *
// x3 W^T + b) in the operand type (FP8 outputs scaled by out_s8); x3 and w
// in stage-major tiles (x3 padded to a multiple of 256 rows), h [n][512].
void launch_fc1_mfma(int prec, long long n, const void* x3, const void* w, const float* bias, float acc_scale,
                     float out_s8, void* h, hipStream_t s);

// fc1 with fc2 folded into its epilogue (BF16 / FP8; w2 [32][512] in the
// operand type, bias b2, accumulator scale scale2): fc2 takes the fc1
// outputs rounded to the operand type, as launch_fc1_mfma stores them; each
// fc1 workgroup sums fc2 over its 256 neurons into part [2][n][32] FP32 (256
// bytes per stack, device memory the caller owns), then a second kernel adds
// the two halves in order and writes V[item] = max over the item's A actions
// and the q0 rows of root items.  The sum over the 512 neurons is associated
// as (0..127 + 128..255) + (256..383 + 384..511).  With ev_after_fc1 an event
// is recorded between the two launches.
void launch_fc12(int prec, long long n, const void* x3, const void* w1, const float* b1, float scale1, float out_s8,
                 const void* w2, float* part, hipStream_t s, hipEvent_t ev_after_fc1, const float* b2, float scale2,
                 const ItemDesc* desc, float* V, float* q0);

// fc1 (+ReLU) and fc2 (+max over A, root rows of Q_0) over a chunk whose
// conv3 output x3 is ready (BF16 / FP8, from the fused kernel, in fc1's
// stage-major tiles).  `h` is [n][512] in the operand type: fc1's output
// when fc2 reads it back (fc2_folded false), the room for launch_fc12's
// partial sums otherwise.  The two forms differ only in how fc2's sum is
// associated.
void launch_qnet_fc(int prec, const QnetDev& q, const ItemDesc* desc, long long n_items,
                    const void* x3, void* h, float* V, float* q0, hipStream_t s,
                    hipEvent_t ev_after_fc1, bool fc2_folded);

// ---- launchers (each in the TU that defines its kernels) ----------------
void launch_expand(int k, long long n_nodes, LevelRoots lr, const RootInfo* roots,
                   const int* root_pos, const uint8_t* prev_pos, const float* prev_ret, const int* prev_keep,
                   const EnvTables& env, float gamma_pow, uint8_t* pos, uint8_t* frames,
                   float* ret, uint8_t* rew, hipStream_t s);

// Beam cut of level k: for every root whose level k is cut and every root
// action a0, the `beam` nodes of a0's block with the largest return (lowest
// index on ties) go, ascending, to keep[kbase + a0 * beam ..].
void launch_prune(int k, int n_level_roots, LevelRoots lr, const RootInfo* roots, const float* ret_k, int* keep_k,
                  int beam, hipStream_t s);

void launch_item_desc(long long item_begin, long long n_items, const Seg* segs, int nsegs,
                      const RootInfo* roots, const FrameBases& fb, ItemDesc* out,
                      hipStream_t s);

// Q-network over a chunk of items (descs already built): writes V[item] and
// q0 rows.  `ws` is a workspace of qnet_workspace_bytes(chunk, prec) bytes.
// With `ev` (6 events) the launches are bracketed: ev[0] before conv1,
// ev[l+1] after layer l.
void launch_qnet(int prec, const QnetDev& q, const ItemDesc* desc, long long n_items,
                 void* ws, float* V, float* q0, hipStream_t s, hipEvent_t* ev = nullptr);

struct LevelRet {
  const float* ret[kMaxD + 1];   // ret_k per level (index 0 unused)
};
void launch_backup_correct(int n_roots, const RootInfo* roots, const float* V, const float* q0,
                           const LevelRet& level_ret, float gamma, float corr_scale,
                           int* out_action, float* out_q, hipStream_t s);

// fp32 -> bf16 / e4m3 conversion of weight arrays on the device
void launch_convert_bf16(const float* src, uint16_t* dst, long long n, hipStream_t s);
void launch_convert_fp8(const float* src, uint8_t* dst, long long n, float scale, hipStream_t s);
void launch_absmax(const float* src, long long n, float* out, hipStream_t s);

}  // namespace bcts
