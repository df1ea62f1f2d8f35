// Data layout shared by the host planner and the kernels of libbcts: sizes,
// the per-root and per-item descriptors the planner writes and the kernels
// read, and fc1's tiled operand layout.  No HIP types: the planner builds
// without the HIP toolchain (its host tests do).
#pragma once
#include <stdint.h>

#ifdef __HIPCC__
#define BCTS_HD __host__ __device__
#else
#define BCTS_HD
#endif

namespace bcts {

constexpr int kFrame = 84;
constexpr int kMaxBeam = 256;           // largest beam of the pruned search
constexpr int kFrameBytes = 84 * 84;
constexpr int kSprites = 8;
constexpr int kMaxA = 18;
constexpr int kMaxD = 6;

// fc1's operands (its input x3 [rows][3136] and its weights [512][3136], in
// the operand type of eb bytes per element) are stored in stage-major tiles:
// rows in tiles of 256, and in a tile each 64-byte K slice of all 256 rows is
// one contiguous 16 KB block, the block fc1 streams per stage.  Byte kb of
// row r lives at fc1_tiled_offset(r, kb, eb).  Row counts are padded to a
// multiple of 256 (fc1 reads the padding rows and stores nothing for them).
constexpr int kFc1Rows = 256;
constexpr int kFc1K = 3136;
constexpr int kFc1StageBytes = kFc1Rows * 64;
BCTS_HD inline long long fc1_tile_bytes(int eb) { return (long long)(kFc1K * eb / 64) * kFc1StageBytes; }
BCTS_HD inline long long fc1_tiled_offset(long long r, int kb, int eb) {
  return (r / kFc1Rows) * fc1_tile_bytes(eb) + (long long)(kb >> 6) * kFc1StageBytes + (r % kFc1Rows) * 64 + (kb & 63);
}
inline long long fc1_padded_rows(long long n) { return (n + kFc1Rows - 1) / kFc1Rows * kFc1Rows; }

// K slices of the FP32 fc1 (its 98 K stages of 32 split evenly).
constexpr int kFc1Split = 7;

// Precisions (mirrors bcts_precision).
enum Prec { P_FP32 = 0, P_BF16 = 1, P_FP8 = 2 };

// Per-root descriptor (device resident).
struct RootInfo {
  int A, d;
  float gamma_d;          // gamma^d
  float pen_e, pen_o;     // penalty B = pen_e * d_e - pen_o * d_o
  int corr;               // correction applied (d >= 1 and enabled)
  int q_stride;           // output row stride of out_q
  int pad_;
  long long base[kMaxD + 1];   // first node of this root at level k (k >= 1)
  long long lcnt[kMaxD + 1];   // nodes of this root at level k (A^k unless a beam cuts earlier levels)
  long long kbase[kMaxD + 1];  // level k cut by the beam: first entry of this root's keep list, else -1
  long long leaf_blk;          // leaves per root action (A^(d-1) unless cut)
  long long leaf_item;         // first leaf eval item (d >= 1), else -1
  long long d1_item;           // first depth-1 eval item (corr and d >= 2, or d = 1 with FP32 correction evals), else -1
  long long root_item;         // root eval item, else -1
};

// A run of eval items that belong to one root and one level.
struct Seg {
  long long item0;
  int root, level, A, kind;    // kind: 0 leaf, 1 depth-1, 2 root
};

struct EnvTables {
  int delta[kMaxA][2];
  int vel[kSprites - 1][2];
};

// Per-item Q-network input/outputs for one chunk of eval items.
struct ItemDesc {
  const uint8_t* frame[4];     // the 4 stack frames, channel 0 oldest
  int A;                       // valid Q outputs
  int q0_root;                 // root id whose q0 row this item fills, or -1
};

// A sibling group: consecutive eval items whose stacks share channels 0..2
// (the A children of one node, the A depth-1 nodes of a root, or one root).
struct FusedGroup {
  long long item0;             // first item (plan-global index)
  int count;
  int pad_;
};

}  // namespace bcts
