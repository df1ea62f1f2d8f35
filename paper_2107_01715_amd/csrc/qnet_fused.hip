// Fused convolution stack of the Nature-DQN (conv1 -> conv2 -> conv3) for
// BF16 / FP8 operands on the CDNA4 matrix cores.  Work comes in sibling
// groups of eval items; the kernel is persistent: one workgroup per resident
// slot loops over groups b, b + gridDim.x, ...
//
// Siblings (the A children of one node, or the A depth-1 nodes of a root)
// share stack channels 0..2: a child's stack is its parent's last three
// frames plus its own.  conv1 is linear in the input channels, so its
// pre-activation splits into
//     S = sum_{c<3} W1_c * frame_c   (identical for the whole group)
//       + W1_3 * frame_3             (per item)
// S is computed once per group and kept in registers; each item then adds
// only its own channel (a quarter of conv1's K).
//
// Data path of a workgroup (8 wavefronts):
//   * a frame is read from HBM once, converted to the operand type once and
//     staged in LDS; the next round's frames (in a group's last round, the
//     next group's) load into registers during conv2/conv3 and are staged at
//     the end of the round;
//   * conv1 -> x1 (20x20x32) and conv2 -> x2 (9x9x64) of T items at a time
//     stay in LDS (layouts below);
//   * conv3 -> x3 (7x7x64, channels-last) goes to HBM for fc1, in fc1's
//     stage-major tiles (a 4- or 8-byte store stays inside one 64-byte slice).
// Every layer is an implicit GEMM computed transposed, D[channel][pixel] =
// W[channel][k] * X[k][pixel], with 16x16x32 MFMAs (BF16 or OCP e4m3, FP32
// accumulate): the weights are the A operand and the im2col pixels the B
// operand, so each lane ends with 4 consecutive channels of one pixel per
// channel fragment.  The weight rows of every layer are paired (conv1 at its
// loads, conv2 / conv3 in launch_fragment_major) so that a lane's two channel
// fragments hold 8 consecutive channels, stored with one 16-byte (BF16) or
// 8-byte (FP8) write; the pixel strides of x1 (5 x 16 bytes, its x phases
// 8000 bytes apart) and x2 (9 x 16 bytes) keep any 8 consecutive lanes of
// such a write on distinct LDS bank groups.  A wavefront owns
// a set of 16-pixel fragments and, in conv2 / conv3, half the channel
// fragments (in conv1 both halves).  The sum order of every output element
// is fixed by the layer, never by the group size, round size or chunking, so
// results do not depend on batching.
#include "bcts_internal.h"

#include <atomic>

namespace bcts {
namespace {

typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(8))) int v8i;
typedef __attribute__((ext_vector_type(4))) unsigned u32x4;
typedef __attribute__((ext_vector_type(2))) float f32x2;
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;

constexpr int kThreads = 512;          // 8 wavefronts
constexpr int kF1 = 4;                 // conv1 pixel fragments per wave: w + 8i
constexpr int kSteps = 16 + 18;        // K steps of conv2 then conv3
constexpr int kD = 5;                  // weight lookahead in K steps
constexpr int kRing = kD + 1;
// K8: conv2 / conv3 e4m3 weights held in LDS for the whole launch: per
// (layer, channel fragment cf, K = 128 step s) two 1 KB blocks, the low and
// high 16 bytes of each lane's 32 (lane l at 16 l: a 16-byte read of the
// block is free of bank conflicts), conv2 at 0, conv3 at 32 KB, then conv3's
// two K = 32 tail units per fragment (512 bytes each, lane l at 8 l).
constexpr int kWk3 = 32768, kWkTail = 65536, kWkBytes = 69632;

__device__ __forceinline__ unsigned bf2_pack(float a, float b) {
  const bf16x2 h = __builtin_convertvector(f32x2{a, b}, bf16x2);   // v_cvt_pk_bf16_f32 (RNE)
  return *reinterpret_cast<const unsigned*>(&h);
}
__device__ __forceinline__ unsigned fp8_pack4(float a, float b, float c, float d) {
  a = fminf(fmaxf(a, -448.f), 448.f);
  b = fminf(fmaxf(b, -448.f), 448.f);
  c = fminf(fmaxf(c, -448.f), 448.f);
  d = fminf(fmaxf(d, -448.f), 448.f);
  const int lo = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
  return (unsigned)__builtin_amdgcn_cvt_pk_fp8_f32(c, d, lo, true);
}

// Workgroup barrier for LDS hand-offs only.  __syncthreads() also waits for
// every outstanding global load (its workgroup fence drains vmcnt), which
// would cancel the frame and weight prefetches at each barrier; here only
// the LDS queue is drained before s_barrier, global loads stay in flight.
__device__ __forceinline__ void lds_barrier() {
  __asm__ volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Keep global prefetch loads where they are issued: the scheduler may move
// ALU, MFMA and LDS instructions across this point, but no global read, so a
// prefetch is not sunk next to its first use.
__device__ __forceinline__ void pin_vmem_reads() { __builtin_amdgcn_sched_barrier(0x78F); }

// ---- operand traits ------------------------------------------------------
// EB: bytes per element; UB: bytes per 8-element unit (one lane's K group).
template <int P> struct F;
template <> struct F<P_BF16> {
  typedef uint16_t E;
  typedef bf16x8 V;
  static constexpr int EB = 2, UB = 16;
  __device__ static V ld(const void* p) { return *reinterpret_cast<const V*>(p); }
  // 8 pixels starting at a 4-byte-aligned LDS address (two 8-byte reads)
  __device__ static V ld_pix(const unsigned char* p) {
    uint4 u;
    const uint2 a = *reinterpret_cast<const uint2*>(p);
    const uint2 b = *reinterpret_cast<const uint2*>(p + 8);
    u.x = a.x; u.y = a.y; u.z = b.x; u.w = b.y;
    return *reinterpret_cast<const V*>(&u);
  }
  __device__ static f32x4 mma(V a, V b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
  // one lane's weight operand through a buffer resource: byte offset voff + soff
  __device__ static V ldw(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
  }
  // 16 raw pixels -> 16 operands in LDS (32 bytes)
  __device__ static void stage16(unsigned char* dst, uint4 raw, float) {
    const unsigned w[4] = {raw.x, raw.y, raw.z, raw.w};
    uint4 o0, o1;
    unsigned o[8];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      o[2 * i] = bf2_pack((float)(w[i] & 255u), (float)((w[i] >> 8) & 255u));
      o[2 * i + 1] = bf2_pack((float)((w[i] >> 16) & 255u), (float)(w[i] >> 24));
    }
    o0 = make_uint4(o[0], o[1], o[2], o[3]);
    o1 = make_uint4(o[4], o[5], o[6], o[7]);
    *reinterpret_cast<uint4*>(dst) = o0;
    *reinterpret_cast<uint4*>(dst + 16) = o1;
  }
  // 4 consecutive channels -> 8 bytes
  __device__ static void st4(void* p, float a, float b, float c, float d, float) {
    *reinterpret_cast<uint2*>(p) = make_uint2(bf2_pack(a, b), bf2_pack(c, d));
  }
  // 8 consecutive channels as two packed halves of 4 -> 16 bytes
  typedef uint2 PK;
  __device__ static PK pk4(float a, float b, float c, float d, float) {
    return make_uint2(bf2_pack(a, b), bf2_pack(c, d));
  }
  __device__ static void st8(void* p, PK lo, PK hi) {
    *reinterpret_cast<uint4*>(p) = make_uint4(lo.x, lo.y, hi.x, hi.y);
  }
};
template <> struct F<P_FP8> {
  typedef uint8_t E;
  typedef long V;
  static constexpr int EB = 1, UB = 8;
  __device__ static V ld(const void* p) { return *reinterpret_cast<const V*>(p); }
  __device__ static V ld_pix(const unsigned char* p) {
    const unsigned a = *reinterpret_cast<const unsigned*>(p);
    const unsigned b = *reinterpret_cast<const unsigned*>(p + 4);
    return (long)(((unsigned long long)b << 32) | a);
  }
  __device__ static f32x4 mma(V a, V b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c, 0, 0, 0); }
  __device__ static V ldw(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  }
  __device__ static void stage16(unsigned char* dst, uint4 raw, float s8) {
    const unsigned w[4] = {raw.x, raw.y, raw.z, raw.w};
    unsigned o[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
      o[i] = fp8_pack4((float)(w[i] & 255u) * s8, (float)((w[i] >> 8) & 255u) * s8,
                       (float)((w[i] >> 16) & 255u) * s8, (float)(w[i] >> 24) * s8);
    *reinterpret_cast<uint4*>(dst) = make_uint4(o[0], o[1], o[2], o[3]);
  }
  __device__ static void st4(void* p, float a, float b, float c, float d, float s8) {
    *reinterpret_cast<unsigned*>(p) = fp8_pack4(a * s8, b * s8, c * s8, d * s8);
  }
  typedef unsigned PK;
  __device__ static PK pk4(float a, float b, float c, float d, float s8) {
    return fp8_pack4(a * s8, b * s8, c * s8, d * s8);
  }
  __device__ static void st8(void* p, PK lo, PK hi) { *reinterpret_cast<uint2*>(p) = make_uint2(lo, hi); }
};

// LDS layouts (byte offsets), arranged so that every K step of a lane reads
// at a compile-time offset from one per-fragment base address, and padded to
// spread the operand reads over the banks.  (gfx950 serves a 16-byte read of
// each 32-lane half-wavefront in two cycles, one per parity of lane bits
// 2^3^4, each needing 16 distinct 16-byte bank groups; under that rule
// conv2's reads of x1 take about twice the conflict-free cycles, which
// measurements put off the kernel's critical path: the conv2/conv3 weight
// stream is.)
//  x1: conv1 output 20x20x32 split into the 4 stride-2 phases (y&1, x&1) of
//      10x10 pixels each; pixel stride 40 elements (32 channels + 8 pad).
//      conv2's input pixel (2oy+kh, 2ox+kw) is then pixel (oy + kh/2,
//      ox + kw/2) of phase (kh&1, kw&1): neighbouring output pixels read
//      neighbouring LDS pixels.
//  x2: conv2 output 9x9x64, pixel stride 72 elements (64 channels + 8 pad).
//  With the FP8 K = 128 instruction (K8) a lane reads 32 consecutive channels
//  of one pixel per step, two 16-byte reads, and the layouts follow the bank
//  rule above.  x1: 32-byte pixels on rows of 17 pixel slots (17 = 1 mod 8,
//  so consecutive output pixels, row-major within a stack, sit on
//  consecutive bank-group pairs across row ends), phases 341 units of 16
//  bytes apart (odd: a cycle's lanes of the two column phases land on
//  opposite unit parities) and items 1378 units apart (consecutive across
//  items too); conv2's reads are then free of conflicts.  x2: 80-byte
//  pixels, items 409 units apart (conv3's reads at 2x the conflict-free
//  cycles, against 2.4x without the gap and the lane order below).
template <int P, bool K8 = false> struct Lay {
  static constexpr int EB = F<P>::EB;
  static constexpr int X1P = K8 ? 32 : 40 * EB;     // pixel stride
  static constexpr int X1W = K8 ? 17 : 10;          // pixel slots per phase row
  static constexpr int X1PH = K8 ? 341 * 16 : 100 * X1P;   // phase stride
  static constexpr int X1T = K8 ? 1378 * 16 : 4 * X1PH;    // item stride
  static constexpr int X2P = K8 ? 80 : 72 * EB;
  static constexpr int X2T = K8 ? 409 * 16 : 81 * X2P;
  __device__ static int x1(int t, int y, int x, int c) {
    return t * X1T + ((y & 1) * 2 + (x & 1)) * X1PH + ((y >> 1) * X1W + (x >> 1)) * X1P + c * EB;
  }
  __device__ static int x2(int t, int p, int c) { return t * X2T + p * X2P + c * EB; }
};

// One workgroup of 8 wavefronts per CU (the rounds use most of the LDS), so
// two wavefronts share each SIMD and cover each other's memory latency.  In
// conv2 / conv3 wave w takes channel half (w & 1) and pixel fragments
// (w >> 1) + 4i; their weight fragments stream from L2 kD K steps ahead.
//
// K8 (FP8 only, rounds of 3): conv2 and conv3 run on
// v_mfma_scale_f32_16x16x128_f8f6f4 (unit scales): a K step is 128 values --
// 4 taps x 32 channels in conv2, 2 taps x 64 channels in conv3 -- at twice
// the matrix rate of the K = 32 instruction.  Their weights (68 KB in e4m3)
// are copied into LDS once per launch, so no weight stream competes with the
// matrix work; conv3's last 64 K values (its ninth tap) use two K = 32
// steps.  conv1 is unchanged.
// Makes the accumulators' current values materialise here (an empty asm
// that reads and rewrites them): without it the compiler sinks a fragment's
// whole chain of matrix instructions into its conditional epilogue, which
// keeps every step's operands live at once and spills.
template <int N>
__device__ __forceinline__ void pin_acc(f32x4 (&acc)[N][2]) {
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) asm volatile("" : "+v"(acc[i][j]));
}

template <int P, int T, bool K8 = false>
__global__ void __launch_bounds__(kThreads, 1) conv_fused_kernel(FusedConvArgs a) {
  static_assert(!K8 || (P == P_FP8 && T == 3), "the K = 128 path is FP8 in rounds of 3");
  typedef F<P> Fr;
  typedef typename Fr::V V;
  constexpr int EB = Fr::EB;
  constexpr int FRB = kFrameBytes * EB;                 // staged frame bytes
  constexpr int R2 = T * 81, F2 = (R2 + 15) / 16, F2W = (F2 + 3) / 4;
  constexpr int R3 = T * 49, F3 = (R3 + 15) / 16, F3W = (F3 + 3) / 4;
  typedef Lay<P, K8> L;
  // x1 of the round's items; ux holds the round's input frames during conv1
  // and x2 from conv2's epilogue to the end of conv3 (never both at once)
  constexpr int NFR = T > 3 ? T : 3;                    // frames staged at once
  constexpr int UXB = (T * L::X2T > NFR * FRB) ? T * L::X2T : NFR * FRB;
  __shared__ __attribute__((aligned(16))) unsigned char x1[T * L::X1T];
  __shared__ __attribute__((aligned(16))) unsigned char ux[UXB];
  __shared__ __attribute__((aligned(16))) unsigned char w1l[12 * 64 * 8 * EB];   // conv1 weights, channels 0..2
  __shared__ __attribute__((aligned(16))) float sbias[2][64];   // conv2, conv3 biases
  __shared__ __attribute__((aligned(16))) unsigned char wk[K8 ? kWkBytes : 16];   // K8 weights (layout above)

  // Item descriptors and groups are read-only here: reading them through the
  // constant address space makes their uniform loads scalar (counted by
  // lgkmcnt), so waiting for one never waits for the weight loads in flight.
  typedef const __attribute__((address_space(4))) ItemDesc CDesc;
  typedef const __attribute__((address_space(4))) FusedGroup CGroup;
  CDesc* const dsc = (CDesc*)a.desc;
  CGroup* const grp = (CGroup*)a.groups;
  // Persistent: workgroup b takes groups b, b + gridDim.x, ... of the chunk.
  int gi = blockIdx.x;
  if (gi >= a.n_groups) return;
  int G = grp[gi].count;
  long long i0 = grp[gi].item0 - a.item_base;   // chunk-relative first item
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r16 = lane & 15, g = lane >> 4;
  const int half = wave & 1, fq = wave >> 1;      // channel half, first pixel fragment
  const unsigned char* W1 = reinterpret_cast<const unsigned char*>(a.w[0]);
  // conv2 / conv3 weights, fragment-major: the A operand of channel
  // fragment cf at K step s is 64 lanes x 8 elements, contiguous.  They are
  // read through buffer resources so that a step's offset is a scalar: the
  // only per-lane address is the lane offset within this wave's fragments.
  constexpr int FB = 64 * 8 * EB;                       // bytes per weight fragment
  const __amdgpu_buffer_rsrc_t W2r = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<void*>(a.w[1]), (short)0, 64 * 512 * EB, 0x00020000);
  const __amdgpu_buffer_rsrc_t W3r = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<void*>(a.w[2]), (short)0, 64 * 576 * EB, 0x00020000);
  const int v2 = half * 2 * 16 * FB + lane * 8 * EB;    // channel fragments 2*half, +1
  const int v3 = half * 2 * 18 * FB + lane * 8 * EB;
  // weight step u of the conv2 -> conv3 sequence: this wave's 2 channel fragments
  auto wstep = [&](int u, V (&w)[2]) {
    if (u < 16) {
#pragma unroll
      for (int j = 0; j < 2; ++j) w[j] = Fr::ldw(W2r, v2, (j * 16 + u) * FB);
    } else {
#pragma unroll
      for (int j = 0; j < 2; ++j) w[j] = Fr::ldw(W3r, v3, (j * 18 + u - 16) * FB);
    }
  };
  // K8: this wave's two channel fragments at weight step u (conv2 0..3,
  // conv3 4..7), read from the LDS copy
  auto wlds = [&](int u, v8i (&w)[2]) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int blk = (u < 4 ? 0 : kWk3) + (((2 * half + j) * 4 + (u & 3)) * 2) * 1024 + lane * 16;
      const u32x4 lo = *reinterpret_cast<const u32x4*>(&wk[blk]);
      const u32x4 hi = *reinterpret_cast<const u32x4*>(&wk[blk + 1024]);
      w[j] = v8i{(int)lo[0], (int)lo[1], (int)lo[2], (int)lo[3], (int)hi[0], (int)hi[1], (int)hi[2], (int)hi[3]};
    }
  };
  unsigned char* X3 = reinterpret_cast<unsigned char*>(a.x3);
  const float s8 = a.pix_s8;

  // frames: 441 16-byte chunks, one per thread; threads past the last chunk
  // load and stage a duplicate of the last chunk (identical bytes to the
  // same LDS address), so neither the load nor its use sits behind a branch
  const bool cf = tid < kFrameBytes / 16;
  const int ck = cf ? tid : kFrameBytes / 16 - 1;
  // (frame pointers come from memory, so they are generic; the cast makes
  // these global loads, which the LDS-only barrier's lgkmcnt wait ignores;
  // a flat load would be counted there too and end the prefetch early)
  auto fload = [&](const uint8_t* fr) {
    typedef __attribute__((ext_vector_type(4))) unsigned u32x4;
    const u32x4 v = ((const __attribute__((address_space(1))) u32x4*)fr)[ck];
    return make_uint4(v[0], v[1], v[2], v[3]);
  };
  auto fstage = [&](int slot, const uint4& u) { Fr::stage16(&ux[slot * FRB + ck * 16 * EB], u, s8); };

  // conv1 and the group's S phase map wavefront w to pixel fragments
  // f = w + 8i (i < 3) and slot i = 3 to fragment 24, for BOTH channel
  // halves: each pixel operand read from LDS feeds two MFMAs.  (conv2 /
  // conv3 split channel halves between wavefront pairs.)
  // conv1 weights (A operand): K step s covers stack channel s/2, kernel rows
  // 4(s&1)..+3; lane group g holds kernel row 4(s&1)+g (8 kw values).  Only
  // channel 3 (s = 6, 7) stays in registers; channels 0..2 (used once per
  // group, by S) are kept in LDS, operand-major: unit (h2, s, lane).
  // Row l of channel fragment h2 is channel 8(l/4) + 4 h2 + l%4 (paired
  // rows), so lane group g's results of both fragments are the 8
  // consecutive channels 8g .. 8g + 7, stored with one write.
  auto w1row = [](int h2, int l) { return 8 * (l >> 2) + 4 * h2 + (l & 3); };
  auto w1ld = [&](int h2, int s) { return Fr::ld(W1 + (w1row(h2, r16) * 256 + 32 * s + 8 * g) * EB); };
  for (int k = tid; k < 12 * 64; k += kThreads) {
    const int hs = k >> 6, l = k & 63, h2 = hs / 6, s2 = hs % 6;
    *reinterpret_cast<V*>(&w1l[k * 8 * EB]) = Fr::ld(W1 + (w1row(h2, l & 15) * 256 + 32 * s2 + 8 * (l >> 4)) * EB);
  }
  if constexpr (K8) {
    // the K = 128 weight copies (fragment-major in memory: per fragment, 16
    // rows x K bytes, K = 128 units of 32 bytes per lane, then K = 32 units
    // of 8) into the LDS layout, 16 bytes per thread and pass
    const unsigned char* W2k = reinterpret_cast<const unsigned char*>(a.w[1]);
    const unsigned char* W3k = reinterpret_cast<const unsigned char*>(a.w[2]);
    for (int c = tid; c < kWkBytes / 16; c += kThreads) {
      const unsigned char* src;
      int dst;
      if (c < 4096) {                     // K = 128 units: c = ((cf * 4 + s) * 64 + lane) * 2 + part
        const int c3 = c >= 2048, cc = c & 2047;
        const int part = cc & 1, ln = (cc >> 1) & 63, us = cc >> 7;
        src = c3 ? W3k + (us >> 2) * 16 * 576 + ((us & 3) * 64 + ln) * 32 + part * 16 : W2k + cc * 16;
        // conv3: lane group g of a step takes tap offset g & 1 and channel
        // half g >> 1 (the bank-friendly order of its pixel reads), which in
        // memory is lane group 2 (g & 1) + (g >> 1): the two index bits swap
        const int lg = c3 ? ((((ln >> 4) & 1) << 1) | (ln >> 5)) : (ln >> 4);
        dst = (c3 ? kWk3 : 0) + (us * 2 + part) * 1024 + ((ln & 15) + 16 * lg) * 16;
      } else {                            // conv3's K = 32 units: 1 KB per fragment
        const int cc = c - 4096;
        src = W3k + (cc >> 6) * 16 * 576 + 4 * 2048 + (cc & 63) * 16;
        dst = kWkTail + cc * 16;
      }
      *reinterpret_cast<u32x4*>(&wk[dst]) = *reinterpret_cast<const u32x4*>(src);
    }
  }
  V w1c[2][2];
#pragma unroll
  for (int h2 = 0; h2 < 2; ++h2)
#pragma unroll
    for (int h = 0; h < 2; ++h) w1c[h2][h] = w1ld(h2, 6 + h);
  float b1[2][4];
#pragma unroll
  for (int h2 = 0; h2 < 2; ++h2)
#pragma unroll
    for (int q = 0; q < 4; ++q) b1[h2][q] = a.bias[0][8 * g + 4 * h2 + q];
  // Fragment 24 (slot i = 3) of a round's item t belongs to wavefront t, so
  // the round's 25T fragments spread over the wavefronts as evenly as the
  // per-wave S fragments allow; wavefronts 0..T-1 keep S for fragment 24.
  const bool f3 = wave < T;

  // output pixel 16f + r16 of conv1 fragment i
  int poff[kF1];
#pragma unroll
  for (int i = 0; i < kF1; ++i) {
    const int f = i == kF1 - 1 ? 24 : wave + 8 * i;
    const int p = f * 16 + r16;
    poff[i] = ((p / 20) * 4 * kFrame + (p % 20) * 4) * EB;
  }

  // ---- group inputs ----
  // The first group's shared frames and first round's frames are requested
  // here; a later group's arrive in registers during the previous group's
  // last round (alongside its conv2/conv3) and are staged at that round's
  // end, so a group starts without an HBM round trip.  A later round's
  // frames likewise load during the previous round.
  if (tid < 128) sbias[tid >> 6][tid & 63] = a.bias[1 + (tid >> 6)][tid & 63];
  uint4 sv[3], fv[T];
#pragma unroll
  for (int c = 0; c < 3; ++c) sv[c] = fload(dsc[i0].frame[c]);
#pragma unroll
  for (int t = 0; t < T; ++t) fv[t] = fload(dsc[i0 + (t < G ? t : G - 1)].frame[3]);
#pragma unroll
  for (int c = 0; c < 3; ++c) fstage(c, sv[c]);

  for (;;) {
  // ---- S: channels 0..2 of the group's shared stack ----
  f32x4 S[kF1][2];
#pragma unroll
  for (int i = 0; i < kF1; ++i) S[i][0] = S[i][1] = f32x4{0.f, 0.f, 0.f, 0.f};
  lds_barrier();         // the group's shared frames are staged
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    V w[2][2];
#pragma unroll
    for (int h2 = 0; h2 < 2; ++h2)
#pragma unroll
      for (int h = 0; h < 2; ++h) w[h2][h] = Fr::ld(&w1l[((h2 * 6 + 2 * c + h) * 64 + lane) * 8 * EB]);
#pragma unroll
    for (int i = 0; i < kF1; ++i) {
      if (i == kF1 - 1 && !f3) continue;                 // wave-uniform: fragment 24
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const V pix = Fr::ld_pix(&ux[c * FRB + poff[i] + (4 * h + g) * kFrame * EB]);
#pragma unroll
        for (int h2 = 0; h2 < 2; ++h2) S[i][h2] = Fr::mma(w[h2][h], pix, S[i][h2]);
      }
    }
  }
  lds_barrier();         // the S reads are done
#pragma unroll
  for (int t = 0; t < T; ++t) fstage(t, fv[t]);

  // the next group of this workgroup (this group's own when there is none)
  const int gn = gi + (int)gridDim.x;
  const bool has_next = gn < a.n_groups;
  const int gq = __builtin_amdgcn_readfirstlane(has_next ? gn : gi);
  const int Gq = grp[gq].count;
  const long long iq = grp[gq].item0 - a.item_base;

  for (int r0 = 0; r0 < G; r0 += T) {
    const int nt = (G - r0) < T ? (G - r0) : T;
    V wr[kRing][2];      // conv2 / conv3 weight ring (its first kD steps load during conv1)
    lds_barrier();       // the round's frames are staged

    // ---- conv1: S + channel 3 of each item -> x1 ----
    // Software-pipelined over the round's items: item t+1's pixel operands
    // are read and its MFMAs issued before item t's epilogue, so the
    // epilogue's VALU work runs while the matrix core is busy.  All T items
    // are computed: a slot past the group's last item holds a staged copy of
    // a valid frame, and its x1 rows are never read by conv2.
    {
      const float sc = a.acc_scale[0], o8 = a.out_s8[0];
      V pv[kF1][2];
      f32x4 cc[2][kF1][2];
      auto reads = [&](int t) {
#pragma unroll
        for (int i = 0; i < kF1; ++i)
#pragma unroll
          for (int h = 0; h < 2; ++h) pv[i][h] = Fr::ld_pix(&ux[t * FRB + poff[i] + (4 * h + g) * kFrame * EB]);
      };
      auto mmas = [&](int t, int b) {
#pragma unroll
        for (int i = 0; i < kF1 - 1; ++i)
#pragma unroll
          for (int h2 = 0; h2 < 2; ++h2) cc[b][i][h2] = Fr::mma(w1c[h2][0], pv[i][0], S[i][h2]);
#pragma unroll
        for (int i = 0; i < kF1 - 1; ++i)
#pragma unroll
          for (int h2 = 0; h2 < 2; ++h2) cc[b][i][h2] = Fr::mma(w1c[h2][1], pv[i][1], cc[b][i][h2]);
        if (wave == t) {                                  // wave-uniform: fragment 24 of item t
#pragma unroll
          for (int h2 = 0; h2 < 2; ++h2) cc[b][3][h2] = Fr::mma(w1c[h2][0], pv[3][0], S[3][h2]);
#pragma unroll
          for (int h2 = 0; h2 < 2; ++h2) cc[b][3][h2] = Fr::mma(w1c[h2][1], pv[3][1], cc[b][3][h2]);
        }
      };
      auto epi = [&](int t, int b) {
#pragma unroll
        for (int i = 0; i < kF1; ++i) {
          if (i == kF1 - 1 && wave != t) continue;       // wave-uniform: fragment 24 is wave t's
          const int p = (i == kF1 - 1 ? 24 : wave + 8 * i) * 16 + r16;
          typename Fr::PK pk[2];
#pragma unroll
          for (int h2 = 0; h2 < 2; ++h2)
            pk[h2] = Fr::pk4(fmaxf(cc[b][i][h2][0] * sc + b1[h2][0], 0.f), fmaxf(cc[b][i][h2][1] * sc + b1[h2][1], 0.f),
                             fmaxf(cc[b][i][h2][2] * sc + b1[h2][2], 0.f), fmaxf(cc[b][i][h2][3] * sc + b1[h2][3], 0.f),
                             o8);
          Fr::st8(&x1[L::x1(t, p / 20, p % 20, 8 * g)], pk[0], pk[1]);
        }
      };
      // The first kD K steps of conv2's weights are requested in T parts,
      // each after an item's MFMAs: issued all at once they wait on the
      // vector-memory path (8 wavefronts x 2 KB per step), which conv1 does
      // not otherwise use, so spread out they overlap conv1's work.
      auto ring_part = [&](int j) {
        if constexpr (!K8) {
#pragma unroll
          for (int u = j * kD / T; u < (j + 1) * kD / T; ++u) wstep(u, wr[u % kRing]);
        }
        __builtin_amdgcn_sched_barrier(0);
      };
      reads(0);
      mmas(0, 0);
      ring_part(0);
#pragma unroll
      for (int t = 0; t < T; ++t) {
        if (t + 1 < T) {
          reads(t + 1);
          mmas(t + 1, (t + 1) & 1);
          ring_part(t + 1);
        }
        epi(t, t & 1);
      }
    }
    lds_barrier();       // x1 complete, frame reads done: conv2's epilogue may overwrite ux
    // The next round's frames; in the group's last round, the next group's
    // shared frames and first round's frames.  Slots past a group's end load
    // its last item's frame (staged, never used).
    const bool last = r0 + T >= G;
    {
      const bool nxt = last && has_next;
      const long long ib = nxt ? iq : i0;
      const int gb = nxt ? Gq : G, kb = nxt ? 0 : r0 + T;
#pragma unroll
      for (int t = 0; t < T; ++t) {
        const int k = kb + t;
        fv[t] = fload(dsc[ib + (k < gb ? k : gb - 1)].frame[3]);
      }
      if (nxt) {
#pragma unroll
        for (int c = 0; c < 3; ++c) sv[c] = fload(dsc[iq].frame[c]);
      }
    }

    if constexpr (K8) {
    // ---- conv2 and conv3 on the K = 128 instruction ----
    // conv2 step s (s = 0..3): lane group g holds tap (kh = s, kw = g), all
    // 32 channels; conv3 step s (s = 0..3): tap 2s + (g & 1), channels
    // 32 (g >> 1) .. +31; then conv3's ninth tap as two K = 32 steps.
    {
      const int rows2 = nt * 81;
      f32x4 acc[F2W][2];
      int base[F2W];
      bool ok[F2W];
#pragma unroll
      for (int i = 0; i < F2W; ++i) {
        const int r = (fq + 4 * i) * 16 + r16;
        ok[i] = r < rows2;
        // rows past the round's items read some in-bounds pixel (results
        // unused): their own slot, or 16 rows back past the last item, which
        // keeps the cycle's bank groups distinct
        const int rr = r < T * 81 ? r : r - 16;
        const int t = rr / 81, p = rr % 81;
        base[i] = t * L::X1T + ((p / 9) * L::X1W + (p % 9)) * L::X1P;
        acc[i][0] = acc[i][1] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
      // (gp: the lane group, re-derived here so that the compiler keeps the
      // per-step offsets inside the round instead of holding all of them in
      // registers across it)
      int gp = g;
      asm volatile("" : "+v"(gp));
      auto koff2 = [&](int st) {   // this lane's tap (kh = st, kw = g)
        return ((st & 1) * 2 + (gp & 1)) * L::X1PH + ((st >> 1) * L::X1W + (gp >> 1)) * L::X1P;
      };
      auto ld32 = [](const unsigned char* q) {
        const u32x4 lo = *reinterpret_cast<const u32x4*>(q);
        const u32x4 hi = *reinterpret_cast<const u32x4*>(q + 16);
        return v8i{(int)lo[0], (int)lo[1], (int)lo[2], (int)lo[3], (int)hi[0], (int)hi[1], (int)hi[2], (int)hi[3]};
      };
      // A step reads the next step's weights, and each fragment the next
      // fragment's pixels (the last one the next step's first), one ahead;
      // the steps rotate by slot index (compile-time after unrolling).  A
      // scheduling barrier closes every step, so the compiler cannot hoist a
      // later step's reads and run out of registers.
      v8i wq[2][2], pv[2];
      wlds(0, wq[0]);
      pv[0] = ld32(&x1[base[0] + koff2(0)]);
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        if (st + 1 < 4) wlds(st + 1, wq[(st + 1) & 1]);
        const int ko = koff2(st);
#pragma unroll
        for (int i = 0; i < F2W; ++i) {
          const int n = st * F2W + i;      // pixel operand slot n & 1
          if (i + 1 < F2W) pv[(n + 1) & 1] = ld32(&x1[base[i + 1] + ko]);   // clamped rows
          else if (st + 1 < 4) pv[(n + 1) & 1] = ld32(&x1[base[0] + koff2(st + 1)]);
          __builtin_amdgcn_sched_barrier(0);   // the next fragment's read goes out before these
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(wq[st & 1][j], pv[n & 1], acc[i][j],
                                                                          0, 0, 0, 127, 0, 127);
          __builtin_amdgcn_sched_barrier(0);
        }
        pin_acc(acc);
        __builtin_amdgcn_sched_barrier(0);
      }
      const float sc = a.acc_scale[1], o8 = a.out_s8[1];
      float bb[2][4];
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) bb[j][q] = sbias[0][32 * half + 8 * g + 4 * j + q];   // paired rows
#pragma unroll
      for (int i = 0; i < F2W; ++i) {
        if (!ok[i]) continue;
        const int r = (fq + 4 * i) * 16 + r16;
        const int t = r / 81, p = r % 81;
        typename Fr::PK pk[2];
#pragma unroll
        for (int j = 0; j < 2; ++j)
          pk[j] = Fr::pk4(fmaxf(acc[i][j][0] * sc + bb[j][0], 0.f), fmaxf(acc[i][j][1] * sc + bb[j][1], 0.f),
                          fmaxf(acc[i][j][2] * sc + bb[j][2], 0.f), fmaxf(acc[i][j][3] * sc + bb[j][3], 0.f), o8);
        Fr::st8(&ux[L::x2(t, p, 32 * half + 8 * g)], pk[0], pk[1]);
      }
    }
    lds_barrier();
    {
      const int rows3 = nt * 49;
      f32x4 acc[F3W][2];
      int base[F3W], pt[F3W];
      bool ok[F3W];
#pragma unroll
      for (int i = 0; i < F3W; ++i) {
        const int r = (fq + 4 * i) * 16 + r16;
        ok[i] = r < rows3;
        const int rr = r < T * 49 ? r : r - 16;   // as in conv2
        const int p = rr % 49;
        pt[i] = rr / 49;
        base[i] = pt[i] * L::X2T + ((p / 7) * 9 + (p % 7)) * L::X2P;
        acc[i][0] = acc[i][1] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
      int gp = g;                  // (re-derived in the round, as in conv2)
      asm volatile("" : "+v"(gp));
      auto koff3 = [&](int st) {   // this lane's tap 2 st + (g & 1), channels 32 (g >> 1)
        const int kk = 2 * st + (gp & 1);
        return ((kk / 3) * 9 + kk % 3) * L::X2P + 32 * (gp >> 1);
      };
      auto ld32 = [](const unsigned char* q) {
        const u32x4 lo = *reinterpret_cast<const u32x4*>(q);
        const u32x4 hi = *reinterpret_cast<const u32x4*>(q + 16);
        return v8i{(int)lo[0], (int)lo[1], (int)lo[2], (int)lo[3], (int)hi[0], (int)hi[1], (int)hi[2], (int)hi[3]};
      };
      v8i wq[2][2], pv[2];
      wlds(4, wq[0]);
      pv[0] = ld32(&ux[base[0] + koff3(0)]);
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        if (st + 1 < 4) wlds(st + 5, wq[(st + 1) & 1]);
        const int ko = koff3(st);
#pragma unroll
        for (int i = 0; i < F3W; ++i) {
          const int n = st * F3W + i;
          if (i + 1 < F3W) pv[(n + 1) & 1] = ld32(&ux[base[i + 1] + ko]);   // clamped rows
          else if (st + 1 < 4) pv[(n + 1) & 1] = ld32(&ux[base[0] + koff3(st + 1)]);
          __builtin_amdgcn_sched_barrier(0);   // the next fragment's read goes out before these
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(wq[st & 1][j], pv[n & 1], acc[i][j],
                                                                          0, 0, 0, 127, 0, 127);
          __builtin_amdgcn_sched_barrier(0);
        }
        pin_acc(acc);
        __builtin_amdgcn_sched_barrier(0);
      }
      // the ninth tap's weights: two K = 32 units of 8 bytes per lane
      V wt[2][2];
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int j = 0; j < 2; ++j) wt[t][j] = Fr::ld(&wk[kWkTail + (2 * half + j) * 1024 + (t * 64 + lane) * 8]);
      // tap 8 (kh = 2, kw = 2): K = 32 steps t = 0, 1 over channels 32t + 8g .. +7
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int ko = (2 * 9 + 2) * L::X2P + 32 * t + 8 * g;
#pragma unroll
        for (int i = 0; i < F3W; ++i) {
          const V pvt = Fr::ld(&ux[base[i] + ko]);
#pragma unroll
          for (int j = 0; j < 2; ++j) acc[i][j] = Fr::mma(wt[t][j], pvt, acc[i][j]);
        }
      }
      const float sc = a.acc_scale[2], o8 = a.out_s8[2];
      float bb[2][4];
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) bb[j][q] = sbias[1][32 * half + 8 * g + 4 * j + q];   // permuted rows
      const long long item_first = i0 + r0;
#pragma unroll
      for (int i = 0; i < F3W; ++i) {
        if (!ok[i]) continue;
        const int r = (fq + 4 * i) * 16 + r16;
        const long long item = item_first + pt[i];
        const int px = r - pt[i] * 49;
        typename Fr::PK pk[2];
#pragma unroll
        for (int j = 0; j < 2; ++j)
          pk[j] = Fr::pk4(fmaxf(acc[i][j][0] * sc + bb[j][0], 0.f), fmaxf(acc[i][j][1] * sc + bb[j][1], 0.f),
                          fmaxf(acc[i][j][2] * sc + bb[j][2], 0.f), fmaxf(acc[i][j][3] * sc + bb[j][3], 0.f), o8);
        Fr::st8(X3 + fc1_tiled_offset(item, (px * 64 + 32 * half + 8 * g) * EB, EB), pk[0], pk[1]);
      }
    }
    } else {
    // ---- conv2 (x1 -> x2) and conv3 (x2 -> x3) ----
    // The K steps of both layers form one sequence u = 0..33 (conv2 steps
    // 0..15, conv3 steps 16..33).  Weight fragments stream from L2 kD steps
    // ahead through a register ring that runs across the layer boundary;
    // pixel fragments are read from LDS one step ahead.  A full scheduling
    // barrier between steps keeps every load at its issue point.
    {
      const int rows2 = nt * 81;
      f32x4 acc[F2W][2];
      int base[F2W];
      bool ok[F2W];
#pragma unroll
      for (int i = 0; i < F2W; ++i) {
        const int r = (fq + 4 * i) * 16 + r16;
        ok[i] = r < rows2;
        const int rr = ok[i] ? r : 0;
        const int t = rr / 81, p = rr % 81;
        base[i] = t * L::X1T + ((p / 9) * L::X1W + (p % 9)) * L::X1P + 8 * g * EB;
        acc[i][0] = acc[i][1] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
      // conv2 K step s: kernel row kh = s/4, column kw = s%4; lane group g
      // holds input channels 8g..8g+7 of that tap
      auto koff2 = [](int s) {
        const int kh = s >> 2, kw = s & 3;
        return ((kh & 1) * 2 + (kw & 1)) * L::X1PH + ((kh >> 1) * L::X1W + (kw >> 1)) * L::X1P;
      };
      V pv[2][F2W];
#pragma unroll
      for (int i = 0; i < F2W; ++i) pv[0][i] = Fr::ld(&x1[base[i] + koff2(0)]);
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        if (s + kD < kSteps) wstep(s + kD, wr[(s + kD) % kRing]);
        if (s + 1 < 16) {
#pragma unroll
          for (int i = 0; i < F2W; ++i) pv[(s + 1) & 1][i] = Fr::ld(&x1[base[i] + koff2(s + 1)]);  // clamped rows
        }
#pragma unroll
        for (int i = 0; i < F2W; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) acc[i][j] = Fr::mma(wr[s % kRing][j], pv[s & 1][i], acc[i][j]);
        __builtin_amdgcn_sched_barrier(0);
      }
      const float sc = a.acc_scale[1], o8 = a.out_s8[1];
      float bb[2][4];
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) bb[j][q] = sbias[0][32 * half + 8 * g + 4 * j + q];   // paired rows
#pragma unroll
      for (int i = 0; i < F2W; ++i) {
        if (!ok[i]) continue;
        const int r = (fq + 4 * i) * 16 + r16;
        const int t = r / 81, p = r % 81;
        typename Fr::PK pk[2];
#pragma unroll
        for (int j = 0; j < 2; ++j)
          pk[j] = Fr::pk4(fmaxf(acc[i][j][0] * sc + bb[j][0], 0.f), fmaxf(acc[i][j][1] * sc + bb[j][1], 0.f),
                          fmaxf(acc[i][j][2] * sc + bb[j][2], 0.f), fmaxf(acc[i][j][3] * sc + bb[j][3], 0.f), o8);
        Fr::st8(&ux[L::x2(t, p, 32 * half + 8 * g)], pk[0], pk[1]);
      }
    }
    lds_barrier();
    {
      // conv3 K step s: kernel tap kk = s/2 (kh = kk/3, kw = kk%3),
      // channels 32(s&1) + 8g .. +7; output to HBM, channels-last [item][49][64]
      const int rows3 = nt * 49;
      f32x4 acc[F3W][2];
      int base[F3W], pt[F3W];
      bool ok[F3W];
#pragma unroll
      for (int i = 0; i < F3W; ++i) {
        const int r = (fq + 4 * i) * 16 + r16;
        ok[i] = r < rows3;
        const int rr = ok[i] ? r : 0;
        const int p = rr % 49;
        pt[i] = rr / 49;
        base[i] = pt[i] * L::X2T + ((p / 7) * 9 + (p % 7)) * L::X2P + 8 * g * EB;
        acc[i][0] = acc[i][1] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
      auto koff3 = [](int s) {
        const int kk = s >> 1;
        return ((kk / 3) * 9 + kk % 3) * L::X2P + 32 * (s & 1) * EB;
      };
      V pv[2][F3W];
#pragma unroll
      for (int i = 0; i < F3W; ++i) pv[0][i] = Fr::ld(&ux[base[i] + koff3(0)]);
#pragma unroll
      for (int s = 0; s < 18; ++s) {
        const int u = 16 + s;
        if (u + kD < kSteps) wstep(u + kD, wr[(u + kD) % kRing]);
        if (s + 1 < 18) {
#pragma unroll
          for (int i = 0; i < F3W; ++i) pv[(s + 1) & 1][i] = Fr::ld(&ux[base[i] + koff3(s + 1)]);  // clamped rows
        }
#pragma unroll
        for (int i = 0; i < F3W; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) acc[i][j] = Fr::mma(wr[u % kRing][j], pv[s & 1][i], acc[i][j]);
        __builtin_amdgcn_sched_barrier(0);
      }
      const float sc = a.acc_scale[2], o8 = a.out_s8[2];
      float bb[2][4];
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) bb[j][q] = sbias[1][32 * half + 8 * g + 4 * j + q];   // permuted rows
      const long long item_first = i0 + r0;
#pragma unroll
      for (int i = 0; i < F3W; ++i) {
        if (!ok[i]) continue;
        const int r = (fq + 4 * i) * 16 + r16;
        const long long item = item_first + pt[i];
        const int px = r - pt[i] * 49;
        typename Fr::PK pk[2];
#pragma unroll
        for (int j = 0; j < 2; ++j)
          pk[j] = Fr::pk4(fmaxf(acc[i][j][0] * sc + bb[j][0], 0.f), fmaxf(acc[i][j][1] * sc + bb[j][1], 0.f),
                          fmaxf(acc[i][j][2] * sc + bb[j][2], 0.f), fmaxf(acc[i][j][3] * sc + bb[j][3], 0.f), o8);
        Fr::st8(X3 + fc1_tiled_offset(item, (px * 64 + 32 * half + 8 * g) * EB, EB), pk[0], pk[1]);
      }
    }
    }
    lds_barrier();       // conv3's reads of x2 are done: ux takes the next frames
    if (!last) {
#pragma unroll
      for (int t = 0; t < T; ++t) fstage(t, fv[t]);
    } else if (has_next) {
#pragma unroll
      for (int c = 0; c < 3; ++c) fstage(c, sv[c]);
    }
    // x1 was last read by conv2, before the barrier after conv2's epilogue
  }
  if (!has_next) break;
  gi = gq;
  G = Gq;
  i0 = iq;
  }
}

// Fragment-major copy of W[N][K]: unit u = (cf, s, lane) receives the 8
// elements W[row][32s + 8(lane/16) .. +7] of row 16cf + lane%16, or with
// `pair8` of row 32(cf/2) + 8(l/4) + 4(cf%2) + l%4 (l = lane%16): then the
// two fragments 2h, 2h + 1 leave lane group g of an MFMA result with the 8
// consecutive channels 32h + 8g .. +7.
__global__ void fragment_major_kernel(const unsigned char* __restrict__ src, unsigned char* __restrict__ dst, int N,
                                      int K, int eb, int pair8) {
  const int NS = K / 32;
  const long long units = (long long)(N / 16) * NS * 64;
  const long long u = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= units) return;
  const int lane = (int)(u % 64), s = (int)((u / 64) % NS), cf = (int)(u / 64 / NS);
  const int l = lane % 16;
  const int row = pair8 ? 32 * (cf / 2) + 8 * (l / 4) + 4 * (cf % 2) + l % 4 : 16 * cf + l;
  const unsigned char* sp = src + ((long long)row * K + 32 * s + 8 * (lane / 16)) * eb;
  unsigned char* dp = dst + u * 8 * eb;
  for (int b = 0; b < 8 * eb; ++b) dp[b] = sp[b];
}

// Fragment-major copy for the FP8 K = 128 instruction: per channel
// fragment cf, K128 units (s, lane) of 32 bytes -- W[row][128s + 32(lane/16)
// .. +31] -- for s < K / 128, then K = 32 units (t, lane) of 8 bytes for the
// remaining K % 128 values -- W[row][128 (K/128) + 32t + 8(lane/16) .. +7];
// rows paired as in fragment_major_kernel.  A fragment's 16 rows x K bytes
// stay one contiguous block.
__global__ void fragment_major_k128_kernel(const unsigned char* __restrict__ src, unsigned char* __restrict__ dst,
                                           int N, int K) {
  const int NS = K / 128, NT = (K % 128) / 32;
  const long long units = (long long)(N / 16) * (NS + NT) * 64;
  const long long u = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= units) return;
  const int lane = (int)(u % 64), su = (int)((u / 64) % (NS + NT)), cf = (int)(u / 64 / (NS + NT));
  const int l = lane % 16, g = lane / 16;
  const int row = 32 * (cf / 2) + 8 * (l / 4) + 4 * (cf % 2) + l % 4;
  const unsigned char* sp;
  unsigned char* dp = dst + (long long)cf * 16 * K;
  int nb;
  if (su < NS) {
    sp = src + (long long)row * K + 128 * su + 32 * g;
    dp += ((long long)su * 64 + lane) * 32;
    nb = 32;
  } else {
    const int t = su - NS;
    sp = src + (long long)row * K + 128 * NS + 32 * t + 8 * g;
    dp += (long long)NS * 64 * 32 + ((long long)t * 64 + lane) * 8;
    nb = 8;
  }
  for (int b = 0; b < nb; ++b) dp[b] = sp[b];
}

}  // namespace

void launch_fragment_major_k128(const void* src, void* dst, int N, int K, hipStream_t s) {
  const long long units = (long long)(N / 16) * (K / 128 + (K % 128) / 32) * 64;
  hipLaunchKernelGGL(fragment_major_k128_kernel, dim3((unsigned)((units + 255) / 256)), dim3(256), 0, s,
                     reinterpret_cast<const unsigned char*>(src), reinterpret_cast<unsigned char*>(dst), N, K);
}

void launch_fragment_major(const void* src, void* dst, int N, int K, int eb, bool pair8, hipStream_t s) {
  const long long units = (long long)(N / 16) * (K / 32) * 64;
  hipLaunchKernelGGL(fragment_major_kernel, dim3((unsigned)((units + 255) / 256)), dim3(256), 0, s,
                     reinterpret_cast<const unsigned char*>(src), reinterpret_cast<unsigned char*>(dst), N, K, eb,
                     pair8 ? 1 : 0);
}

void launch_conv_fused(int prec, int T, const FusedConvArgs& args, int n_groups, hipStream_t s, bool k8) {
  if (n_groups <= 0) return;
  typedef void (*Kern)(FusedConvArgs);
  // BF16 at T = 4 exceeds the LDS of one CU: T <= 3; FP8 takes T <= 4 with
  // the K = 32 instruction and 3 with the K = 128 one (its weights take 68 KB
  // of LDS); other values take 3
  k8 = k8 && prec == P_FP8;
  const int Tk = k8 ? 3 : (T == 1 || T == 2 || (T == 4 && prec != P_BF16)) ? T : 3;
  Kern k;
  if (prec == P_BF16) {
    k = Tk == 1 ? conv_fused_kernel<P_BF16, 1> : Tk == 2 ? conv_fused_kernel<P_BF16, 2> : conv_fused_kernel<P_BF16, 3>;
  } else if (k8) {
    k = conv_fused_kernel<P_FP8, 3, true>;
  } else {
    k = Tk == 1 ? conv_fused_kernel<P_FP8, 1> : Tk == 2 ? conv_fused_kernel<P_FP8, 2>
        : Tk == 4 ? conv_fused_kernel<P_FP8, 4> : conv_fused_kernel<P_FP8, 3>;
  }
  // one workgroup per resident slot (all CUs, at the kernel's occupancy);
  // each loops over the groups b, b + grid, ...  The slot count of a
  // (device, kernel) pair is queried once and cached.
  constexpr int kDevs = 64;
  static std::atomic<int> slot_cache[kDevs][3][6];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) dev = 0;
  std::atomic<int>* cached = dev < kDevs ? &slot_cache[dev][prec == P_BF16 ? 0 : k8 ? 2 : 1][Tk] : nullptr;
  int slots = cached ? cached->load(std::memory_order_relaxed) : 0;
  if (slots <= 0) {
    int ncu = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0) ncu = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k), kThreads, 0) !=
            hipSuccess || per_cu <= 0)
      per_cu = 1;
    slots = ncu * per_cu;
    if (cached) cached->store(slots, std::memory_order_relaxed);
  }
  FusedConvArgs a = args;
  a.n_groups = n_groups;
  const unsigned grid = (unsigned)(n_groups < slots ? n_groups : slots);
  hipLaunchKernelGGL(k, dim3(grid), dim3(kThreads), 0, s, a);
}

}  // namespace bcts
